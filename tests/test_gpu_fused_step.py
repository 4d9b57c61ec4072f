"""The plain fitting step's fused calls against the separate calls they
replace, bit for bit.  plane_render_step (forward, loss, backward and Adam
with one render launch) in several weight modes and with deep lists; and the
fused backward (plane_render_bwd_adam: the
backward, Adam of Sec. 3.3 and the loss sums of Eq. 14 in one call, the
sums formed by workgroups of the backward's reduction) against the separate
calls it replaces (plane_render_fwd_loss with its own loss sums,
plane_render_bwd, adam_step_planes): the same bits for the
planes, the Adam moments, the gradients and the loss, over several steps of a
two-job, two-camera batch.  Also checks that the binning counts, cleared by
plane_project, do not carry over between steps."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


@pytest.fixture(scope="module")
def batch():
    from paper_2412_03451_amd.splat import Job
    gt, info = synth.room_planes(seed=11, target_K=120)
    cams = synth.room_trajectory(11, 2, info, width=96, height=80, f=86.5)
    init = synth.room_init_planes(gt, seed=12)
    K = init.K
    jobs = [Job(0, K, 0, 96, 80, (16, 16)), Job(0, K, 1, 96, 80, (8, 8))]
    tD, tN = [], []
    for cm in cams:
        D, N, _ = oracle.render(gt.center, gt.quat, gt.radii, cm, 300.0, oracle.OracleParams())
        tD.append(D.numpy().astype(np.float32).ravel())
        tN.append(N.numpy().astype(np.float32).ravel())
    # targets laid out like the jobs: each job's depth, then its three normal planes
    return init, cams, jobs, _dev(np.concatenate(tD)), _dev(np.concatenate([n.reshape(3, -1).ravel() for n in tN]))


def _run(batch, fused, steps: int = 4, params=None):
    """fused: False (separate calls), True (plane_render_bwd_adam) or "step"
    (plane_render_step: forward, loss, backward and Adam in one launch)."""
    from paper_2412_03451_amd.splat import Renderer, adam_step
    init, cams, jobs, tD, tN = batch
    r = Renderer(jobs, cams, params=params)
    c, q, rr = _dev(init.center), _dev(init.quat), _dev(init.radii)
    K = c.shape[0]
    m = torch.zeros(11 * K, device="cuda")
    v = torch.zeros(11 * K, device="cuda")
    out = []
    for it in range(steps):
        lam = torch.tensor([float(np.float32(oracle.lambda_at(200 * it)))], device="cuda")
        step = torch.tensor([it + 1], dtype=torch.int32, device="cuda")
        r.project(c, q, rr, lam)
        r.bin()
        if fused == "step":
            loss = torch.empty(len(jobs), 4, device="cuda")
            D, N, gD, gN, gc, gq, gr = r.step(tD, tN, m, v, step, loss=loss)
            torch.cuda.synchronize()
            out.append([x.detach().cpu().numpy().copy() for x in (loss, gc, gq, gr, c, q, rr, m, v, D, N, gD, gN)])
            continue
        D, N, loss, gD, gN = r.forward_loss(tD, tN, reduce=not fused)
        if fused:
            loss = torch.empty(len(jobs), 4, device="cuda")
            gc, gq, gr = r.backward_adam(c, q, rr, lam, gD, gN, m, v, step, loss=loss)
        else:
            gc, gq, gr = r.backward(c, q, rr, lam, gD, gN)
            adam_step(c, q, rr, gc, gq, gr, m, v, step)
        torch.cuda.synchronize()
        out.append([x.detach().cpu().numpy().copy() for x in (loss, gc, gq, gr, c, q, rr, m, v, D, N, gD, gN)])
    return out


def test_fused_backward_adam_gives_the_separate_calls_bits(batch):
    a = _run(batch, fused=False)
    b = _run(batch, fused=True)
    names = ("loss", "g_center", "g_quat", "g_radii", "center", "quat", "radii", "m", "v", "depth", "normal",
             "g_depth", "g_normal")
    for it, (sa, sb) in enumerate(zip(a, b)):
        print(f"step {it}: loss {sa[0].sum(0)}", flush=True)
        for n, x, y in zip(names, sa, sb):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (it, n)
    # the fit actually moved and the gradients are not trivial
    assert np.abs(a[-1][4] - batch[0].center).max() > 0
    assert np.abs(a[0][1]).max() > 0


@pytest.mark.parametrize("mode,flags", [(0, 0), (2, 0), (1, 1), (0, 2 << 4), (0, 1 << 10)])
def test_one_launch_step_gives_the_separate_calls_bits(batch, mode, flags):
    """plane_render_step (each 8x8 block's forward, loss and backward in one
    launch, the hits committed again from the walk's recorded positions)
    against plane_render_fwd_loss + plane_render_bwd + adam_step_planes:
    the same bits for everything, in the default weight mode, the Gaussian
    (Eq. 5), mode 1 with the exact fallback forced for every pixel, with an
    8-hit pending buffer, and with the wave-per-plane reduction (flags bit
    10), after which the Adam update is a launch of its own rather than part
    of the reduction."""
    from paper_2412_03451_amd.splat import SplatParams
    prm = SplatParams(weight_mode=mode, flags=flags)
    a = _run(batch, fused=False, params=prm)
    b = _run(batch, fused="step", params=prm)
    names = ("loss", "g_center", "g_quat", "g_radii", "center", "quat", "radii", "m", "v", "depth", "normal",
             "g_depth", "g_normal")
    for it, (sa, sb) in enumerate(zip(a, b)):
        for n, x, y in zip(names, sa, sb):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (mode, flags, it, n)
    assert np.abs(a[0][1]).max() > 0


def test_one_launch_step_deep_lists():
    """Deep per-pixel lists (more than one 8-hit chunk per pixel, several
    staged batches per tile): the one-launch step's gradients are the
    separate calls' bits."""
    from paper_2412_03451_amd.splat import Renderer, SplatParams, adam_step
    ps = synth.random_planes(150, seed=4, center_range=0.3, extent_range=(0.4, 0.9))
    cam = synth.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    _, _, aux = oracle.render(ps.center, ps.quat, ps.radii, cam, 8.0, oracle.OracleParams(weight_mode="B"))
    assert int(aux["count"].max()) > 16   # three chunks of 8 hits for some pixels
    tgt = synth.random_planes(150, seed=5, center_range=0.3, extent_range=(0.4, 0.9))
    tD, tN, _ = oracle.render(tgt.center, tgt.quat, tgt.radii, cam, 300.0, oracle.OracleParams(weight_mode="B"))
    tD = _dev(tD.numpy().astype(np.float32).ravel())
    tN = _dev(tN.numpy().astype(np.float32).reshape(3, -1).ravel())
    outs = []
    for form in ("separate", "step"):
        r = Renderer.single_scene([cam], ps.K, params=SplatParams(weight_mode=1))
        c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
        m = torch.zeros(11 * ps.K, device="cuda")
        v = torch.zeros(11 * ps.K, device="cuda")
        step = torch.tensor([1], dtype=torch.int32, device="cuda")
        lam = torch.tensor([8.0], device="cuda")
        r.project(c, q, rr, lam)
        r.bin()
        if form == "step":
            loss = torch.empty(1, 4, device="cuda")
            D, N, gD, gN, gc, gq, gr = r.step(tD, tN, m, v, step, loss=loss)
        else:
            D, N, loss, gD, gN = r.forward_loss(tD, tN)
            gc, gq, gr = r.backward(c, q, rr, lam, gD, gN)
            adam_step(c, q, rr, gc, gq, gr, m, v, step)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy().copy() for x in (loss, gc, gq, gr, c, q, rr, D, N)])
    for x, y in zip(*outs):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert np.abs(outs[0][1]).max() > 0


def test_one_launch_step_without_maps(batch):
    """plane_render_step with null map and loss-gradient outputs (what the
    fitting loop passes): the same loss, gradients, planes and moments."""
    from paper_2412_03451_amd.splat import Renderer
    init, cams, jobs, tD, tN = batch
    outs = []
    for maps in (True, False):
        r = Renderer(jobs, cams)
        c, q, rr = _dev(init.center), _dev(init.quat), _dev(init.radii)
        m = torch.zeros(11 * c.shape[0], device="cuda")
        v = torch.zeros(11 * c.shape[0], device="cuda")
        step = torch.tensor([1], dtype=torch.int32, device="cuda")
        loss = torch.empty(len(jobs), 4, device="cuda")
        r.project(c, q, rr, torch.tensor([float(np.float32(oracle.lambda_at(0)))], device="cuda"))
        r.bin()
        D, N, gD, gN, gc, gq, gr = r.step(tD, tN, m, v, step, loss=loss, maps=maps)
        assert (D is None) == (not maps)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy().copy() for x in (loss, gc, gq, gr, c, q, rr, m, v)])
    for x, y in zip(*outs):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


@pytest.mark.parametrize("kp", [1, 5, 8, 13])
def test_one_launch_step_bits_for_few_planes(batch, kp):
    """With a workgroup per plane the reduction deals the planes to its
    workgroups in contiguous runs per XCD (workgroups equal mod 8 take one
    run), the last K mod 8 planes in order; below 8 planes every plane is
    in that tail.  Every plane is still reduced and updated once, with the
    separate calls' bits (plane counts 1, 5, 8 and 13 of the room's planes,
    both jobs kept)."""
    from types import SimpleNamespace
    from paper_2412_03451_amd.splat import Job
    init, cams, jobs, tD, tN = batch
    sub = SimpleNamespace(center=init.center[:kp], quat=init.quat[:kp], radii=init.radii[:kp], K=kp)
    jobs_k = [Job(0, kp, j.cam, j.width, j.height, j.tile) for j in jobs]
    b = (sub, cams, jobs_k, tD, tN)
    x = _run(b, fused=False, steps=2)
    y = _run(b, fused="step", steps=2)
    names = ("loss", "g_center", "g_quat", "g_radii", "center", "quat", "radii", "m", "v", "depth", "normal",
             "g_depth", "g_normal")
    for it, (sa, sb) in enumerate(zip(x, y)):
        for n, p, q in zip(names, sa, sb):
            assert np.array_equal(p.view(np.uint32), q.view(np.uint32)), (kp, it, n)
