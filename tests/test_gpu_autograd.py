"""The torch.autograd front end (recompute in backward): gradients of any
scalar of the rendered maps match the float64 oracle's; a render in between
forward and backward on the same workspace does not change them; the
per-camera-target loss variant matches the plain loss."""

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import cosine, f32, grad_check

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def test_autograd_matches_oracle_and_survives_reuse():
    from paper_2412_03451_amd.autograd import plane_splat
    from paper_2412_03451_amd.splat import Renderer
    ps = synth.random_planes(64, seed=7, independent_radii=True)
    other = synth.perturb_planes(ps, seed=8, center_sigma=0.2, rot_sigma_deg=20.0)
    cam = synth.tiny_camera()
    lam = f32(30.0)
    rng = np.random.default_rng(5)
    P = cam.width * cam.height
    wD = rng.normal(size=P).astype(np.float32)
    wN = rng.normal(size=(3, P)).astype(np.float32)
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, lam, wD, wN)

    r = Renderer.single_scene([cam], ps.K)
    res = []
    for reuse in (False, True):
        c, q, rr = (_dev(x).requires_grad_(True) for x in (ps.center, ps.quat, ps.radii))
        D, N = plane_splat(c, q, rr, lam, r)
        if reuse:   # another render overwrites the workspace before the backward
            r.render(_dev(other.center), _dev(other.quat), _dev(other.radii), torch.tensor([lam], device="cuda"))
        L = (D * _dev(wD)).sum() + (N * _dev(wN).reshape(-1)).sum()
        L.backward()
        torch.cuda.synchronize()
        res.append((c.grad.clone(), q.grad.clone(), rr.grad.clone()))
    for name, g, gr, s in zip(("center", "quat", "radii"), res[0], grads, abss):
        g = g.cpu().numpy()
        err, tol = grad_check(g, gr.numpy(), s.numpy())
        assert np.all(err <= tol), name
        assert cosine(g, gr.numpy()) >= 1 - 1e-8
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_loss_cam_matches_loss():
    from paper_2412_03451_amd.splat import Job, Renderer
    cams = [synth.tiny_camera(), synth.tiny_camera()]
    r = Renderer([Job(0, 1, 1, 128, 96), Job(0, 1, 0, 128, 96)], cams)
    rng = np.random.default_rng(6)
    P = 128 * 96
    tD = rng.uniform(0.5, 4, size=(2, P)).astype(np.float32)
    tN = rng.normal(size=(2, 3, P)).astype(np.float32)
    D = rng.uniform(0.5, 4, size=2 * P).astype(np.float32)
    N = rng.normal(size=2 * 3 * P).astype(np.float32)
    # job 0 uses camera 1, job 1 camera 0: the plain loss sees the targets in job order
    l1, gD1, gN1 = r.loss(_dev(D), _dev(N), _dev(tD[[1, 0]].reshape(-1)), _dev(tN[[1, 0]].reshape(-1)))
    off = torch.tensor([0, P], dtype=torch.int64, device="cuda")
    l2, gD2, gN2 = r.loss_cam(_dev(D), _dev(N), _dev(tD.reshape(-1)), _dev(tN.reshape(-1)), off)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2) and torch.equal(gD1, gD2) and torch.equal(gN1, gN2)


@pytest.mark.parametrize("mode,lam", [(0, 30.0), (1, 8.0)])
def test_list_storing_variant_gives_the_same_bits(mode, lam):
    """Forward lists and list-reading backward equal the recompute path
    (including lists longer than one recompute chunk in mode B)."""
    from paper_2412_03451_amd.autograd import PlaneSplatFn, PlaneSplatListsFn
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    if mode == 1:
        ps = synth.random_planes(80, seed=4, center_range=0.3, extent_range=(0.4, 0.9))
        cam = synth.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3, dtype=np.float32),
                           np.array([0.0, 0.0, 3.0], np.float32))
    else:
        ps = synth.random_planes(64, seed=7, independent_radii=True)
        cam = synth.tiny_camera()
    rng = np.random.default_rng(9)
    P = cam.width * cam.height
    wD = _dev(rng.normal(size=P))
    wN = _dev(rng.normal(size=3 * P))
    lt = torch.tensor([f32(lam)], device="cuda")
    res = []
    for fn in (PlaneSplatFn, PlaneSplatListsFn):
        r = Renderer.single_scene([cam], ps.K, params=SplatParams(weight_mode=mode))
        c, q, rr = (_dev(x).requires_grad_(True) for x in (ps.center, ps.quat, ps.radii))
        D, N = fn.apply(c, q, rr, lt, r)
        ((D * wD).sum() + (N * wN).sum()).backward()
        torch.cuda.synchronize()
        res.append((D.detach().clone(), N.detach().clone(), c.grad.clone(), q.grad.clone(), rr.grad.clone()))
    for x, y in zip(*res):
        assert torch.equal(x, y)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_forward_loss_matches_forward_then_loss(tile):
    """plane_render_fwd_loss gives the bits of plane_render_fwd followed by
    the loss call: three jobs of two sizes (one ragged against the tiles),
    per-camera targets with a mask, and the job-ordered targets."""
    from paper_2412_03451_amd.splat import Job, Renderer
    ps = synth.random_planes(90, seed=31, independent_radii=True)
    c0 = synth.tiny_camera()
    c1 = synth.scaled_camera(synth.tiny_camera(), 100, 70, 80.0)
    cams = [c0, c1, c0]
    jobs = [Job(0, 90, 0, 128, 96, tile), Job(0, 60, 1, 100, 70, tile), Job(30, 90, 2, 128, 96, tile)]
    r = Renderer(jobs, cams)
    lam = torch.tensor([9.0], device="cuda")
    r.project(_dev(ps.center), _dev(ps.quat), _dev(ps.radii), lam)
    r.bin()
    rng = np.random.default_rng(7)
    sizes = [128 * 96, 100 * 70, 128 * 96]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    P = int(offs[-1])
    tD = _dev(rng.uniform(0.5, 4, size=P).astype(np.float32))
    tN = _dev(rng.normal(size=3 * P).astype(np.float32))
    mask = torch.as_tensor(rng.uniform(size=P) < 0.8, dtype=torch.uint8, device="cuda")
    D0, N0 = r.forward()
    off = torch.as_tensor(offs[:-1], dtype=torch.int64, device="cuda")
    for kwargs in ({}, {"tgt_off": off, "mask": mask}):
        if "tgt_off" in kwargs:
            l0, gD0, gN0 = r.loss_cam(D0, N0, tD, tN, kwargs["tgt_off"], mask=kwargs["mask"])
        else:
            l0, gD0, gN0 = r.loss(D0, N0, tD, tN)
        D1, N1, l1, gD1, gN1 = r.forward_loss(tD, tN, **kwargs)
        torch.cuda.synchronize()
        print(f"tile {tile} {sorted(kwargs)}: loss {l1.cpu().numpy().round(3).tolist()}", flush=True)
        assert torch.equal(D0, D1) and torch.equal(N0, N1)
        assert torch.equal(gD0, gD1) and torch.equal(gN0, gN1)
        assert torch.equal(l0, l1)
