"""GPU parity of loss_depth_normal, plane_render_bwd and adam_step_planes
against the float64 oracle (run on an MI355X).

Gradient bar per coordinate: |g - g_ref| <= 1e-4 |g_ref| + 32 u32 S
+ 1e-4 u32 max|g_ref|, where S is the oracle's sum over pixels of
|contribution| to that coordinate (float32 sums over thousands of pixels that
cancel cannot be closer than a few roundoffs of S) and the last term only
matters for coordinates far below one float32 roundoff of the group's largest
gradient; plus a cosine >= 1 - 1e-8 per parameter group.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import cosine, f32, grad_check

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _upstream(ps, tgt, cam, lam, prm):
    """Loss gradient of the oracle's render against the oracle's target render,
    rounded to float32 (the GPU receives the same values)."""
    D, N, _ = oracle.render(ps.center, ps.quat, ps.radii, cam, lam, prm)
    Dt, Nt, _ = oracle.render(tgt.center, tgt.quat, tgt.radii, cam, 300.0, prm)
    Dv = D.clone().requires_grad_(True)
    Nv = N.clone().requires_grad_(True)
    oracle.render_loss(Dv, Nv, Dt, Nt).backward()
    return Dv.grad.numpy().astype(np.float32), Nv.grad.numpy().astype(np.float32)


def _check_grads(gpu, ref, abss, label, c=32.0, conds=None):
    for i, (name, g, gr, s) in enumerate(zip(("center", "quat", "radii"), gpu, ref, abss)):
        g = g.detach().cpu().numpy()
        err, tol = grad_check(g, gr.numpy(), s.numpy(), c=c, cond=None if conds is None else conds[i].numpy())
        cs = cosine(g, gr.numpy())
        ratio = err / np.maximum(tol, 1e-300)
        w = np.unravel_index(np.argmax(ratio), ratio.shape)
        print(f"{label} {name}: max err/tol {ratio.max():.3g} at {w} (err {err[w]:.3g} tol {tol[w]:.3g} "
              f"ref {gr.numpy()[w]:.4g} gpu {g[w]:.4g} abssum {s.numpy()[w]:.3g}), cosine-1 {cs - 1:.3g}, "
              f"|g|max {np.abs(gr.numpy()).max():.3g}", flush=True)
        assert np.all(err <= tol), (name, np.unravel_index(np.argmax(ratio), ratio.shape))
        assert cs >= 1 - 1e-8


@pytest.mark.parametrize("mode,lam", [(0, oracle.lambda_at(0)), (0, 60.0), (0, 300.0), (1, 20.0), (2, 10.0)])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_backward_tiny_scene(mode, lam, tile):
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    ps = synth.random_planes(64, seed=0, independent_radii=True)
    tgt = synth.perturb_planes(ps, seed=1, center_sigma=0.05, rot_sigma_deg=5.0)
    cam = synth.tiny_camera()
    prm = oracle.OracleParams(weight_mode="ABG"[mode])
    gD, gN = _upstream(ps, tgt, cam, f32(lam), prm)
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, f32(lam), gD, gN, prm)
    r = Renderer.single_scene([cam], ps.K, tile=tile, params=SplatParams(weight_mode=mode))
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], device="cuda")
    r.render(c, q, rr, lt)
    out = r.backward(c, q, rr, lt, _dev(gD).reshape(-1), _dev(gN).reshape(-1))
    torch.cuda.synchronize()
    _check_grads(out, grads, abss, f"mode {mode} lam {lam:.3g} tile {tile}")
    # bitwise deterministic
    out2 = r.backward(c, q, rr, lt, _dev(gD).reshape(-1), _dev(gN).reshape(-1))
    for a, b in zip(out, out2):
        assert torch.equal(a, b)


def test_backward_fallback_path_is_identical():
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    ps = synth.random_planes(64, seed=3, independent_radii=True)
    cam = synth.tiny_camera()
    rng = np.random.default_rng(0)
    gD = rng.normal(size=cam.width * cam.height).astype(np.float32)
    gN = rng.normal(size=3 * cam.width * cam.height).astype(np.float32)
    outs = []
    for flags in (0, 1):
        r = Renderer.single_scene([cam], ps.K, params=SplatParams(flags=flags))
        c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
        lt = torch.tensor([25.0], device="cuda")
        r.render(c, q, rr, lt)
        outs.append(r.backward(c, q, rr, lt, _dev(gD), _dev(gN)))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_backward_deep_lists_multi_pass():
    """Dense semi-transparent overlap (mode B, small lambda) gives per-pixel
    lists longer than one LDS chunk, exercising the recompute passes."""
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    ps = synth.random_planes(80, seed=4, center_range=0.3, extent_range=(0.4, 0.9))
    cam = synth.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    lam = 8.0
    prm = oracle.OracleParams(weight_mode="B")
    _, _, aux = oracle.render(ps.center, ps.quat, ps.radii, cam, lam, prm)
    assert int(aux["count"].max()) > 12
    rng = np.random.default_rng(1)
    gD = rng.normal(size=cam.width * cam.height).astype(np.float32)
    gN = rng.normal(size=(3, cam.width * cam.height)).astype(np.float32)
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, lam, gD, gN, prm)
    r = Renderer.single_scene([cam], ps.K, params=SplatParams(weight_mode=1))
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], device="cuda")
    r.render(c, q, rr, lt)
    out = r.backward(c, q, rr, lt, _dev(gD).reshape(-1), _dev(gN).reshape(-1))
    torch.cuda.synchronize()
    _check_grads(out, grads, abss, "deep lists")


def test_backward_multi_view_sums_over_views():
    from paper_2412_03451_amd.splat import Job, Renderer
    ps = synth.random_planes(48, seed=5, independent_radii=True)
    cams = [synth.tiny_camera(),
            synth.Camera(80, 60, 70.0, 70.0, 41.0, 29.0, np.eye(3, dtype=np.float32),
                         np.array([0.3, -0.1, 3.2], np.float32))]
    lam = 40.0
    rng = np.random.default_rng(2)
    gDs = [rng.normal(size=c.width * c.height).astype(np.float32) for c in cams]
    gNs = [rng.normal(size=(3, c.width * c.height)).astype(np.float32) for c in cams]
    tot = None
    for cam, gD, gN in zip(cams, gDs, gNs):
        g, s = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, lam, gD, gN)
        tot = (g, s) if tot is None else ([a + b for a, b in zip(tot[0], g)], [a + b for a, b in zip(tot[1], s)])
    jobs = [Job(0, ps.K, i, c.width, c.height, (16, 16)) for i, c in enumerate(cams)]
    r = Renderer(jobs, cams)
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], device="cuda")
    r.render(c, q, rr, lt)
    gD = torch.cat([_dev(x) for x in gDs])
    gN = torch.cat([_dev(x).reshape(-1) for x in gNs])
    out = r.backward(c, q, rr, lt, gD, gN)
    torch.cuda.synchronize()
    _check_grads(out, tot[0], tot[1], "two views")


def test_reduction_shape_does_not_change_bits():
    """The per-plane reduction of the partial rows takes a workgroup per plane
    for few planes and a wave per plane for many (flags bit 10 forces the
    latter): the same summation order, so the same bits.  Two views (two
    records per plane) and 8x8 tiles on a 320x240 image, so large planes have
    more than 256 rows."""
    from paper_2412_03451_amd.splat import Job, Renderer, SplatParams
    ps = synth.random_planes(60, seed=9, center_range=0.3, extent_range=(0.4, 0.9), independent_radii=True)
    cams = [synth.Camera(320, 240, 300.0, 300.0, 160.0, 120.0, np.eye(3, dtype=np.float32),
                         np.array([0.0, 0.0, 3.0], np.float32)),
            synth.Camera(320, 240, 280.0, 280.0, 161.0, 119.0, np.eye(3, dtype=np.float32),
                         np.array([0.2, -0.1, 3.3], np.float32))]
    rng = np.random.default_rng(3)
    n = sum(c.width * c.height for c in cams)
    gD = _dev(rng.normal(size=n).astype(np.float32))
    gN = _dev(rng.normal(size=3 * n).astype(np.float32))
    outs = []
    for flags in (0, 1 << 10):
        jobs = [Job(0, ps.K, i, c.width, c.height, (8, 8)) for i, c in enumerate(cams)]
        r = Renderer(jobs, cams, params=SplatParams(flags=flags))
        c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
        lt = torch.tensor([20.0], device="cuda")
        r.render(c, q, rr, lt)
        outs.append([x.clone() for x in r.backward(c, q, rr, lt, gD, gN)])
        rows = r.region(3, torch.int32, r.L.n_records).max().item()   # 8x8 tiles: rows = tiles of a record
    assert rows > 256
    for a, b in zip(*outs):
        assert torch.equal(a, b)
        assert float(a.abs().max()) > 0


def test_loss_matches_oracle():
    from paper_2412_03451_amd.splat import Renderer
    cam = synth.tiny_camera(100, 70, 90.0)
    r = Renderer.single_scene([cam], 1)
    rng = np.random.default_rng(3)
    P = cam.width * cam.height
    Dt = rng.uniform(0.5, 4, size=P).astype(np.float32)
    Nt = rng.normal(size=(3, P))
    Nt = (Nt / np.linalg.norm(Nt, axis=0)).astype(np.float32)
    D = (Dt + rng.normal(scale=0.1, size=P)).astype(np.float32)
    N = (Nt + rng.normal(scale=0.2, size=(3, P))).astype(np.float32)
    D[:500] = Dt[:500]          # exact matches: sgn(0) = 0
    N[:, :300] = Nt[:, :300]
    D[600:700] = 0.0             # background pixels
    N[:, 600:700] = 0.0
    mask = (rng.uniform(size=P) > 0.2).astype(np.uint8)
    for m in (None, mask):
        loss, gD, gN = r.loss(_dev(D), _dev(N).reshape(-1), _dev(Dt), _dev(Nt).reshape(-1),
                              mask=None if m is None else torch.as_tensor(m, device="cuda"))
        torch.cuda.synchronize()
        Dv = torch.tensor(D, dtype=torch.float64, requires_grad=True)
        Nv = torch.tensor(N, dtype=torch.float64, requires_grad=True)
        terms = oracle.loss_terms(Dv.reshape(cam.height, cam.width), Nv.reshape(3, cam.height, cam.width),
                                  Dt.reshape(cam.height, cam.width), Nt.reshape(3, cam.height, cam.width),
                                  mask=None if m is None else m.reshape(cam.height, cam.width))
        sum(terms).backward()
        lg = loss.cpu().numpy()[0]
        for i in range(3):
            assert lg[i] == pytest.approx(float(terms[i]), rel=1e-6)
        np.testing.assert_array_equal(gD.cpu().numpy(), Dv.grad.numpy().astype(np.float32))
        np.testing.assert_allclose(gN.cpu().numpy(), Nv.grad.numpy().reshape(-1), rtol=1e-6, atol=1e-6)


def test_adam_matches_oracle():
    from paper_2412_03451_amd.splat import adam_step
    rng = np.random.default_rng(4)
    K = 1000
    params = [rng.normal(size=(K, 3)), rng.normal(size=(K, 4)), rng.uniform(1e-4, 0.5, size=(K, 4))]
    params[2][:5] = 1e-4 + 1e-7  # will hit the clamp
    dev = [_dev(p) for p in params]
    ref = [p.astype(np.float32).astype(np.float64) for p in params]
    m = torch.zeros(11 * K, device="cuda")
    v = torch.zeros(11 * K, device="cuda")
    mr = [np.zeros(p.shape) for p in params]
    vr = [np.zeros(p.shape) for p in params]
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for it in range(1, 4):
        grads = [rng.normal(size=p.shape) * 10 ** rng.uniform(-3, 2, size=p.shape) for p in params]
        grads[2][:5] = 1.0
        g32 = [g.astype(np.float32) for g in grads]
        step.fill_(it)
        adam_step(*dev, *[_dev(g) for g in g32], m, v, step)
        for i in range(3):
            ref[i], mr[i], vr[i] = oracle.adam_step(ref[i], g32[i].astype(np.float64), mr[i], vr[i], it,
                                                    clamp_min=1e-4 if i == 2 else None)
        torch.cuda.synchronize()
        for i in range(3):
            got = dev[i].cpu().numpy()
            # each step moves a parameter by at most ~lr; float32 rounding of the parameter dominates
            assert np.all(np.abs(got - ref[i]) <= 2e-6 * (1 + np.abs(ref[i]))), (it, i)
    assert np.all(dev[2].cpu().numpy()[:5] == np.float32(1e-4))


def test_full_step_tiny_config():
    """Tiny config: one forward, one loss + backward, one Adam step at ite 0,
    against the oracle chain."""
    from paper_2412_03451_amd.splat import Renderer, adam_step
    ps = synth.random_planes(64, seed=0)
    tgt = synth.perturb_planes(ps, seed=1, center_sigma=0.05, rot_sigma_deg=5.0)
    cam = synth.tiny_camera()
    lam = oracle.lambda_at(0)
    Dt, Nt, _ = oracle.render(tgt.center, tgt.quat, tgt.radii, cam, 300.0)
    r = Renderer.single_scene([cam], ps.K)
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], device="cuda")
    D, N = r.render(c, q, rr, lt)
    loss, gD, gN = r.loss(D, N, _dev(Dt.numpy()).reshape(-1), _dev(Nt.numpy()).reshape(-1))
    gc, gq, gr = r.backward(c, q, rr, lt, gD, gN)
    m = torch.zeros(11 * ps.K, device="cuda")
    v = torch.zeros(11 * ps.K, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    adam_step(c, q, rr, gc, gq, gr, m, v, step)
    torch.cuda.synchronize()
    # oracle chain
    cc, qq, rq = (torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in (ps.center, ps.quat, ps.radii))
    Do, No, _ = oracle.render_pixels(cc, qq, rq, cam, f32(lam), torch.arange(cam.width * cam.height))
    Lo = oracle.render_loss(Do.reshape(cam.height, cam.width), No.T.reshape(3, cam.height, cam.width), Dt, Nt)
    Lo.backward()
    lg = loss.cpu().numpy()[0]
    assert float(lg[:3].sum()) == pytest.approx(float(Lo), rel=1e-5)
    assert cosine(gc.cpu().numpy(), cc.grad.numpy()) > 1 - 1e-6
    for got, p0, g in ((c, ps.center, cc.grad), (q, ps.quat, qq.grad), (rr, ps.radii, rq.grad)):
        ref, _, _ = oracle.adam_step(p0.astype(np.float64), g.numpy(), np.zeros(p0.shape), np.zeros(p0.shape), 1)
        if got is rr:
            ref = np.maximum(ref, 1e-4)
        delta_ref = ref - p0
        delta = got.cpu().numpy().astype(np.float64) - p0
        # first step moves each coordinate by lr * sign(g) unless g vanishes
        big = np.abs(g.numpy()) > 1e-3
        np.testing.assert_allclose(delta[big], delta_ref[big], rtol=1e-3, atol=2e-7)


def test_room_backward_sampled_pixels():
    """Full-size room view (640x480, ~2000 planes, the benchmark's shape):
    upstream gradients on 300 sampled pixels, zero elsewhere, so the oracle
    differentiates those pixels only; at the first iteration's lambda and at 300.

    Bound per coordinate: the small scenes' 1e-4 |g_ref| + 32 u32 S, plus 64
    float32 roundoffs of the weight path's cancellation-free magnitude
    (oracle.weight_path_magnitude): in pixels with many hits at the first
    iteration's wide fringes, dL/dw_j = T_j (c_j - S_{j+1}) cancels (c_j,
    formed from the float32 depth and normal, is close to the composite
    S_{j+1} of what lies behind), which the sum of |contribution| over pixels
    cannot see; without that term one contribution was 9e-5 off in relative
    terms with the same hit list as the oracle's."""
    from paper_2412_03451_amd.splat import Renderer
    gt, info = synth.room_planes(seed=0, target_K=2000)
    init = synth.room_init_planes(gt, seed=1)
    cams = synth.room_trajectory(seed=0, n_views=1, info=info)
    cam = cams[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(17)
    for lam in (oracle.lambda_at(0), 300.0):
        print(f"room backward lambda {lam:.4g}", flush=True)
        r = Renderer.single_scene(cams, init.K, tile=(16, 16))
        lt = torch.tensor([lam], device="cuda")
        c, q, rr = _dev(init.center), _dev(init.quat), _dev(init.radii)
        r.project(c, q, rr, lt)
        r.bin()
        r.forward()
        pix = rng.choice(P, size=300, replace=False)
        gD = np.zeros(P, np.float32)
        gN = np.zeros((3, P), np.float32)
        gD[pix] = rng.normal(size=300).astype(np.float32)
        gN[:, pix] = rng.normal(size=(3, 300)).astype(np.float32)
        gpu = r.backward(c, q, rr, lt, _dev(gD), _dev(gN.reshape(-1)))
        torch.cuda.synchronize()
        grads, abss = oracle.per_pixel_abs_grad(init.center, init.quat, init.radii, cam, f32(lam), gD, gN,
                                                chunk=25, pix=pix)
        conds = oracle.weight_path_magnitude(init.center, init.quat, init.radii, cam, f32(lam), gD, gN,
                                             chunk=25, pix=pix)
        _check_grads(gpu, grads, abss, f"room lambda {lam:.4g}", conds=conds)


@pytest.mark.parametrize("mode", [0, 2])
def test_pending_buffer_size_does_not_change_results(mode):
    """The pending-hit buffer size (4, 6, 8 or 12 per lane) is a tuning knob:
    forward maps and gradients are bitwise identical for every size and for
    the exact fallback ordering forced on every pixel (the path a lane takes
    when its buffer overflows)."""
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    ps = synth.random_planes(160, seed=12, independent_radii=True, center_range=0.4, extent_range=(0.2, 0.7))
    cam = synth.tiny_camera()
    rng = np.random.default_rng(4)
    gD = _dev(rng.normal(size=cam.width * cam.height))
    gN = _dev(rng.normal(size=3 * cam.width * cam.height))
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([12.0], device="cuda")
    outs = {}
    for P, flags in ((6, 0), (4, 1 << 4), (8, 2 << 4), (12, 3 << 4), ("all-fallback", 1)):
        print(f"pending {P} mode {mode}", flush=True)
        r = Renderer.single_scene([cam], ps.K, params=SplatParams(weight_mode=mode, flags=flags))
        D, N = r.render(c, q, rr, lt)
        slow = r.counters()["slow_pixels"]
        g = r.backward(c, q, rr, lt, gD, gN)
        torch.cuda.synchronize()
        outs[P] = (D.clone(), N.clone(), [x.clone() for x in g], slow)
    print({P: o[3] for P, o in outs.items()}, flush=True)
    assert outs["all-fallback"][3] == cam.width * cam.height
    # a buffer of 4 overflows on some pixels, not all: the mixed walk + fallback path is exercised
    assert 0 < outs[4][3] < cam.width * cam.height
    for P in (4, 8, 12, "all-fallback"):
        assert torch.equal(outs[P][0], outs[6][0]) and torch.equal(outs[P][1], outs[6][1])
        for a, b in zip(outs[P][2], outs[6][2]):
            assert torch.equal(a, b)
