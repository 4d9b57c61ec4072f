"""Parity at the benchmark's shape and through the fitting loop (run on an MI355X).

* Whole 640x480 room views (K ~ 2000, the benchmark's workload): every pixel
  of the forward against the oracle, at the first iteration's lambda and at
  300, under both readings of the per-ray order (float32 and exact float64
  depth), Sec. 3.2, Eq. 4-13.
* The backward on a stratified pixel sample of a room view that holds every
  pixel the forward sent down the exact fallback ordering path, fringe pixels
  (semi-transparent hits only) and deep pixels (20 or more hits).
* The differentiation check: GPU gradients of 256 rectangles in a 256x192
  view against float64 central differences (h = 1e-6) of the oracle on 1000
  seeded coordinates, and against the oracle's autograd gradient, at
  lambda(0) and 300 (the adjoint of Eq. 4-13).
* Five graph-replayed fitting iterations (Eq. 10 lambda, the view schedule,
  Adam with bias correction), each step checked against the oracle's step
  from the same state.
"""

import os
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import U32, cosine, depth_err, f32, grad_check, normal_err

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LAM0 = f32(oracle.lambda_at(0))


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


@pytest.fixture(scope="module")
def room():
    gt, info = synth.room_planes(seed=0, target_K=2000)
    init = synth.room_init_planes(gt, seed=1)
    cams = synth.room_trajectory(seed=0, n_views=2, info=info)
    return gt, init, cams


# ----------------------------------------------------------------- forward, whole views
@pytest.mark.parametrize("lam", [LAM0, 300.0])
def test_room_whole_views_every_pixel(room, lam):
    from paper_2412_03451_amd.splat import Renderer
    gt, init, cams = room
    cases = [("init", init, s) for s in range(2)]
    if lam == 300.0:
        cases.append(("ground truth", gt, 0))   # many float32 depth ties between coplanar cells
    for name, ps, s in cases:
        cam = cams[s]
        print(f"whole view: {name} planes, view {s}, lambda {lam:.4g}", flush=True)
        r = Renderer.single_scene([cam], ps.K, tile=(16, 16))
        D, N, T, cnt = (x.cpu().numpy() for x in r.render_diag(_dev(ps.center), _dev(ps.quat), _dev(ps.radii),
                                                                torch.tensor([lam], device="cuda")))
        for order in ("f32", "f64"):
            Dr, Nr, aux = oracle.render_tiled(ps.center, ps.quat, ps.radii, cam, lam, oracle.OracleParams(order=order))
            ed = depth_err(D.reshape(cam.height, cam.width), Dr.numpy())
            en = normal_err(N.reshape(3, cam.height, cam.width), Nr.numpy())
            same_cnt = float(np.mean((cnt & 255).reshape(cam.height, cam.width) == aux["count"].numpy()))
            print(f"  order {order}: max depth err / bar {ed.max():.3g}, normal {en.max():.3g}, "
                  f"hit counts equal on {same_cnt:.5f} of pixels", flush=True)
            assert ed.max() <= 1.0 and en.max() <= 1.0


# ----------------------------------------------------------------- backward, stratified sample
def _stratified(cnt_gpu, aux, rng, n_each=120):
    """Every fallback-path pixel (at most cap), plus fringe, deep and random pixels."""
    fallback = np.flatnonzero(cnt_gpu >= 256)
    count = aux["count"].numpy().reshape(-1)
    T = aux["T"].numpy().reshape(-1)
    fringe = np.flatnonzero((count > 0) & (T > 0))
    deep = np.flatnonzero(count >= 20)
    pick = [fallback]
    for pool in (fringe, deep, np.arange(count.size)):
        if pool.size:
            pick.append(rng.choice(pool, size=min(n_each, pool.size), replace=False))
    return np.unique(np.concatenate(pick)), fallback.size, fringe.size, deep.size


@pytest.mark.parametrize("pending", [6, 4])
def test_room_backward_fallback_fringe_deep_pixels(room, pending):
    """Room view 0 at the first iteration's lambda (widest fringes, deepest
    lists).  With the default 6 pending hits every pixel that took the
    fallback path is in the sample; with 4 the fallback path is common and
    its pixels are sampled (at most 300).  Bound as for the sampled room
    backward: 1e-4 |g_ref| + 32 u32 S + 64 u32 C per coordinate."""
    from paper_2412_03451_amd.splat import Renderer, SplatParams
    gt, init, cams = room
    cam = cams[0]
    P = cam.width * cam.height
    flags = {6: 0, 4: 1 << 4}[pending]
    r = Renderer.single_scene([cam], init.K, tile=(16, 16), params=SplatParams(flags=flags))
    c, q, rr = _dev(init.center), _dev(init.quat), _dev(init.radii)
    lt = torch.tensor([LAM0], device="cuda")
    D, N, T, cnt = r.render_diag(c, q, rr, lt)
    cnt = cnt.cpu().numpy()
    slow = int(r.counters()["slow_pixels"])
    assert slow == int(np.sum(cnt >= 256))
    assert 0 < slow < P, slow
    _, _, aux = oracle.render_tiled(init.center, init.quat, init.radii, cam, LAM0)
    rng = np.random.default_rng(23)
    pix, n_fb, n_fr, n_dp = _stratified(cnt, aux, rng)
    if n_fb > 300:
        fb = np.flatnonzero(cnt >= 256)
        keep = np.setdiff1d(pix, fb)
        pix = np.unique(np.concatenate([keep, rng.choice(fb, size=300, replace=False)]))
    print(f"pending {pending}: {n_fb} fallback pixels, {n_fr} fringe, {n_dp} deep; sample of {pix.size}",
          flush=True)
    gD = np.zeros(P, np.float32)
    gN = np.zeros((3, P), np.float32)
    gD[pix] = rng.normal(size=pix.size).astype(np.float32)
    gN[:, pix] = rng.normal(size=(3, pix.size)).astype(np.float32)
    gpu = r.backward(c, q, rr, lt, _dev(gD), _dev(gN.reshape(-1)))
    torch.cuda.synchronize()
    grads, abss = oracle.per_pixel_abs_grad(init.center, init.quat, init.radii, cam, LAM0, gD, gN, chunk=25, pix=pix)
    conds = oracle.weight_path_magnitude(init.center, init.quat, init.radii, cam, LAM0, gD, gN, chunk=25, pix=pix)
    for i, name in enumerate(("center", "quat", "radii")):
        g = gpu[i].cpu().numpy()
        err, tol = grad_check(g, grads[i].numpy(), abss[i].numpy(), cond=conds[i].numpy())
        ratio = err / np.maximum(tol, 1e-300)
        print(f"  {name}: max err/tol {ratio.max():.3g}, cosine-1 {cosine(g, grads[i].numpy()) - 1:.3g}", flush=True)
        assert np.all(err <= tol)
        assert cosine(g, grads[i].numpy()) >= 1 - 1e-8


# ----------------------------------------------------------------- central differences
def _fd_module():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_fd_c3a
    return make_fd_c3a


@pytest.mark.parametrize("name", ["lam0", "lam300"])
def test_gradient_against_central_differences(name):
    """256 rectangles (independent radii) in one 256x192 view: the GPU
    gradient of sum gD D + gN . N against the stored float64 central
    differences (tests/golden/fd_c3a_*.txt, h = 1e-6, written from the
    oracle) on the 1000 seeded coordinates whose moves stay on one smooth
    piece, and against the oracle's autograd gradient on every coordinate.
    Bound against the differences: the GPU's bound against the exact
    gradient (1e-4 |g| + 32 u32 S + 64 u32 C + 1e-4 u32 max|g|) plus the
    differences' own (5e-5 of the per-pixel difference magnitude for the
    truncation, 4 rounding bounds, 1e-9)."""
    from paper_2412_03451_amd.splat import Renderer
    m = _fd_module()
    from test_oracle_fd_c3a import fd_bound, load_fd
    ps, cam, gD, gN = m.scene()
    lam = m.lambdas()[name]
    r = Renderer.single_scene([cam], ps.K, tile=(16, 16))
    c, q, rr = _dev(ps.center), _dev(ps.quat), _dev(ps.radii)
    lt = torch.tensor([lam], device="cuda")
    r.render(c, q, rr, lt)
    gpu = [x.cpu().numpy().astype(np.float64) for x in r.backward(c, q, rr, lt, _dev(gD), _dev(gN.reshape(-1)))]
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, lam, gD, gN, chunk=512)
    conds = oracle.weight_path_magnitude(ps.center, ps.quat, ps.radii, cam, lam, gD, gN, chunk=512)
    tols = []
    for i, gname in enumerate(("center", "quat", "radii")):
        err, tol = grad_check(gpu[i], grads[i].numpy(), abss[i].numpy(), cond=conds[i].numpy())
        print(f"{name} {gname} vs autograd: max err/tol {(err / tol).max():.3g}, "
              f"cosine-1 {cosine(gpu[i], grads[i].numpy()) - 1:.3g}", flush=True)
        assert np.all(err <= tol) and cosine(gpu[i], grads[i].numpy()) >= 1 - 1e-8
        tols.append(tol)
    coords, fd, fd_err, absd, cont = load_fd(name)
    g_at = np.array([gpu[w][k, cc] for (w, k, cc) in coords])
    tol_at = np.array([tols[w][k, cc] for (w, k, cc) in coords]) + fd_bound(absd, fd_err)
    dev = np.abs(g_at - fd)
    ratio = (dev / tol_at)[cont]
    rel = (dev / np.maximum(np.abs(fd), 1e-30))[cont]
    print(f"{name}: {int(cont.sum())} of {len(coords)} coordinates on one smooth piece; GPU vs central "
          f"differences max err/tol {ratio.max():.3g}, median relative error {np.median(rel):.3g}", flush=True)
    assert cont.sum() >= 900
    assert np.all(ratio <= 1.0)


# ----------------------------------------------------------------- the fitting loop
def _adam_ref(theta, g, m, v, step, lr=f32(1e-3), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8)):
    """The oracle's Adam with the constants the kernel receives: float32
    values of lr, beta1, beta2 and eps (inputs reach both sides rounded to
    float32, as cameras and lambda do)."""
    return oracle.adam_step(theta, g, m, v, step, lr=lr, b1=b1, b2=b2, eps=eps)


def _adam_spread(theta, g, e, m, v, step):
    """Largest move of the Adam update over gradients in [g - e, g + e]
    (nine points), the update's sensitivity to the gradient's error bound."""
    base, _, _ = _adam_ref(theta, g, m, v, step)
    worst = np.zeros_like(base)
    for f in np.linspace(-1.0, 1.0, 9):
        th, _, _ = _adam_ref(theta, g + f * e, m, v, step)
        worst = np.maximum(worst, np.abs(th - base))
    return worst


@pytest.mark.parametrize("n_views", [1, 3])
def test_five_graph_replayed_iterations_against_oracle_steps(n_views):
    """The small configuration (64 planes, 128x96; with n_views = 3 the same
    planes seen from three cameras, so the view schedule picks a camera per
    step).  Five iterations replayed from the captured graph; before each the
    state (planes, Adam moments, iteration counter) is read, and the oracle
    takes the same iteration from it: lambda of Eq. 10, the scheduled view,
    the render, the loss of Eq. 14 and its gradient (upstream gradients are
    the GPU's: the loss's sign decisions are checked bit for bit elsewhere),
    then Adam with bias correction and the radius clamp.  Per coordinate the
    GPU's new parameters must lie within the Adam update's spread over the
    gradient's error bound, plus float32 rounding."""
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    from paper_2412_03451_amd.splat import Renderer
    ps = synth.random_planes(64, seed=0)
    tgt = synth.perturb_planes(ps, seed=1, center_sigma=0.05, rot_sigma_deg=5.0)
    cams = [synth.tiny_camera()]
    if n_views == 3:
        for ang in (8.0, -8.0):
            a = np.deg2rad(ang)
            R = np.array([[np.cos(a), 0, -np.sin(a)], [0, 1, 0], [np.sin(a), 0, np.cos(a)]], np.float32)
            cams.append(synth.Camera(128, 96, 100.0, 100.0, 64.0, 48.0, R, np.array([0.1, 0.0, 3.0], np.float32)))
    Dt, Nt = [], []
    for cm in cams:
        D, N, _ = oracle.render(tgt.center, tgt.quat, tgt.radii, cm, 300.0)
        Dt.append(D.numpy().astype(np.float32).ravel())
        Nt.append(N.numpy().astype(np.float32).ravel())
    tD = torch.tensor(np.stack(Dt), device="cuda")
    tN = torch.tensor(np.stack(Nt), device="cuda")
    fit = SceneFit(ps.center, ps.quat, ps.radii, cams, tD, tN, cfg=FitConfig(check_every=1))
    table = fit.table.cpu().numpy()
    K = ps.K
    views_seen = set()
    for it in range(5):
        th0 = [t.detach().cpu().numpy().astype(np.float64) for t in (fit.c, fit.q, fit.r)]
        m0 = fit.m.cpu().numpy().astype(np.float64)
        v0 = fit.v.cpu().numpy().astype(np.float64)
        ite = int(fit.ite.item())
        assert ite == it
        view = int(table[ite % table.shape[0], 0])
        views_seen.add(view)
        cam = cams[view]
        lam = f32(oracle.lambda_at(ite))
        # the GPU's upstream gradient at this state (eager, the graph step's bits)
        rr = Renderer.single_scene([cam], K)
        lt = torch.tensor([lam], device="cuda")
        Dg, Ng = rr.render(_dev(th0[0]), _dev(th0[1]), _dev(th0[2]), lt)
        loss_g, gD, gN = rr.loss(Dg, Ng, tD[view], tN[view])
        gD = gD.cpu().numpy().reshape(cam.height, cam.width)
        gN = gN.cpu().numpy().reshape(3, cam.height, cam.width)
        fit.run(1, graph=True)
        torch.cuda.synchronize()
        assert abs(float(fit.lam.item()) - lam) == 0.0
        # the oracle's iteration from the same state
        Do, No, _ = oracle.render(th0[0], th0[1], th0[2], cam, lam)
        Lo = float(oracle.render_loss(Do, No, torch.as_tensor(Dt[view]).reshape(cam.height, cam.width),
                                      torch.as_tensor(Nt[view]).reshape(3, cam.height, cam.width)))
        assert float(loss_g[0, :3].sum()) == pytest.approx(Lo, rel=1e-5)
        grads, abss = oracle.per_pixel_abs_grad(th0[0], th0[1], th0[2], cam, lam, gD, gN)
        conds = oracle.weight_path_magnitude(th0[0], th0[1], th0[2], cam, lam, gD, gN)
        g = np.concatenate([x.numpy().ravel() for x in grads])
        e = np.concatenate([grad_check(x.numpy(), x.numpy(), s.numpy(), cond=cd.numpy())[1].ravel()
                            for x, s, cd in zip(grads, abss, conds)])
        theta = np.concatenate([x.ravel() for x in th0])
        ref, mref, vref = _adam_ref(theta, g, m0, v0, ite + 1)
        ref[7 * K:] = np.maximum(ref[7 * K:], 1e-4)
        spread = _adam_spread(theta, g, e, m0, v0, ite + 1)
        got = np.concatenate([t.detach().cpu().numpy().astype(np.float64).ravel() for t in (fit.c, fit.q, fit.r)])
        tol = spread + 4 * U32 * 2 * np.abs(theta) + 1e-9
        ratio = np.abs(got - ref) / tol
        moved = np.abs(ref - theta) > 0
        w = int(np.argmax(ratio))
        print(f"  worst coordinate {w}: theta {theta[w]:.9g} g {g[w]:.6g} +- {e[w]:.3g} ref {ref[w]:.9g} "
              f"gpu {got[w]:.9g} spread {spread[w]:.3g}", flush=True)
        print(f"views {n_views} iteration {ite} (view {view}, lambda {lam:.5g}): loss {Lo:.6g}, "
              f"max |step error| / bound {ratio.max():.3g}, {int(moved.sum())} of {theta.size} coordinates moved",
              flush=True)
        assert np.all(ratio <= 1.0)
        # Adam moments: the float32 moments of the GPU against the oracle's
        mg = fit.m.cpu().numpy().astype(np.float64)
        vg = fit.v.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(mg - mref) <= 0.1 * e + 4 * U32 * 2 * np.abs(mref) + 1e-30)
        assert np.all(np.abs(vg - vref) <= 0.001 * (2 * np.abs(g) * e + e * e) + 4 * U32 * 2 * np.abs(vref) + 1e-30)
    if n_views == 3:
        assert len(views_seen) >= 2
