"""Pins of the FP64 oracle against closed forms, invariants, symmetries and an
independent scalar brute force (CPU only).

Each test would fail under a plausible slip in the oracle: a dropped term of
the composite, a wrong sign of the facing normal, a swapped radius branch, a
transposed camera rotation, a wrong fringe margin or an off-by-half pixel
center.
"""

import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.render import OracleParams, fringe_margin

HERE = os.path.dirname(os.path.abspath(__file__))


def sig(x):
    if x < -700:
        return 0.0
    return 1.0 / (1.0 + math.exp(-x))


def one_plane(center, quat=(1.0, 0.0, 0.0, 0.0), radii=(0.3, 0.2, 0.25, 0.15)):
    return (np.asarray([center], np.float32), np.asarray([quat], np.float32),
            np.asarray([radii], np.float32))


# ---------------------------------------------------------------- P1: closed form
@pytest.mark.parametrize("mode", ["A", "B"])
@pytest.mark.parametrize("lam", [oracle.lambda_at(0), 60.0, 300.0])
def test_fronto_parallel_closed_form(mode, lam):
    """One plane facing the camera at world z0: every ray hits it at depth
    z0 + 3; with identity rotation P_X, P_Y are the world x, y offsets of the
    hit from the center; the normal faces the camera, (0, 0, -1)."""
    x0, y0, z0 = 0.11, -0.07, 0.4
    radii = (0.3, 0.2, 0.25, 0.15)
    c, q, r = one_plane((x0, y0, z0), radii=radii)
    cam = synth.tiny_camera()
    prm = OracleParams(weight_mode=mode)
    D, N, aux = oracle.render(c, q, r, cam, lam, prm)
    D = D.numpy()
    N = N.numpy()
    c32 = c[0].astype(np.float64)
    r32 = r[0].astype(np.float64)
    depth = c32[2] + 3.0
    n_interior = 0
    for j in range(cam.height):
        for i in range(cam.width):
            u = (i + 0.5 - cam.cx) / cam.fx
            v = (j + 0.5 - cam.cy) / cam.fy
            px = depth * u - c32[0]
            py = depth * v - c32[1]
            ax = (r32[0] if px > 0 else r32[1]) - abs(px)
            ay = (r32[2] if py > 0 else r32[3]) - abs(py)
            a = min(ax, ay)
            if mode == "A":
                w = 1.0 if a >= 0 else 2 * sig(5 * lam * a)
            else:
                w = sig(5 * lam * a)
            if w < 1e-4:
                w = 0.0
            if w == 1.0:
                n_interior += 1
            assert D[j, i] == pytest.approx(w * depth, rel=1e-12, abs=1e-13)
            assert N[0, j, i] == 0.0 and N[1, j, i] == 0.0
            assert N[2, j, i] == pytest.approx(-w, rel=1e-12, abs=1e-13)
    if mode == "A":
        assert n_interior > 100
        inside = aux["coverage"].numpy() == 1.0
        # interior pixels: depth exactly the plane depth, exact normal
        assert np.all(np.abs(D[inside] - depth) <= 4e-16 * depth)
        assert np.all(N[2][inside] == -1.0)


def test_fronto_parallel_gaussian_closed_form():
    """Mode "G" (Eq. 5): on a fronto-parallel plane the weight is the planar
    Gaussian of the in-plane offsets with the hit side's radius as standard
    deviation, cut at tau; depth w (z0 + 3), normal (0, 0, -w)."""
    x0, y0, z0 = 0.11, -0.07, 0.4
    radii = (0.1, 0.06, 0.08, 0.05)
    c, q, r = one_plane((x0, y0, z0), radii=radii)
    cam = synth.tiny_camera()
    D, N, aux = oracle.render(c, q, r, cam, 50.0, OracleParams(weight_mode="G"))
    D = D.numpy()
    N = N.numpy()
    c32 = c[0].astype(np.float64)
    r32 = r[0].astype(np.float64)
    depth = c32[2] + 3.0
    cut = 0
    for j in range(cam.height):
        for i in range(cam.width):
            px = depth * (i + 0.5 - cam.cx) / cam.fx - c32[0]
            py = depth * (j + 0.5 - cam.cy) / cam.fy - c32[1]
            sx = r32[0] if px > 0 else r32[1]
            sy = r32[2] if py > 0 else r32[3]
            w = math.exp(-0.5 * ((px / sx) ** 2 + (py / sy) ** 2))
            if w < 1e-4:
                w = 0.0
                cut += 1
            assert D[j, i] == pytest.approx(w * depth, rel=1e-12, abs=1e-13)
            assert N[2, j, i] == pytest.approx(-w, rel=1e-12, abs=1e-13)
    assert 0 < cut < cam.width * cam.height
    assert D.max() < depth                     # never opaque


# ---------------------------------------------------------------- P2: two planes
def test_two_stacked_planes_closed_form():
    lam = 30.0
    c = np.asarray([[0.0, 0.0, 0.2], [0.05, 0.02, 0.9]], np.float32)
    q = np.asarray([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32)
    r = np.asarray([[0.2, 0.2, 0.2, 0.2], [0.5, 0.4, 0.45, 0.35]], np.float32)
    cam = synth.tiny_camera()
    D, N, _ = oracle.render(c, q, r, cam, lam)
    D = D.numpy()
    N = N.numpy()
    c64 = c.astype(np.float64)
    r64 = r.astype(np.float64)
    for j in range(0, cam.height, 3):
        for i in range(0, cam.width, 3):
            u = (i + 0.5 - cam.cx) / cam.fx
            v = (j + 0.5 - cam.cy) / cam.fy
            ws, ts = [], []
            for k in range(2):
                t = c64[k, 2] + 3.0
                px, py = t * u - c64[k, 0], t * v - c64[k, 1]
                a = min((r64[k, 0] if px > 0 else r64[k, 1]) - abs(px),
                        (r64[k, 2] if py > 0 else r64[k, 3]) - abs(py))
                w = 1.0 if a >= 0 else 2 * sig(5 * lam * a)
                ws.append(w if w >= 1e-4 else 0.0)
                ts.append(t)
            d = ws[0] * ts[0] + (1 - ws[0]) * ws[1] * ts[1]
            n = ws[0] + (1 - ws[0]) * ws[1]
            assert D[j, i] == pytest.approx(d, rel=1e-12, abs=1e-13)
            assert N[2, j, i] == pytest.approx(-n, rel=1e-12, abs=1e-13)


# ---------------------------------------------------------------- scalar brute force
def _scalar_render(c, q, r, cam, lam, M=30, tau=1e-4, z_near=0.01):
    """Independent per-pixel, per-plane loop in plain Python floats."""
    K = len(c)
    Rc = [[float(cam.R[a][b]) for b in range(3)] for a in range(3)]
    tc = [float(x) for x in cam.t]
    o = [-(Rc[0][a] * tc[0] + Rc[1][a] * tc[1] + Rc[2][a] * tc[2]) for a in range(3)]
    frames = []
    for k in range(K):
        w_, x_, y_, z_ = (float(v) for v in q[k])
        s = math.sqrt(w_ * w_ + x_ * x_ + y_ * y_ + z_ * z_)
        w_, x_, y_, z_ = w_ / s, x_ / s, y_ / s, z_ / s
        Rm = [[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
              [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
              [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]]
        frames.append(([Rm[a][0] for a in range(3)], [Rm[a][1] for a in range(3)], [Rm[a][2] for a in range(3)]))
    D = np.zeros((cam.height, cam.width))
    N = np.zeros((3, cam.height, cam.width))
    for j in range(cam.height):
        for i in range(cam.width):
            dc = [(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, 1.0]
            d = [sum(Rc[b][a] * dc[b] for b in range(3)) for a in range(3)]
            hits = []
            for k in range(K):
                vx, vy, n = frames[k]
                p = [float(v) for v in c[k]]
                dn = sum(d[a] * n[a] for a in range(3))
                if abs(dn) <= 1e-12 * math.sqrt(sum(x * x for x in d)):
                    continue
                pon = sum((p[a] - o[a]) * n[a] for a in range(3))
                t = pon / dn
                if t <= z_near:
                    continue
                x = [o[a] + t * d[a] for a in range(3)]
                PX = sum((x[a] - p[a]) * vx[a] for a in range(3))
                PY = sum((x[a] - p[a]) * vy[a] for a in range(3))
                rk = [float(v) for v in r[k]]
                wx = 2 * sig(5 * lam * ((rk[0] if PX > 0 else rk[1]) - abs(PX)))
                wy = 2 * sig(5 * lam * ((rk[2] if PY > 0 else rk[3]) - abs(PY)))
                w = min(1.0, wx if wx < wy else wy)
                if w < tau:
                    continue
                sgn = -1.0 if pon > 0 else 1.0
                ncam = [sgn * sum(Rc[a][b] * n[b] for b in range(3)) for a in range(3)]
                hits.append((float(np.float32(t)), k, t, w, ncam))
            hits.sort(key=lambda h: (h[0], h[1]))
            T = 1.0
            for (_, _, t, w, ncam) in hits[:M]:
                D[j, i] += T * w * t
                for a in range(3):
                    N[a, j, i] += T * w * ncam[a]
                T *= 1 - w
    return D, N


def test_matches_scalar_brute_force():
    ps = synth.random_planes(6, seed=3, independent_radii=True, center_range=0.5)
    cam = synth.Camera(16, 12, 14.0, 14.0, 8.0, 6.0)
    # a rotated camera exercises the world/camera transforms
    ang = 0.3
    cam.R = np.asarray([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0], [-math.sin(ang), 0, math.cos(ang)]], np.float32)
    cam.t = np.asarray([0.1, -0.05, 2.5], np.float32)
    lam = 12.0
    D, N, _ = oracle.render(ps.center, ps.quat, ps.radii, cam, lam)
    Ds, Ns = _scalar_render(ps.center, ps.quat, ps.radii, cam, lam)
    assert (Ds > 0).sum() > 20
    np.testing.assert_allclose(D.numpy(), Ds, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(N.numpy(), Ns, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P3: invariants
@pytest.mark.parametrize("lam", [oracle.lambda_at(0), 300.0])
@pytest.mark.parametrize("mode", ["A", "B"])
def test_invariants(lam, mode):
    ps = synth.random_planes(64, seed=0)
    cam = synth.tiny_camera()
    prm = OracleParams(weight_mode=mode)
    D, N, aux = oracle.render(ps.center, ps.quat, ps.radii, cam, lam, prm)
    cov = aux["coverage"].numpy()
    assert np.all(cov >= 0) and np.all(cov <= 1 + 1e-12)
    nn = np.linalg.norm(N.numpy(), axis=0)
    assert np.all(nn <= cov + 1e-12)
    assert np.all(aux["count"].numpy() <= prm.M)
    # depth lies between (min t) * coverage and (max t) * coverage of the list
    from oracle.render import _pairs
    pix = torch.as_tensor(np.flatnonzero(aux["count"].numpy().ravel() > 0)[:400])
    c, q, r = (torch.as_tensor(x, dtype=torch.float64) for x in (ps.center, ps.quat, ps.radii))
    t = _pairs(c, q, r, cam, lam, pix, prm)["t"].numpy()
    ids = aux["ids"].reshape(-1, aux["ids"].shape[-1]).numpy()
    Df = D.numpy().ravel()
    covf = cov.ravel()
    for row, p in enumerate(pix.tolist()):
        sel = ids[p][ids[p] >= 0]
        ts = t[row, sel]
        assert ts.min() * covf[p] - 1e-12 <= Df[p] <= ts.max() * covf[p] + 1e-12
    assert np.all(D.numpy() >= 0)


def test_transmittance_and_order():
    """The selected list is ordered by float32 depth then plane index."""
    ps = synth.random_planes(64, seed=5)
    cam = synth.tiny_camera()
    pix = torch.arange(cam.width * cam.height)
    c, q, r = (torch.as_tensor(x, dtype=torch.float64) for x in (ps.center, ps.quat, ps.radii))
    from oracle.render import _pairs
    qq = _pairs(c, q, r, cam, 10.0, pix, OracleParams())
    D, N, aux = oracle.render_pixels(c, q, r, cam, 10.0, pix)
    t32 = qq["t"].to(torch.float32)
    ids = aux["ids"]
    for p in range(0, pix.numel(), 7):
        sel = ids[p][ids[p] >= 0]
        keys = [(t32[p, k].item(), k.item()) for k in sel]
        assert keys == sorted(keys)
        # every kept pair not in the list is behind the last selected one
        kept = torch.nonzero(qq["keep"][p]).flatten().tolist()
        assert set(sel.tolist()) <= set(kept)
        if len(kept) <= 30:
            assert len(kept) == len(sel)


# ---------------------------------------------------------------- P4: symmetries
def _render(c, q, r, cam, lam, prm=OracleParams()):
    D, N, _ = oracle.render(c, q, r, cam, lam, prm)
    return D.numpy(), N.numpy()


def test_quaternion_sign_and_scale():
    ps = synth.random_planes(64, seed=1)
    cam = synth.tiny_camera()
    D0, N0 = _render(ps.center, ps.quat, ps.radii, cam, 20.0)
    D1, N1 = _render(ps.center, -ps.quat, ps.radii, cam, 20.0)
    np.testing.assert_array_equal(D0, D1)
    np.testing.assert_array_equal(N0, N1)
    D2, N2 = _render(ps.center, 4.0 * ps.quat, ps.radii, cam, 20.0)  # exact in float32
    np.testing.assert_allclose(D2, D0, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(N2, N0, rtol=1e-10, atol=1e-10)


def _mismatch_fraction(a, b, tol=1e-9):
    return np.mean(np.abs(a - b) > tol)


def test_local_z_rotations_with_radius_relabelling():
    ps = synth.random_planes(48, seed=2, independent_radii=True)
    cam = synth.tiny_camera()
    D0, N0 = _render(ps.center, ps.quat, ps.radii, cam, 40.0)
    # 180 degrees about the local normal: v_x -> -v_x, v_y -> -v_y
    q180 = synth.quat_mul(ps.quat.astype(np.float64), np.array([0.0, 0.0, 0.0, 1.0])).astype(np.float32)
    r180 = ps.radii[:, [1, 0, 3, 2]]
    D1, N1 = _render(ps.center, q180, r180, cam, 40.0)
    assert _mismatch_fraction(D0, D1) < 2e-3
    # +90 degrees: v_x' = v_y, v_y' = -v_x
    h = math.sqrt(0.5)
    q90 = synth.quat_mul(ps.quat.astype(np.float64), np.array([h, 0.0, 0.0, h])).astype(np.float32)
    r90 = ps.radii[:, [2, 3, 1, 0]]
    D2, N2 = _render(ps.center, q90, r90, cam, 40.0)
    # q90 is rounded to float32 (~1e-7 rad), which moves fringe weights by ~1e-5
    assert _mismatch_fraction(D0, D2, 1e-4) < 2e-3
    assert _mismatch_fraction(N0, N2, 1e-4) < 2e-3
    # the wrong relabelling must visibly change the image
    D3, _ = _render(ps.center, q90, ps.radii, cam, 40.0)
    assert _mismatch_fraction(D0, D3, 1e-4) > 1e-2


def test_plane_permutation():
    ps = synth.random_planes(64, seed=4)
    cam = synth.tiny_camera()
    perm = np.random.default_rng(0).permutation(64)
    D0, N0 = _render(ps.center, ps.quat, ps.radii, cam, 20.0)
    D1, N1 = _render(ps.center[perm], ps.quat[perm], ps.radii[perm], cam, 20.0)
    np.testing.assert_allclose(D1, D0, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(N1, N0, rtol=1e-12, atol=1e-12)


def test_global_rigid_motion():
    ps = synth.random_planes(64, seed=6)
    cam = synth.tiny_camera()
    D0, N0 = _render(ps.center, ps.quat, ps.radii, cam, 25.0)
    g = np.array([math.cos(0.35), 0.3, -0.5, 0.2])
    g /= np.linalg.norm(g)
    w, x, y, z = g
    G = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    b = np.array([0.4, -1.2, 2.0])
    c2 = (ps.center.astype(np.float64) @ G.T + b).astype(np.float32)
    q2 = synth.quat_mul(g, ps.quat.astype(np.float64)).astype(np.float32)
    cam2 = synth.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                        (cam.R.astype(np.float64) @ G.T).astype(np.float32),
                        (cam.t.astype(np.float64) - cam.R.astype(np.float64) @ G.T @ b).astype(np.float32))
    D1, N1 = _render(c2, q2, ps.radii, cam2, 25.0)
    # float32 rounding of the moved inputs only perturbs fringe weights
    assert _mismatch_fraction(D0, D1, 1e-4) < 5e-3
    assert _mismatch_fraction(N0, N1, 1e-4) < 5e-3


# ---------------------------------------------------------------- P6: tiled == untiled
@pytest.mark.parametrize("lam", [oracle.lambda_at(0), 100.0, 300.0])
@pytest.mark.parametrize("tiles", [(8, 8), (16, 16), (32, 8)])
def test_tiled_equals_untiled(lam, tiles):
    ps = synth.random_planes(64, seed=7, independent_radii=True)
    cam = synth.tiny_camera()
    D0, N0, _ = oracle.render(ps.center, ps.quat, ps.radii, cam, lam)
    D1, N1, _ = oracle.render(ps.center, ps.quat, ps.radii, cam, lam, tiles=tiles)
    assert torch.equal(D0, D1) and torch.equal(N0, N1)


def test_fringe_margin_is_exact():
    """w = tau exactly at a = -delta for both weight modes."""
    for mode, lam in (("A", 7.0), ("A", 300.0), ("B", 50.0)):
        prm = OracleParams(weight_mode=mode)
        dl = fringe_margin(lam, prm)
        s = sig(5 * lam * -dl)
        w = 2 * s if mode == "A" else s
        assert w == pytest.approx(1e-4, rel=1e-12)


def test_behind_camera_and_near_clip():
    """A plane behind the camera renders nothing; one crossing the near plane
    only shows the part in front of it."""
    c, q, r = one_plane((0.0, 0.0, -3.5))
    cam = synth.tiny_camera()
    D, N, _ = oracle.render(c, q, r, cam, 50.0)
    assert float(D.abs().max()) == 0.0
    # tilted plane through the camera's z range
    h = math.sqrt(0.5)
    # 90 deg about x: a horizontal plane 0.2 m off the camera height reaching behind it
    c, q, r = one_plane((0.0, 0.2, -2.9), quat=(h, h, 0.0, 0.0), radii=(0.5, 0.5, 2.0, 2.0))
    D, N, aux = oracle.render(c, q, r, cam, 50.0)
    assert float(D.max()) > 0.0
    opaque = aux["coverage"] == 1.0
    assert int(opaque.sum()) > 100
    assert float(D[opaque].min()) > 0.01


def test_transmittance_behind_nearly_opaque_layers():
    """Mode B: behind two layers the transmittance is sigmoid(-z1) sigmoid(-z2)
    with full relative precision, although 1 - w is below 1e-12."""
    lam = 40.0
    c = np.asarray([[0.0, 0.0, 0.2], [0.0, 0.0, 0.9]], np.float32)
    q = np.asarray([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32)
    r = np.asarray([[0.25, 0.25, 0.25, 0.25], [0.3, 0.3, 0.3, 0.3]], np.float32)
    cam = synth.tiny_camera()
    D, N, aux = oracle.render(c, q, r, cam, lam, OracleParams(weight_mode="B"))
    j, i = cam.height // 2, cam.width // 2          # pixel (64, 48): ray offset (0.005, 0.005)
    u = (i + 0.5 - cam.cx) / cam.fx
    v = (j + 0.5 - cam.cy) / cam.fy
    T = 1.0
    for k in range(2):
        t = float(c[k, 2]) + 3.0
        a = min(float(r[k, 0]) - abs(t * u), float(r[k, 2]) - abs(t * v))
        z = 5 * lam * a
        T *= 1.0 / (1.0 + math.exp(z))           # sigmoid(-z)
    assert T < 1e-15
    assert float(aux["T"][j, i]) == pytest.approx(T, rel=1e-12)


def test_floor_through_the_camera_closed_form():
    """Plane 0 of the degenerate set: the floor y = 0.3 (camera frame) whose
    rectangle runs from 2 m behind to 2 m in front of the camera.  A pixel
    below the horizon sees it at z-depth t = 0.3 f / (v + 1/2 - c_y); where
    the hit lies inside the rectangle (|x| < 2, t < 2) the weight is 1, so
    D = t and the normal, turned to the camera, is (0, -1, 0).  Pixels above
    the horizon meet the plane behind the camera: nothing.  The plane through
    the camera center (t = 0), the one 5 mm away (inside the near distance)
    and the one behind the camera render nothing at all."""
    ps = synth.degenerate_planes()
    cam = synth.tiny_camera()
    lam = 50.0

    def sub(i):
        return ps.center[i:i + 1], ps.quat[i:i + 1], ps.radii[i:i + 1]
    D, N, aux = oracle.render(*sub(0), cam, lam)
    D = D.numpy().reshape(cam.height, cam.width)
    N = N.numpy().reshape(3, cam.height, cam.width).transpose(1, 2, 0)
    v = np.arange(cam.height)[:, None] + 0.5 - cam.cy
    u = np.arange(cam.width)[None, :] + 0.5 - cam.cx
    y0 = float(ps.center[0, 1])    # 0.3 rounded to float32
    t = np.where(v > 0, y0 * cam.fy / np.where(v > 0, v, 1.0), -1.0) * np.ones_like(u)
    x = t * u / cam.fx
    inside = (t > 0) & (t < 1.99) & (np.abs(x) < 1.99)
    assert inside.sum() > 500
    np.testing.assert_allclose(D[inside], t[inside], rtol=1e-12)
    np.testing.assert_allclose(N[inside], np.broadcast_to([0.0, -1.0, 0.0], N[inside].shape), rtol=0, atol=1e-12)
    above = np.broadcast_to(v < 0, D.shape)
    assert np.all(D[above] == 0.0) and np.all(N[above] == 0.0)
    for i in (1, 4, 5):
        Di, Ni, aux = oracle.render(*sub(i), cam, lam)
        assert float(Di.abs().max()) == 0.0 and float(Ni.abs().max()) == 0.0
        assert int(aux["count"].max()) == 0
