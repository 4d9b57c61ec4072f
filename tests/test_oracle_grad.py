"""P7: the oracle's autograd gradient against float64 central finite
differences (CPU only).

The filter and the first-M cut make the rendered maps piecewise smooth; a
coordinate whose +-h perturbation changes any pixel's selected list or the
set of opaque entries is excluded, since a finite difference is meaningless
across a jump or a kink.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.render import OracleParams, _composite, _pairs


def _objective(c, q, r, cam, lam, gD, gN, prm):
    pix = torch.arange(cam.width * cam.height)
    qq = _pairs(c, q, r, cam, lam, pix, prm)
    D, N, aux = _composite(qq, prm)
    opaque = (qq["w"] >= 1) & qq["keep"]
    sig = (aux["ids"], opaque.sum(1))
    return float((gD * D).sum() + (gN * N).sum()), sig


@pytest.mark.parametrize("lam,mode", [(oracle.lambda_at(0), "A"), (60.0, "A"), (10.0, "G")])
def test_autograd_matches_central_differences(lam, mode):
    ps = synth.random_planes(12, seed=11, independent_radii=True, center_range=0.6)
    cam = synth.Camera(40, 30, 30.0, 30.0, 20.0, 15.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    prm = OracleParams(weight_mode=mode)
    rng = np.random.default_rng(0)
    P = cam.width * cam.height
    gD = torch.as_tensor(rng.normal(size=P))
    gN = torch.as_tensor(rng.normal(size=(P, 3)))
    gc, gq, gr = oracle.render_backward(ps.center, ps.quat, ps.radii, cam, lam,
                                        gD.numpy(), gN.numpy().T.copy(), prm)
    base = [torch.as_tensor(x, dtype=torch.float64) for x in (ps.center, ps.quat, ps.radii)]
    grads = [gc, gq, gr]
    h = 1e-6
    checked = 0
    for trial in range(60):
        which = int(rng.integers(3))
        k = int(rng.integers(base[which].shape[0]))
        comp = int(rng.integers(base[which].shape[1]))
        vals = []
        sigs = []
        for sgn in (+1, -1, 0):
            args = [b.clone() for b in base]
            args[which][k, comp] += sgn * h
            v, s = _objective(*args, cam, lam, gD, gN, prm)
            vals.append(v)
            sigs.append(s)
        same = all(torch.equal(sigs[i][0], sigs[2][0]) and torch.equal(sigs[i][1], sigs[2][1]) for i in (0, 1))
        if not same:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = float(grads[which][k, comp])
        assert fd == pytest.approx(ad, rel=2e-5, abs=2e-5 * (1 + abs(ad)))
        checked += 1
    assert checked >= 40


def test_per_pixel_abs_grad_sums_to_gradient():
    ps = synth.random_planes(8, seed=12, center_range=0.5)
    cam = synth.Camera(24, 18, 18.0, 18.0, 12.0, 9.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    rng = np.random.default_rng(1)
    P = cam.width * cam.height
    gD = rng.normal(size=P)
    gN = rng.normal(size=(3, P))
    ref = oracle.render_backward(ps.center, ps.quat, ps.radii, cam, 30.0, gD, gN)
    grads, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, 30.0, gD, gN, chunk=100)
    for a, b, s in zip(ref, grads, abss):
        np.testing.assert_allclose(b.numpy(), a.numpy(), rtol=1e-10, atol=1e-10)
        assert np.all(s.numpy() >= np.abs(b.numpy()) - 1e-12)


def test_single_radii_gradient_is_the_pair_sum():
    """Single-direction radii (Sec. 4.3 ablation): moving r^{x+} and r^{x-}
    together changes the objective at the rate g[x+] + g[x-] (likewise y),
    the gradient plane_tie_radii writes to both entries."""
    ps = synth.random_planes(10, seed=13, center_range=0.6)
    r = ps.radii.astype(np.float64)
    r[:, 1] = r[:, 0]
    r[:, 3] = r[:, 2]
    cam = synth.Camera(40, 30, 30.0, 30.0, 20.0, 15.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    prm = OracleParams()
    lam = oracle.lambda_at(0)
    rng = np.random.default_rng(3)
    P = cam.width * cam.height
    gD = torch.as_tensor(rng.normal(size=P))
    gN = torch.as_tensor(rng.normal(size=(P, 3)))
    _, _, gr = oracle.render_backward(ps.center, ps.quat, r, cam, lam, gD.numpy(), gN.numpy().T.copy(), prm)
    c = torch.as_tensor(ps.center, dtype=torch.float64)
    q = torch.as_tensor(ps.quat, dtype=torch.float64)
    h = 1e-6
    checked = 0
    for k in range(10):
        for ax in (0, 1):
            vals, sigs = [], []
            for sgn in (+1, -1, 0):
                rr = torch.as_tensor(r.copy())
                rr[k, 2 * ax] += sgn * h
                rr[k, 2 * ax + 1] += sgn * h
                v, s = _objective(c, q, rr, cam, lam, gD, gN, prm)
                vals.append(v)
                sigs.append(s)
            if not all(torch.equal(sigs[i][0], sigs[2][0]) and torch.equal(sigs[i][1], sigs[2][1]) for i in (0, 1)):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            tied = float(gr[k, 2 * ax] + gr[k, 2 * ax + 1])
            assert fd == pytest.approx(tied, rel=2e-5, abs=2e-5 * (1 + abs(tied)))
            checked += 1
    assert checked >= 12


def test_weight_path_magnitude_closed_form():
    """One pixel of the tiny camera (ray (0.005, 0.005, 1) from (0, 0, -3))
    through two fronto-parallel planes: plane 0 at z = 0 (t = 3) reaches the
    pixel through its x- fringe (a* = r^{x-} + P_X < 0, w_0 = 2 s(5 lam a*)),
    plane 1 at z = 1 (t = 4) covers it (w_1 = 1).  Both normals face the
    camera as (0, 0, -1), so
      M_0 = T_0 (|g_D| (t_0 + w_1 t_1) + |g_Nz| (1 + w_1)) = 7 |g_D| + 2 |g_Nz|,
    and the magnitude of a coordinate of plane 0 is M_0 |dw_0/dtheta| with
    |dw_0/dr^{x-}| = |dw_0/dx_0| = 10 lam s (1 - s), |dw_0/dz_0| = 0.005 of
    that; its other center and radius coordinates, and all of plane 1
    (w_1 = 1 flat), are 0."""
    cam = synth.tiny_camera()
    x0 = float(np.float32(0.3))
    center = np.array([[x0, 0.0, 0.0], [0.0, 0.0, 1.0]], np.float32)
    quat = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32)
    radii = np.array([[0.5, 0.2, 0.5, 0.5], [1, 1, 1, 1]], np.float32)
    lam = 10.0
    p = 48 * cam.width + 64
    P = cam.width * cam.height
    gD = np.zeros(P)
    gN = np.zeros((3, P))
    gD[p], gN[:, p] = -1.5, (0.25, -0.5, 0.75)
    mc, mq, mr = oracle.weight_path_magnitude(center, quat, radii, cam, lam, gD, gN, pix=[p])
    a = float(np.float32(0.2)) + (0.005 * 3.0 - x0)
    s = 1.0 / (1.0 + np.exp(-5.0 * lam * a))
    dw = 10.0 * lam * s * (1.0 - s)
    M0 = 7.0 * 1.5 + 2.0 * 0.75
    exp_c = np.zeros((2, 3))
    exp_c[0, 0], exp_c[0, 2] = M0 * dw, M0 * dw * 0.005
    exp_r = np.zeros((2, 4))
    exp_r[0, 1] = M0 * dw
    np.testing.assert_allclose(mc.numpy(), exp_c, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(mr.numpy(), exp_r, rtol=1e-9, atol=1e-12)
    # plane 1 is flat at w = 1: no magnitude for its rotation either
    assert float(mq[1].abs().max()) == 0.0 and float(mq[0].abs().max()) > 0.0


def test_weight_path_magnitude_bounds_the_weight_path():
    """On a random scene the magnitude dominates the gradient of the weight
    path alone (g . c_j - g . S_{j+1} replaced by its parts' magnitudes can
    only grow), coordinate by coordinate."""
    ps = synth.random_planes(24, seed=5, independent_radii=True, center_range=0.5)
    cam = synth.Camera(40, 30, 30.0, 30.0, 20.0, 15.0, np.eye(3, dtype=np.float32),
                       np.array([0.0, 0.0, 3.0], np.float32))
    lam = oracle.lambda_at(0)
    rng = np.random.default_rng(3)
    P = cam.width * cam.height
    gD = rng.normal(size=P)
    gN = rng.normal(size=(3, P))
    mags = oracle.weight_path_magnitude(ps.center, ps.quat, ps.radii, cam, lam, gD, gN, chunk=300)
    # the radius gradient runs through the weight only: bounded per coordinate
    _, abss = oracle.per_pixel_abs_grad(ps.center, ps.quat, ps.radii, cam, lam, gD, gN, chunk=300)
    assert np.all(mags[2].numpy() >= abss[2].numpy() * (1 - 1e-12))
    assert float(mags[2].sum()) > 0.0
