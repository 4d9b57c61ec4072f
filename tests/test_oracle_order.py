"""Pins of the oracle's per-ray order reading and of its tiled evaluation (CPU only).

Sec. 3.2 sorts each ray's surviving intersections by depth.  The order is an
integer result decided by floating point; the oracle decides it on the depth
rounded to float32 by default (the precision the kernels decide it in) and on
the exact float64 depth with OracleParams(order="f64").  These tests state
what separates the two readings: the orders differ only by permutations
inside runs of hits whose depths round to the same float32 value, and the
rendered depth and normal then differ by no more than what such a run can
move them (bounds computed from the hits themselves).  They also pin the tiled
evaluation (each tile against its candidate planes only) to the brute force,
bit for bit, which the full-size parity tests rely on.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.render import OracleParams, _pairs, _t

F32_LAM0 = float(np.float32(oracle.lambda_at(0)))


def _room():
    gt, info = synth.room_planes(seed=0, target_K=2000)
    init = synth.room_init_planes(gt, seed=1)
    cams = synth.room_trajectory(seed=0, n_views=2, info=info)
    return init, cams


@pytest.mark.parametrize("mode", ["A", "B", "G"])
@pytest.mark.parametrize("tiles", [(16, 16), (8, 8), (32, 8)])
def test_tiled_evaluation_equals_brute_force_tiny(mode, tiles):
    ps = synth.random_planes(64, seed=3, independent_radii=True)
    cam = synth.tiny_camera()
    prm = OracleParams(weight_mode=mode)
    for lam in (F32_LAM0, 300.0):
        D0, N0, a0 = oracle.render(ps.center, ps.quat, ps.radii, cam, lam, prm)
        D1, N1, a1 = oracle.render_tiled(ps.center, ps.quat, ps.radii, cam, lam, prm, tiles)
        assert torch.equal(D0, D1) and torch.equal(N0, N1)
        assert torch.equal(a0["ids"], a1["ids"]) and torch.equal(a0["T"], a1["T"])
        assert torch.equal(a0["count"], a1["count"])


def test_tiled_evaluation_equals_brute_force_room():
    """Full-size room view (640x480, ~2000 planes): the tiled evaluation equals
    the brute force on every 61st pixel, bit for bit."""
    init, cams = _room()
    cam = cams[0]
    pix = torch.arange(0, cam.width * cam.height, 61)
    for lam in (F32_LAM0, 300.0):
        D1, N1, a1 = oracle.render_tiled(init.center, init.quat, init.radii, cam, lam)
        D0, N0, a0 = oracle.render_pixels(init.center, init.quat, init.radii, cam, lam, pix)
        assert torch.equal(D0, D1.reshape(-1)[pix])
        assert torch.equal(N0, N1.reshape(3, -1).T[pix])
        assert torch.equal(a0["ids"], a1["ids"].reshape(-1, a1["ids"].shape[-1])[pix])


def _compare_orders(center, quat, radii, cam, lam, render, n_check=1500):
    """Render with both order readings; returns (differing pixels, max |dD|,
    max |dN| over all of them, max |dD| / bound, max |dN| / bound over
    n_check of them spread evenly), after checking at those pixels that the
    two ordered lists carry the same float32 depth at every position (they
    differ only inside float32 ties)."""
    D32, N32, a32 = render(center, quat, radii, cam, lam, OracleParams(order="f32"))
    D64, N64, a64 = render(center, quat, radii, cam, lam, OracleParams(order="f64"))
    ids32 = a32["ids"].reshape(-1, a32["ids"].shape[-1])
    ids64 = a64["ids"].reshape(-1, a64["ids"].shape[-1])
    diff = torch.nonzero((ids32 != ids64).any(1)).flatten()
    D32, D64 = D32.reshape(-1), D64.reshape(-1)
    N32, N64 = N32.reshape(3, -1).T, N64.reshape(3, -1).T
    # where the lists agree, the maps agree bit for bit
    same = torch.ones(D32.numel(), dtype=torch.bool)
    same[diff] = False
    assert torch.equal(D32[same], D64[same]) and torch.equal(N32[same], N64[same])
    if diff.numel() == 0:
        return 0, 0.0, 0.0, 0.0, 0.0
    n_diff = int(diff.numel())
    worst_d = float((D64[diff] - D32[diff]).abs().max())
    worst_n = float((N64[diff] - N32[diff]).abs().max())
    if n_diff > n_check:
        diff = diff[torch.linspace(0, n_diff - 1, n_check).round().long()]
    planes = torch.unique(torch.cat([ids32[diff], ids64[diff]]).flatten())
    planes = planes[planes >= 0]
    q = _pairs(_t(center)[planes], _t(quat)[planes], _t(radii)[planes], cam, lam, diff, OracleParams())
    col = {int(k): i for i, k in enumerate(planes.tolist())}
    rd = rn = 0.0
    for row, p in enumerate(diff.tolist()):
        l32 = [int(k) for k in ids32[p] if k >= 0]
        l64 = [int(k) for k in ids64[p] if k >= 0]
        assert len(l32) == len(l64)
        t = {k: float(q["t"][row, col[k]]) for k in set(l32) | set(l64)}
        w = {k: float(q["w"][row, col[k]]) for k in t}
        nrow = q["n"][row if q["n"].shape[0] > 1 else 0]
        n = {k: nrow[col[k]].numpy() for k in t}
        f32 = {k: float(np.float32(t[k])) for k in t}
        # same float32 depth at every position: only ties in float32 reorder
        assert [f32[k] for k in l32] == [f32[k] for k in l64], (p, l32, l64)
        # bound: the lists split into the same runs of equal float32 depth.
        # A run with the same members in both lists is a weighted average
        # whose total weight (transmittance in front of it times
        # 1 - prod(1 - w)) does not depend on the order inside it, so the two
        # orders differ by at most that weight times the spread of depth (of
        # each normal component) inside the run.  A run cut by the M-th
        # position may keep different members; it is bounded by the whole
        # transmittance in front of it times the largest value.
        bD = 0.0
        bN = np.zeros(3)
        Tf = 1.0
        j = 0
        while j < len(l32):
            k = j
            while k < len(l32) and f32[l32[k]] == f32[l32[j]]:
                k += 1
            run = set(l32[j:k]) | set(l64[j:k])
            ts = [t[m] for m in run]
            ns = np.array([n[m] for m in run])
            if set(l32[j:k]) == set(l64[j:k]):
                keep = 1.0
                for m in l32[j:k]:
                    keep *= 1.0 - w[m]
                bD += Tf * (1.0 - keep) * (max(ts) - min(ts))
                bN += Tf * (1.0 - keep) * (ns.max(0) - ns.min(0))
                Tf *= keep
            else:
                assert k == len(l32)   # only at the end of a full list
                bD += Tf * max(abs(x) for x in ts)
                bN += Tf * 2.0 * np.abs(ns).max(0)
            j = k
        dD = abs(float(D64[p]) - float(D32[p]))
        dN = np.abs(N64[p].numpy() - N32[p].numpy())
        tolD = bD + 1e-14 * max(1.0, abs(float(D32[p])))
        tolN = bN + 1e-14
        rd = max(rd, dD / tolD)
        rn = max(rn, float((dN / tolN).max()))
    return n_diff, worst_d, worst_n, rd, rn


def test_order_readings_tiny_scene():
    """The small configuration (64 planes, 128x96): float32 ties are rare, and
    wherever the orders differ the maps move within the bound."""
    ps = synth.random_planes(64, seed=0)
    cam = synth.tiny_camera()
    for lam in (F32_LAM0, 300.0):
        n, dD, dN, rd, rn = _compare_orders(ps.center, ps.quat, ps.radii, cam, lam, oracle.render)
        print(f"tiny lam {lam:.4g}: {n} pixels differ, max |dD| {dD:.3g}, max |dN| {dN:.3g}")
        assert rd <= 1.0 and rn <= 1.0


def test_order_readings_room_views():
    """Two full 640x480 views of the room (K ~ 2000) from the noisy
    initialisation and from the ground truth, at lambda(0) and 300.  Cells of
    one box face are coplanar and overlap in their fringes, so their hits tie
    in float32 on many pixels; both readings then give the same maps to
    float64 rounding, and no pixel moves beyond the bound."""
    gt, info = synth.room_planes(seed=0, target_K=2000)
    init = synth.room_init_planes(gt, seed=1)
    cams = synth.room_trajectory(seed=0, n_views=2, info=info)
    total = 0
    for name, ps in (("init", init), ("gt", gt)):
        for cam_i, cam in enumerate(cams):
            for lam in (F32_LAM0, 300.0):
                n, dD, dN, rd, rn = _compare_orders(ps.center, ps.quat, ps.radii, cam, lam, oracle.render_tiled)
                total += n
                print(f"room {name} view {cam_i} lam {lam:.4g}: {n} pixels differ, max |dD| {dD:.3g} m, "
                      f"max |dN| {dN:.3g}, worst / bound {max(rd, rn):.3g}")
                assert rd <= 1.0 and rn <= 1.0
                # the maps of the two readings agree within the forward's parity bar
                assert dD <= 1e-5 and dN <= 1e-5
    assert total > 0   # the float32 ties do occur on this workload
