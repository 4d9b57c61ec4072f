"""The learned initializer's per-view geometry on the GPU against its oracle
(oracle/viewinit.py), called through the C ABI: back-projected samples bit
for bit, decoded world proposals and refined planes to within one float32
unit in the last place, the nearest-proposal choices bit for bit."""

import numpy as np
import pytest
import torch

import synth
from oracle import viewinit as vi

pytestmark = pytest.mark.gpu


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _ulps(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return np.abs(a.astype(np.float64) - b.astype(np.float64)) / np.spacing(np.maximum(np.abs(a), np.abs(b)))


def _cams(n, W, H, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        ang = rng.uniform(0, np.pi)
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        R = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
        out.append(synth.Camera(W, H, 0.9 * W, 0.9 * W, W / 2 + 0.3, H / 2 - 0.2, R, rng.normal(size=3)))
    return out


def test_view_points_match_the_oracle(lib):
    from paper_2412_03451_amd._lib import check
    from paper_2412_03451_amd.splat import _ptr, _stream, pack_cameras
    V, H, W, N, n_cand = 5, 48, 64, 256, 600
    rng = np.random.default_rng(3)
    depth = rng.uniform(0.5, 6.0, (V, H, W)).astype(np.float32)
    depth[rng.random((V, H, W)) < 0.3] = 0.0
    depth[4, :, :] = 0.0
    depth[4, 10, 3:6] = 2.5          # a view with three valid pixels: the samples repeat
    cams = _cams(V, W, H, 4)
    cand = rng.integers(0, H * W, (V, n_cand)).astype(np.int32)
    eps = rng.normal(size=(V, n_cand)).astype(np.float32)
    X = torch.empty(V, N, 3, device="cuda")
    kept = torch.empty(V, dtype=torch.int32, device="cuda")
    d_depth, d_cams, d_cand, d_eps = _dev(depth), pack_cameras(cams), _dev(cand, torch.int32), _dev(eps)
    check(lib.initnet_view_points(_ptr(d_depth), _ptr(d_cams), V, H, W, _ptr(d_cand), _ptr(d_eps), n_cand, N, 0.01,
                                  _ptr(X), _ptr(kept), _stream()))
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    kept = kept.cpu().numpy()
    for v in range(V):
        Xr, kr = vi.view_points(depth[v], cams[v], cand[v], eps[v], N, 0.01)
        assert kept[v] == kr
        assert np.array_equal(X[v].view(np.uint32), Xr.view(np.uint32)), v


def test_proposals_to_world_match_the_oracle(lib):
    from paper_2412_03451_amd._lib import check
    from paper_2412_03451_amd.splat import _ptr, _stream, pack_cameras
    B, P = 6, 256
    rng = np.random.default_rng(5)
    out = rng.normal(0, 0.6, (B, 12 * P)).astype(np.float32)
    out[:, 3::12] = rng.uniform(-3.0, 3.0, (B, P))        # all branches of Shepperd's method
    cams = _cams(B, 64, 48, 6)
    view_cam = np.arange(B)[::-1].astype(np.int32)       # view b uses camera B-1-b
    c = torch.empty(B * P, 3, device="cuda")
    q = torch.empty(B * P, 4, device="cuda")
    r = torch.empty(B * P, 4, device="cuda")
    f = torch.empty(B * P, device="cuda")
    d_out, d_cams, d_vc = _dev(out), pack_cameras(cams), _dev(view_cam, torch.int32)
    check(lib.initnet_proposals_to_world(_ptr(d_out), B, P, _ptr(d_cams), _ptr(d_vc), _ptr(c), _ptr(q), _ptr(r),
                                         _ptr(f), _stream()))
    torch.cuda.synchronize()
    cr, qr, rr, fr = vi.proposals_to_world(out, [cams[i] for i in view_cam], P)
    for got, ref in ((c, cr), (q, qr), (r, rr), (f, fr)):
        assert _ulps(got.cpu().numpy(), ref).max() <= 1.0


def test_refinement_matches_the_oracle(lib):
    from paper_2412_03451_amd._lib import check
    from paper_2412_03451_amd.splat import _ptr, _stream
    K, Q = 300, 900
    init = synth.random_planes(K, seed=7, independent_radii=True)
    rng = np.random.default_rng(8)
    src = rng.integers(0, K, Q)
    pc = (init.center[src] + rng.normal(0, 0.08, (Q, 3))).astype(np.float32)
    pq = (init.quat[src] + rng.normal(0, 0.1, (Q, 4))).astype(np.float32)
    pr = (init.radii[src] * rng.uniform(0.7, 1.3, (Q, 4))).astype(np.float32)
    pf = rng.uniform(0, 1, Q).astype(np.float32)
    oc = torch.empty(K, 3, device="cuda")
    oq = torch.empty(K, 4, device="cuda")
    m = torch.empty(K, dtype=torch.int32, device="cuda")
    ins = [_dev(x) for x in (init.center, init.quat, init.radii, pc, pq, pr, pf)]   # alive through the call
    check(lib.initnet_refine_planes(_ptr(ins[0]), _ptr(ins[1]), _ptr(ins[2]), K, _ptr(ins[3]), _ptr(ins[4]),
                                    _ptr(ins[5]), _ptr(ins[6]), Q, 0.5, 0.05, _ptr(oc), _ptr(oq), _ptr(m), _stream()))
    torch.cuda.synchronize()
    ocr, oqr, mr = vi.refine_planes(init.center, init.quat, init.radii, pc, pq, pr, pf, 0.5, 0.05)
    m = m.cpu().numpy()
    print(f"refined {int((mr >= 0).sum())} of {K} planes", flush=True)
    assert np.array_equal(m, mr)
    assert 0 < (m >= 0).sum() < K
    assert _ulps(oc.cpu().numpy(), ocr).max() <= 1.0
    assert np.abs(oq.cpu().numpy() - oqr).max() <= 2.0 ** -23
