"""Plane splitting on the GPU: plane_split matches the oracle's children
(count, parents, geometry), and a fit that splits every few iterations gives
the same bits replayed from a graph as run eagerly, across the splits."""

import numpy as np
import pytest
import torch

import synth
from oracle.split import split_planes as oracle_split

pytestmark = pytest.mark.gpu


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def test_split_matches_oracle():
    from paper_2412_03451_amd.splat import grad_accumulate, split_planes
    ps = synth.random_planes(300, seed=21, independent_radii=True)
    rng = np.random.default_rng(22)
    # accumulation: |g| summed in iteration order, count of iterations with a gradient
    acc = torch.zeros(300, 4, device="cuda")
    cnt = torch.zeros(300, dtype=torch.int32, device="cuda")
    h_acc = np.zeros((300, 4), np.float32)
    h_cnt = np.zeros(300, np.int64)
    for it in range(9):
        g = rng.normal(scale=0.3, size=(300, 4)).astype(np.float32)
        g[rng.uniform(size=300) < 0.3] = 0.0                  # planes not in this iteration's render
        g[rng.uniform(size=300) < 0.05, 1:] = 0.0             # a gradient on one radius only still counts
        grad_accumulate(_dev(g), acc, cnt)
        h_acc += np.abs(g)
        h_cnt += np.any(g != 0, axis=1)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), h_acc)
    assert np.array_equal(cnt.cpu().numpy(), h_cnt)
    # decision: per-plane averages kept away from the threshold by more than float32 roundoff
    scale = rng.choice([1.0, 0.5, 0.25], size=300).astype(np.float32)
    hc = np.maximum(h_cnt, 1)
    h_cnt = hc
    avg = np.stack([(h_acc[:, 0] + h_acc[:, 1]), (h_acc[:, 2] + h_acc[:, 3])], 1) * scale[:, None] / (2 * hc[:, None])
    h_acc[np.abs(avg[:, 0] - 0.2) < 1e-3, 0:2] += 0.05
    h_acc[np.abs(avg[:, 1] - 0.2) < 1e-3, 2:4] += 0.05
    c, q, r, parent, first = split_planes(_dev(ps.center), _dev(ps.quat), _dev(ps.radii), _dev(h_acc),
                                          _dev(h_cnt, torch.int32), _dev(scale), 0.2)
    torch.cuda.synchronize()
    oc, oq, orr, op = oracle_split(ps.center, ps.quat, ps.radii, h_acc, h_cnt, scale, 0.2)
    assert c.shape[0] == oc.shape[0] > 300
    assert np.array_equal(parent.cpu().numpy(), op)
    fh = first.cpu().numpy()
    assert fh[0] == 0 and fh[-1] == oc.shape[0]
    assert np.abs(c.cpu().numpy() - oc).max() <= 1e-6 * (1 + np.abs(oc).max())
    assert np.abs(r.cpu().numpy() - orr).max() <= 1e-6 * np.abs(orr).max()
    assert np.array_equal(q.cpu().numpy(), ps.quat[op])


def _room_fit(graph, split_every=40, iters=100, thresh=0.02):
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    gt, info = synth.room_planes(seed=31, target_K=150)
    cams = synth.room_trajectory(31, 4, info, width=128, height=96, f=115.4)
    init = synth.room_init_planes(gt, seed=32)
    tD, tN = li.render_targets((gt.center, gt.quat, gt.radii), cams)
    f = SceneFit(init.center, init.quat, init.radii, cams, tD, tN,
                 cfg=FitConfig(check_every=20, split_every=split_every, split_thresh=thresh))
    f.run(iters, graph=graph)
    torch.cuda.synchronize()
    return f


def test_fit_with_splitting_graph_equals_eager():
    fe = _room_fit(False)
    fg = _room_fit(True)
    print("splits", fe.splits, flush=True)
    assert len(fe.splits) == 2 and fe.splits == fg.splits
    assert fe.splits[0][2] > fe.splits[0][1]          # the plane set changed: the graph was captured again
    assert fe.K >= fe.splits[0][1]
    for a, b in zip(fe.state(), fg.state()):
        assert torch.equal(a, b)
    assert bool(torch.isfinite(fg.c).all()) and bool((fg.r > 0).all())
