"""Single-direction radii (the plane-radii ablation of Sec. 4.3) on the GPU:
plane_tie_radii writes the pair sums exactly, and a fit with tied radii keeps
r+ and r- equal bit for bit, graph-replayed as eagerly."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_tie_radii_pair_sums():
    from paper_2412_03451_amd.splat import tie_radii
    rng = np.random.default_rng(5)
    g = rng.normal(size=(1001, 4)).astype(np.float32)
    t = torch.as_tensor(g, device="cuda")
    tie_radii(t)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    sx = g[:, 0] + g[:, 1]
    sy = g[:, 2] + g[:, 3]
    assert np.array_equal(out, np.stack([sx, sx, sy, sy], axis=1))


@pytest.mark.parametrize("graph", [False, True])
def test_fit_keeps_single_radii(graph):
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    gt, info = synth.room_planes(seed=41, target_K=150)
    cams = synth.room_trajectory(41, 4, info, width=128, height=96, f=115.4)
    init = synth.room_init_planes(gt, seed=42)
    tD, tN = li.render_targets((gt.center, gt.quat, gt.radii), cams)
    f = SceneFit(init.center, init.quat, init.radii, cams, tD, tN,
                 cfg=FitConfig(check_every=20, single_radii=True, split_every=30, split_thresh=0.02))
    f.run(80, graph=graph)
    torch.cuda.synchronize()
    r = f.r.cpu().numpy()
    print("K", f.K, "splits", f.splits, flush=True)
    assert np.array_equal(r[:, 0], r[:, 1]) and np.array_equal(r[:, 2], r[:, 3])
    assert np.all(np.isfinite(r)) and np.all(r > 0)
