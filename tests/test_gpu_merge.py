"""plane_merge on the GPU against the oracle (Sec. 3.3): instance labels are
integer results decided in float64 with the same operations on both sides,
so they must be identical."""

import numpy as np
import pytest
import torch

import synth
from oracle.merge import default_center, merge_planes as oracle_merge
from synth.scenes import perturb_planes

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _check(center, quat, scene_center=None, angle=25.0, offset=0.001):
    from paper_2412_03451_amd.scene_init import merge_planes
    print(f"plane_merge K={center.shape[0]} angle={angle} offset={offset}", flush=True)
    lab, n = merge_planes(_dev(center), _dev(quat), None if scene_center is None else _dev(scene_center), angle,
                          offset)
    torch.cuda.synchronize()
    ol, on = oracle_merge(center, quat, scene_center, angle, offset)
    assert n == on
    assert np.array_equal(lab.cpu().numpy().astype(np.int64), ol)
    return on


def test_merge_ground_truth_and_perturbed_rooms():
    gt, _ = synth.room_planes(seed=3, target_K=2000)
    n_gt = _check(gt.center, gt.quat)
    assert 50 < n_gt < gt.K
    # small perturbations: chains of nearly coplanar cells, instances split and join
    noisy = perturb_planes(gt, seed=4, center_sigma=0.0005, rot_sigma_deg=0.5)
    _check(noisy.center, noisy.quat)
    _check(noisy.center, noisy.quat, scene_center=np.array([1.0, -2.0, 0.5], np.float32), offset=0.01)


def test_merge_random_planes_large_thresholds_and_single():
    ps = synth.random_planes(700, seed=9)
    n = _check(ps.center, ps.quat, angle=20.0, offset=0.05)
    assert 1 < n < 700
    _check(ps.center[:1], ps.quat[:1])
    assert _check(ps.center, ps.quat, default_center(ps.center), angle=1e-3, offset=1e-9) == 700
