"""The learned initialisation on the GPU: a network trained on rooms fitted
by the plain method lowers the initial depth error of a held-out room and
reaches the plain fit's target depth error in no more iterations; a network
whose proposals are worse falls back to the plain initialisation."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

W, H, F, K, V = 320, 240, 288.5, 500, 20


def _room(seed):
    gt, info = synth.room_planes(seed=seed, target_K=K)
    cams = synth.room_trajectory(seed, V, info, width=W, height=H, f=F)
    init = synth.room_init_planes(gt, seed=seed + 7919)
    return {"gt": gt, "init": init, "cams": cams}


@pytest.fixture(scope="module")
def trained():
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd.initnet import InitNet
    rooms = [_room(1000 + i) for i in range(16)]
    fitted = li.fit_rooms(rooms, 1500)
    data = li.training_planes(rooms, fitted)
    net = InitNet(1, seed=0)
    hist = li.train_planes(net, data, 1000, batch=256, lr=1e-3)
    assert hist[-1][1] < 0.2 * hist[0][1]
    return net


def test_learned_init_lowers_error_and_iterations(trained):
    from paper_2412_03451_amd import learned_init as li
    rm = _room(5002)
    tD, tN = li.render_targets((rm["gt"].center, rm["gt"].quat, rm["gt"].radii), rm["cams"])
    init = (rm["init"].center, rm["init"].quat, rm["init"].radii)
    planes, info = li.learned_init(trained, init, rm["cams"], tD)
    print(info, flush=True)
    assert info["used"] == "learned"
    assert info["depth_l1_learned_init"] < 0.9 * info["depth_l1_plain_init"]
    it_p, s_p, e_p = li.iterations_to_target(init, rm["cams"], tD, tN, 0.02, 3000)
    it_l, s_l, e_l = li.iterations_to_target(planes, rm["cams"], tD, tN, 0.02, 3000)
    print(f"plain {it_p} its {s_p:.3f} s ({e_p:.4f}), learned {it_l} its {s_l:.3f} s ({e_l:.4f})", flush=True)
    assert e_l <= 0.02 and it_l <= it_p


def test_worse_proposals_fall_back_to_plain():
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd.initnet import InitNet, he_init, param_views
    flat = he_init(1, 3)
    param_views(flat, 1)["bh"][0:3] = [0.0, 0.0, 2.0]   # every plane pushed 2 m along its normal
    net = InitNet(1, params=flat)
    rm = _room(5003)
    tD, _ = li.render_targets((rm["gt"].center, rm["gt"].quat, rm["gt"].radii), rm["cams"])
    init = (rm["init"].center, rm["init"].quat, rm["init"].radii)
    planes, info = li.learned_init(net, init, rm["cams"], tD)
    assert info["used"] == "plain (fallback)"
    for a, b in zip(planes, init):
        assert np.array_equal(a, np.asarray(b, np.float32))
