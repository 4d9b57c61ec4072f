"""Pins of the plane-merge oracle (Sec. 3.3): the angle and offset thresholds
on both sides, two-sided normals, transitivity, labels, and the instance
count of a ground-truth room against a sorted sweep of its face positions."""

import math

import numpy as np

import synth
from oracle.merge import merge_planes, normals_offsets


def _rot(axis, ang):
    axis = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis])


def test_angle_and_offset_thresholds():
    # plane 0: z = 0.5 (identity rotation); others tilted about X, or shifted along z
    q = np.array([[1.0, 0, 0, 0],
                  _rot([1, 0, 0], math.radians(24.9)),
                  _rot([1, 0, 0], math.radians(25.1)),
                  [1.0, 0, 0, 0],
                  [1.0, 0, 0, 0]], np.float32)
    c = np.array([[0, 0, 0.5], [0, 0, 0.5], [0, 0, 0.5], [0, 0, 0.5009], [0, 0, 0.5011]], np.float32)
    # offsets measured from the common point: all zero, only the angle decides
    ctr = np.array([0, 0, 0.5], np.float32)
    lab, n = merge_planes(c[[0, 1]], q[[0, 1]], scene_center=ctr)
    assert list(lab) == [0, 0] and n == 1
    lab, n = merge_planes(c[[0, 2]], q[[0, 2]], scene_center=ctr)
    assert list(lab) == [0, 1] and n == 2
    # 0.2 degrees apart, plane 1 links them: one instance
    lab, n = merge_planes(c[:3], q[:3], scene_center=ctr)
    assert list(lab) == [0, 0, 0] and n == 1
    z0 = np.zeros(3, np.float32)
    lab, n = merge_planes(c[[0, 3]], q[[0, 3]], scene_center=z0)     # 0.9 mm apart
    assert list(lab) == [0, 0] and n == 1
    lab, n = merge_planes(c[[0, 4]], q[[0, 4]], scene_center=z0)     # 1.1 mm apart
    assert list(lab) == [0, 1] and n == 2


def test_two_sided_and_transitive():
    flip = _rot([1, 0, 0], math.pi)             # normal -e_z, same plane z = 1
    q = np.array([[1.0, 0, 0, 0], flip, [1.0, 0, 0, 0], [1.0, 0, 0, 0]], np.float32)
    # offsets 1.0000, 1.0000 (opposite normal), 1.0008, 1.0016: a chain 0 ~ 2 ~ 3, 0 !~ 3
    c = np.array([[0, 0, 1.0], [3, 1, 1.0], [1, 0, 1.0008], [2, 0, 1.0016]], np.float32)
    _, o = normals_offsets(c, q, np.zeros(3, np.float32))
    assert o[1] < 0 < o[0]
    lab, n = merge_planes(c, q, scene_center=np.zeros(3, np.float32))
    assert list(lab) == [0, 0, 0, 0] and n == 1
    lab, n = merge_planes(c[[3, 0]], q[[3, 0]], scene_center=np.zeros(3, np.float32))
    assert list(lab) == [0, 1] and n == 2           # without the middle plane: apart


def test_ground_truth_room_instances():
    """Cells of one face share its plane exactly; instances are the groups of
    faces on one axis whose positions chain within 1 mm (a sorted sweep)."""
    gt, info = synth.room_planes(seed=3, target_K=600)
    X, Y, Z = info["room"]
    pos = {0: [0.0, X], 1: [0.0, Y], 2: [0.0, Z]}
    for (cx, cy, a, b, h) in info["boxes"]:
        pos[0] += [cx - a / 2, cx + a / 2]
        pos[1] += [cy - b / 2, cy + b / 2]
        pos[2] += [h]
    expect = 0
    for ax in range(3):
        p = np.sort(np.float32(pos[ax]).astype(np.float64))
        gaps = np.diff(p)
        assert np.all(np.abs(gaps - 1e-3) > 1e-5)       # no gap at the threshold within float32 rounding
        expect += 1 + int(np.sum(gaps >= 1e-3))
    lab, n = merge_planes(gt.center, gt.quat, scene_center=np.zeros(3, np.float32))
    assert n == expect
    # every label is the smallest index of its instance, and cells of one face agree
    for L in np.unique(lab):
        assert np.nonzero(lab == L)[0].min() == L
