"""Host-side pieces of the learned initialisation (no GPU): rotation helpers
against closed forms, plane-frame targets of unchanged planes, the smallest
rotation between normals."""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_quaternion_matrix_round_trip_and_closed_form():
    from paper_2412_03451_amd.learned_init import matrix_to_quat, quat_to_matrix
    rng = np.random.default_rng(0)
    q = rng.normal(size=(50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    R = quat_to_matrix(q)
    assert np.allclose(R @ np.swapaxes(R, 1, 2), np.eye(3), atol=1e-12)
    q2 = matrix_to_quat(R)
    q2[q2[:, 0] < 0] *= -1
    assert np.allclose(q, q2, atol=1e-10)
    # 90 degrees about x maps y to z
    c = math.cos(math.pi / 4)
    Rx = quat_to_matrix(np.array([c, c, 0.0, 0.0]))
    assert np.allclose(Rx @ np.array([0.0, 1.0, 0.0]), [0.0, 0.0, 1.0], atol=1e-12)


def test_local_targets_of_unchanged_planes_are_identity():
    from paper_2412_03451_amd.learned_init import local_targets
    rng = np.random.default_rng(1)
    c = rng.normal(size=(7, 3))
    q = rng.normal(size=(7, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    r = rng.uniform(0.1, 0.5, size=(7, 4))
    T = local_targets((c, q, r), (c, q, r))
    assert np.allclose(T[:, 0:3], 0, atol=1e-6)
    assert np.allclose(np.abs(T[:, 3]), 1, atol=1e-6)
    assert np.allclose(T[:, 7:11], r, atol=1e-6)
    # a pure shift along the plane normal appears as (0, 0, d) in the plane frame
    from paper_2412_03451_amd.learned_init import quat_to_matrix
    n = quat_to_matrix(q)[:, :, 2]
    T2 = local_targets((c, q, r), (c + 0.3 * n, q, r))
    assert np.allclose(T2[:, 0:3], [0, 0, 0.3], atol=1e-6)


def test_align_takes_a_to_b():
    from paper_2412_03451_amd.learned_init import _align
    rng = np.random.default_rng(2)
    a = rng.normal(size=(9, 3))
    b = rng.normal(size=(9, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    b[0] = a[0]
    R = _align(a, b)
    assert np.allclose(np.einsum("kij,kj->ki", R, a), b, atol=1e-10)
    assert np.allclose(R @ np.swapaxes(R, 1, 2), np.eye(3), atol=1e-10)
    assert np.allclose(R[0], np.eye(3))
