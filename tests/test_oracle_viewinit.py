"""Pins of the oracle of the learned initializer's per-view geometry (CPU only):
closed forms of the back-projection, a round trip of the proposal decoding
through a camera, and constructed cases of the refinement."""

import math

import numpy as np

import synth
from oracle import viewinit as vi


def _rot(axis, ang):
    a = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_view_points_lie_on_the_pixel_rays():
    """A wall at depth 2: every kept point is z (1 + sigma eps) times the
    pixel-center ray with camera z = 1; invalid candidates are skipped in
    order and the kept points repeat when too few are valid."""
    cam = synth.tiny_camera(16, 12, 10.0)
    depth = np.full((12, 16), 2.0, np.float32)
    depth[3, :] = 0.0                                   # a row without surface
    rng = np.random.default_rng(0)
    cand = rng.integers(0, 16 * 12, 40)
    eps = rng.normal(size=40).astype(np.float32)
    X, kept = vi.view_points(depth, cam, cand, eps, 24, 0.01)
    valid = [i for i, p in enumerate(cand) if p // 16 != 3][:24]
    assert kept == 24
    for n, i in enumerate(valid):
        p = int(cand[i])
        z = 2.0 * (1.0 + float(np.float32(0.01)) * float(eps[i]))
        ray = ((p % 16 + 0.5 - cam.cx) / cam.fx, (p // 16 + 0.5 - cam.cy) / cam.fy, 1.0)
        np.testing.assert_allclose(X[n], np.asarray(ray) * z, rtol=1e-6)
    X2, kept2 = vi.view_points(depth, cam, cand[:5], eps[:5], 12, 0.0)
    k = sum(1 for p in cand[:5] if p // 16 != 3)
    assert kept2 == k
    for i in range(12):
        assert np.array_equal(X2[i], X2[i % k])


def test_proposal_round_trip_through_a_camera():
    """A world plane written in a camera's frame as the network's 12 numbers
    decodes back to the same world plane; the confidence is the sigmoid."""
    rng = np.random.default_rng(1)
    R = _rot(rng.normal(size=3), 0.7).astype(np.float32)
    t = np.array([0.3, -1.2, 2.5], np.float32)
    cam = synth.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, R, t)
    Rd, td = cam.R.astype(np.float64), cam.t.astype(np.float64)
    cw = np.array([1.0, 2.0, -0.5])
    Rw = _rot([0.2, 0.5, 1.0], 1.1)
    radii = np.array([0.3, 0.25, 0.4, 0.1])
    cc = Rd @ cw + td
    qc = np.asarray(vi.matrix_quat(Rd @ Rw))
    if qc[0] < 0:
        qc = -qc
    inv_softplus = np.log(np.expm1(radii - vi.R_MIN))
    out = np.concatenate([cc, qc - np.array([1.0, 0, 0, 0]), inv_softplus, [0.3]]).astype(np.float32)
    c, q, r, f = vi.proposals_to_world(out[None], [cam], 1)
    np.testing.assert_allclose(c[0], cw, atol=2e-5)
    np.testing.assert_allclose(vi.quat_matrix(q[0].astype(np.float64)), Rw, atol=2e-5)
    np.testing.assert_allclose(r[0], radii, atol=1e-5)
    assert abs(f[0] - 1 / (1 + math.exp(-float(np.float32(0.3))))) < 1e-7


def test_shepperd_matches_the_matrix_on_every_branch():
    rng = np.random.default_rng(2)
    for ang in (0.3, 2.0, 3.1):   # positive trace and the three diagonal branches
        for axis in ([1, 0.1, 0.1], [0.1, 1, 0.1], [0.1, 0.1, 1], rng.normal(size=3)):
            M = _rot(axis, ang)
            q = vi.matrix_quat(M)
            np.testing.assert_allclose(vi.quat_matrix(q), M, atol=1e-12)
            assert abs(np.linalg.norm(q) - 1) < 1e-15


def test_refinement_takes_the_supporting_plane():
    """An initial plane 5 cm off and 8 degrees tilted from a confident
    proposal: after the refinement its center lies on the proposal's plane,
    moved only along the new normal, its normal is the proposal's (turned to
    the initial side), and its radii and in-plane axes turn by the smallest
    rotation.  A less confident or a farther proposal leaves it unchanged;
    the nearest of two equal proposals is the one with the smaller index."""
    n_p = np.array([0.0, 0.0, -1.0])                  # proposal facing -z at z = 2
    pc = np.array([[0.2, 0.1, 2.0], [0.2, 0.1, 2.0], [5.0, 5.0, 5.0]], np.float32)
    R_p = _rot([1, 0, 0], math.pi)                    # e_z -> -e_z
    pq = np.tile(np.asarray(vi.matrix_quat(R_p), np.float32), (3, 1))
    pr = np.full((3, 4), 0.2, np.float32)
    conf = np.array([0.9, 0.9, 0.9], np.float32)
    R0 = _rot([1, 1, 0], math.radians(8.0))           # initial normal tilted from +z
    c0 = np.array([[0.25, 0.05, 2.05]], np.float32)
    q0 = np.asarray([vi.matrix_quat(R0)], np.float32)
    r0 = np.full((1, 4), 0.2, np.float32)
    oc, oq, m = vi.refine_planes(c0, q0, r0, pc, pq, pr, conf, 0.5, 0.05)
    assert m[0] == 0                                  # equal distances: the smaller index
    n1 = vi.quat_matrix(oq[0].astype(np.float64) / np.linalg.norm(oq[0]))[:, 2]
    n0 = R0[:, 2]
    assert np.dot(n1, n0) > 0                         # turned to the initial side
    np.testing.assert_allclose(np.abs(n1), np.abs(n_p), atol=1e-6)
    assert abs(float(oc[0][2]) - 2.0) < 1e-6          # onto the plane z = 2
    np.testing.assert_allclose(oc[0][:2], c0[0][:2], atol=1e-6)   # along the normal only
    # the smallest rotation: the rotation between the frames has its axis
    # perpendicular to both normals
    Rd = vi.quat_matrix(oq[0].astype(np.float64)) @ R0.T
    w, v = np.linalg.eig(Rd)
    axis = np.real(v[:, np.argmin(np.abs(w - 1))])
    assert abs(np.dot(axis, n0)) < 1e-6 and abs(np.dot(axis, n1)) < 1e-6
    # not confident enough, or too far
    _, _, m2 = vi.refine_planes(c0, q0, r0, pc, pq, pr, np.array([0.4, 0.4, 0.9], np.float32), 0.5, 0.05)
    assert m2[0] == -1
    _, _, m3 = vi.refine_planes(c0, q0, r0, pc, pq, pr, conf, 0.5, 1e-4)
    assert m3[0] == -1
