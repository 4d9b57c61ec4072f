"""Pins of the depth / sphere initialisation oracle (Sec. 3.1, Sec. 4.3).

Each pin checks the oracle against something it does not compute itself:
reprojection through the forward camera model, planes rendered by the
brute-force renderer, a closed-form voxel count, a dictionary walk over the
pixels, scipy's k-d tree, the rotation of Eq. 2-3 and the sphere's geometry.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import depth_init as di
from synth.scenes import Camera, quat_mul, random_depth_maps


def _rot_camera(seed, W=40, H=30, f=35.0):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    R = oracle.quat_to_frame(torch.as_tensor(q)[None])
    Rm = torch.stack(R, dim=-1)[0].numpy()          # columns vx, vy, n: a rotation matrix
    return Camera(W, H, f, f * 1.1, W / 2 + 0.3, H / 2 - 0.2, Rm.astype(np.float32),
                  rng.normal(size=3).astype(np.float32))


def _random_maps(cam, seed):
    return random_depth_maps(cam.width, cam.height, seed)


def test_back_projection_reprojects_to_the_pixel():
    cam = _rot_camera(3)
    D, N = _random_maps(cam, 4)
    p, n, ok = di.back_project(D[None], N[None], [cam], 1)
    H, W = cam.height, cam.width
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    D64, N64 = D.astype(np.float64), N.astype(np.float64)
    ln = np.linalg.norm(N64, axis=0)
    want_ok = (D64 > 0) & (ln >= 0.5)
    assert np.array_equal(ok, want_ok.reshape(-1))
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    Ri = np.linalg.inv(R.T)          # the float32 matrix is orthogonal only to ~1e-7
    pc = p[ok] @ Ri.T + t                                # world -> camera
    z = (D64 / np.where(ln > 0, ln, 1))[want_ok]
    assert np.allclose(pc[:, 2], z, rtol=1e-13, atol=1e-13)
    u = pc[:, 0] / pc[:, 2] * cam.fx + cam.cx
    v = pc[:, 1] / pc[:, 2] * cam.fy + cam.cy
    assert np.allclose(u, ii[want_ok] + 0.5, atol=1e-10)
    assert np.allclose(v, jj[want_ok] + 0.5, atol=1e-10)
    nc = n[ok] @ Ri.T
    assert np.allclose(nc, (N64 / np.where(ln > 0, ln, 1))[:, want_ok].T, atol=1e-13)


def test_points_lie_on_the_rendered_plane():
    cam = Camera(48, 36, 80.0, 80.0, 24.0, 18.0, np.eye(3, dtype=np.float32), np.array([0, 0, 3], np.float32))
    q = np.array([0.95, 0.2, -0.15, 0.1])
    q /= np.linalg.norm(q)
    c = np.array([[0.1, -0.05, 0.4]])
    r = np.array([[0.6, 0.4, 0.5, 0.3]])
    D, N, _ = oracle.render(c, q[None], r, cam, 300.0)
    D = D.numpy().astype(np.float32)
    N = N.numpy().astype(np.float32)
    p, n, ok = di.back_project(D[None], N[None], [cam], 1)
    assert ok.sum() > 200
    vx, vy, nz = (x.numpy()[0] for x in oracle.quat_to_frame(torch.as_tensor(q)[None]))
    full = np.linalg.norm(N.reshape(3, -1), axis=0) > 0.9999
    sel = ok & full
    off = (p[sel] - c[0]) @ nz
    assert np.abs(off).max() < 2e-6                     # float32 depth of the target map
    assert np.allclose(np.abs(n[sel] @ nz), 1.0, atol=1e-6)
    X, Y = (p[sel] - c[0]) @ vx, (p[sel] - c[0]) @ vy
    assert X.max() < r[0, 0] + 1e-3 and X.min() > -r[0, 1] - 1e-3
    assert Y.max() < r[0, 2] + 1e-3 and Y.min() > -r[0, 3] - 1e-3


def test_voxel_count_of_a_fronto_parallel_wall():
    cam = Camera(64, 48, 100.0, 100.0, 32.0, 24.0, np.eye(3, dtype=np.float32), np.array([0, 0, 3], np.float32))
    z0 = 2.0
    D = np.full((1, 48, 64), z0, np.float32)
    N = np.zeros((1, 3, 48, 64), np.float32)
    N[:, 2] = -1.0
    vox = 0.05
    pts, nrm = di.depth_points(D, N, [cam], stride=1, voxel=vox)
    # pixel spacing at z0 is 0.02 < voxel: every voxel between the extreme pixels is occupied
    xs = (np.array([0, 63]) + 0.5 - 32.0) / 100.0 * z0
    ys = (np.array([0, 47]) + 0.5 - 24.0) / 100.0 * z0
    v = float(np.float32(vox))
    nx = math.floor(xs[1] / v) - math.floor(xs[0] / v) + 1
    ny = math.floor(ys[1] / v) - math.floor(ys[0] / v) + 1
    assert pts.shape[0] == nx * ny
    assert np.all(pts[:, 2] == np.float32(z0 - 3.0))
    assert np.all(nrm == np.array([0, 0, -1], np.float32))
    # the first pixel of the first voxel is pixel (0, 0)
    assert np.allclose(pts[0, :2], [xs[0], ys[0]])


def test_one_point_per_voxel_is_the_first_pixel():
    cams = [_rot_camera(s, 20, 15, 12.0) for s in (7, 8)]
    maps = [_random_maps(cm, 20 + i) for i, cm in enumerate(cams)]
    D = np.stack([m[0] for m in maps])
    N = np.stack([m[1] for m in maps])
    vox = 0.3
    pts, nrm = di.depth_points(D, N, cams, stride=2, voxel=vox)
    # plain walk over the pixels in (view, row, column) order, one scalar at a time
    seen = {}
    order = []
    v32 = float(np.float32(vox))
    for v, cm in enumerate(cams):
        R = cm.R.astype(np.float64)
        t = cm.t.astype(np.float64)
        for j in range(0, cm.height, 2):
            for i in range(0, cm.width, 2):
                d = float(D[v, j, i])
                nv = N[v, :, j, i].astype(np.float64)
                ln = math.sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2])
                if not (d > 0 and ln >= 0.5):
                    continue
                z = d / ln
                pc = np.array([(i + 0.5 - cm.cx) / cm.fx * z, (j + 0.5 - cm.cy) / cm.fy * z, z])
                pw = R.T @ (pc - t)
                key = tuple(int(math.floor(x / v32)) for x in pw)
                if key not in seen:
                    seen[key] = len(order)
                    order.append(pw)
    assert pts.shape[0] == len(order)
    assert np.allclose(pts, np.array(order), atol=1e-6)
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0, atol=1e-6)


def test_depth_points_empty_and_out_of_range():
    cam = Camera(8, 6, 10.0, 10.0, 4.0, 3.0)
    D = np.zeros((1, 6, 8), np.float32)
    N = np.zeros((1, 3, 6, 8), np.float32)
    pts, nrm = di.depth_points(D, N, [cam], 1, 0.1)
    assert pts.shape == (0, 3) and nrm.shape == (0, 3)
    D[0, 2, 3] = 1.0
    N[0, 2, 2, 3] = 1.0
    pts, _ = di.depth_points(D, N, [cam], 1, 1e-7)     # |index| >= 2^20: dropped
    assert pts.shape[0] == 0
    pts, _ = di.depth_points(D, N, [cam], 1, 0.1)
    assert pts.shape[0] == 1


def test_radii_are_half_the_nearest_neighbour_distance():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    pts = rng.uniform(-2, 2, size=(700, 3)).astype(np.float32)
    nrm = rng.normal(size=(700, 3)).astype(np.float32)
    sel = rng.choice(700, 300, replace=False)
    c, q, r = di.init_from_points(pts, nrm, sel, r_min=1e-4)
    d, _ = cKDTree(pts[sel].astype(np.float64)).query(pts[sel].astype(np.float64), k=2)
    assert np.array_equal(c, pts[sel])
    assert np.allclose(r[:, 0], 0.5 * d[:, 1], rtol=1e-7)
    assert np.all(r == r[:, :1])
    # two coincident points: the radius floor
    c2, _, r2 = di.init_from_points(np.array([[0, 0, 0], [0, 0, 0], [1, 0, 0]], np.float32),
                                    np.ones((3, 3), np.float32), [0, 1, 2], r_min=1e-4)
    assert np.allclose(r2[:2], np.float32(1e-4)) and np.allclose(r2[2], 0.5)


def test_rotation_takes_ez_to_the_normal():
    rng = np.random.default_rng(6)
    n = rng.normal(size=(200, 3))
    n = np.concatenate([n, [[0, 0, 1], [0, 0, -1], [0, 0, -2.0], [1e-9, 0, -1]]])
    q = di.quat_from_normal(n)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-15)
    _, _, nz = oracle.quat_to_frame(torch.as_tensor(q))
    nh = n / np.linalg.norm(n, axis=1, keepdims=True)
    assert np.allclose(nz.numpy(), nh, atol=1e-12)
    assert np.allclose(q[200], [1, 0, 0, 0])
    # shortest arc: the rotation angle equals the angle between e_z and n
    ang = 2 * np.arccos(np.clip(q[:200, 0], -1, 1))
    assert np.allclose(ang, np.arccos(np.clip(nh[:200, 2], -1, 1)), atol=1e-7)
    # composing with a turn about the normal keeps the normal (the frame's spin is free)
    spin = np.array([math.cos(0.3), 0, 0, math.sin(0.3)])
    q2 = quat_mul(q[:5], spin[None])
    _, _, nz2 = oracle.quat_to_frame(torch.as_tensor(q2))
    assert np.allclose(nz2.numpy(), nh[:5], atol=1e-12)


def test_sphere_initialisation_geometry():
    rng = np.random.default_rng(8)
    pts = rng.uniform([0, 0, 0], [6, 5, 3], size=(500, 3)).astype(np.float32)
    u = rng.normal(size=(64, 3)).astype(np.float32)
    c, q, r = di.init_sphere(pts, u)
    ctr, R = di.bounding_sphere(pts)
    p64 = pts.astype(np.float64)
    assert np.allclose(ctr, 0.5 * (p64.min(0) + p64.max(0)))
    dist = np.linalg.norm(p64 - ctr, axis=1)
    assert dist.max() == pytest.approx(R, rel=1e-15) and np.all(dist <= R * (1 + 1e-15))
    assert np.allclose(np.linalg.norm(c.astype(np.float64) - ctr, axis=1), R, rtol=1e-6)
    _, _, nz = oracle.quat_to_frame(torch.as_tensor(q.astype(np.float64)))
    inward = (ctr - c.astype(np.float64))
    inward /= np.linalg.norm(inward, axis=1, keepdims=True)
    assert np.allclose(nz.numpy(), inward, atol=1e-5)
    assert np.all(r == np.float32(0.05))
