"""Scene initialisation from depth maps, and the sphere initialisation (oracle).

TEST INFRASTRUCTURE ONLY: see the package docstring.

Sec. 3.1 (scene initialisation): plane centers are random points of a coarse
surface built from monocular depth; each plane's radii are half the distance
to its nearest neighbouring center and its rotation follows the surface
normal.  Sec. 4.3 (plane-initialisation ablation): the alternative places
the planes on the scene's bounding sphere, radii 0.05, normals towards the
sphere's center.  Readings:

* coarse surface = the voxels (edge `voxel`, grid anchored at the world
  origin) occupied by the back-projected pixels of the depth maps; one point
  per voxel, the back-projection of the first pixel (view, row, column order)
  that falls in it, with the normal of that pixel.  Sampling points uniformly
  over occupied voxels samples the fused surface about uniformly by area, as
  sampling a mesh does;
* pixels are taken every `stride` rows and columns starting at (0, 0); a
  pixel counts when its depth is > 0 and its normal has length >= 0.5; its
  depth is D / |N| and its normal N / |N| (for a pixel covered by one plane
  with weight w, D = w t and |N| = w, so this undoes partial coverage);
* the point of pixel (i, j) is x = R^T (t_z d_c - t) with
  d_c = ((i + 1/2 - c_x) / f_x, (j + 1/2 - c_y) / f_y, 1), the normal R^T n_c;
  voxel index floor(x / voxel) per axis; points with an index of magnitude
  >= 2^20 on any axis are dropped;
* the planes' points are K distinct voxel indices drawn by the caller
  (random numbers are inputs); every radius is max(0.5 d_nn, r_min);
* the rotation is the shortest arc from e_z to the normal,
  q ~ (1 + n_z, -n_y, n_x, 0); a normal exactly opposite to e_z gives the
  half turn about the X axis;
* bounding sphere: center = middle of the points' axis-aligned box, radius =
  largest distance from it to a point; plane k sits at c + R u_k for the
  caller's direction u_k (normalised), facing the center.

All arithmetic is float64, each operation in the order written here (no
fused multiply-add): decisions that turn a float into an integer (validity,
voxel index) are taken in float64 on both sides.
"""

from __future__ import annotations

import numpy as np

VOXEL_RANGE = 1 << 20


def back_project(depth, normal, cams, stride: int):
    """Every stride-th pixel of every view, in (view, row, column) order:
    (points [N,3], normals [N,3], valid [N]) in float64."""
    pts, nrm, val = [], [], []
    for v, cam in enumerate(cams):
        D = np.asarray(depth[v], np.float32).astype(np.float64)
        N = np.asarray(normal[v], np.float32).astype(np.float64)
        rows = np.arange(0, cam.height, stride)
        cols = np.arange(0, cam.width, stride)
        jj, ii = np.meshgrid(rows, cols, indexing="ij")
        d = D[jj, ii].reshape(-1)
        nx, ny, nz = (N[c][jj, ii].reshape(-1) for c in range(3))
        nn = np.sqrt(nx * nx + ny * ny + nz * nz)
        ok = (d > 0) & (nn >= 0.5)
        safe = np.where(ok, nn, 1.0)
        z = d / safe
        xc = (ii.reshape(-1).astype(np.float64) + 0.5 - float(cam.cx)) / float(cam.fx)
        yc = (jj.reshape(-1).astype(np.float64) + 0.5 - float(cam.cy)) / float(cam.fy)
        R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
        t = np.asarray(cam.t, np.float32).astype(np.float64).reshape(3)
        q0, q1, q2 = xc * z - t[0], yc * z - t[1], z - t[2]
        m0, m1, m2 = nx / safe, ny / safe, nz / safe
        pts.append(np.stack([R[0, r] * q0 + R[1, r] * q1 + R[2, r] * q2 for r in range(3)], axis=1))
        nrm.append(np.stack([R[0, r] * m0 + R[1, r] * m1 + R[2, r] * m2 for r in range(3)], axis=1))
        val.append(ok)
    if not pts:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, bool)
    return np.concatenate(pts), np.concatenate(nrm), np.concatenate(val)


def voxel_index(points, voxel: float):
    """Integer voxel coordinates [N,3] and whether they are inside the range."""
    idx = np.floor(points / float(np.float32(voxel)))
    inside = np.all(np.abs(idx) < VOXEL_RANGE, axis=1)
    return idx, inside


def depth_points(depth, normal, cams, stride: int = 4, voxel: float = 0.02):
    """One float32 point and normal per occupied voxel, voxels numbered in the
    order of their first pixel."""
    p, n, ok = back_project(depth, normal, cams, stride)
    idx, inside = voxel_index(p, voxel)
    keep = np.nonzero(ok & inside)[0]
    if keep.size == 0:
        return np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32)
    key = idx[keep].astype(np.int64) + VOXEL_RANGE
    key = (key[:, 0] << 42) | (key[:, 1] << 21) | key[:, 2]
    _, first = np.unique(key, return_index=True)   # first occurrence = lowest pixel index
    rep = np.sort(keep[first])
    return p[rep].astype(np.float32), n[rep].astype(np.float32)


def quat_from_normal(n):
    """Unit quaternion (w, x, y, z) of the shortest rotation taking e_z to the
    direction of n; [K,3] -> [K,4], float64."""
    n = np.asarray(n, np.float64)
    ln = np.sqrt(n[:, 0] * n[:, 0] + n[:, 1] * n[:, 1] + n[:, 2] * n[:, 2])
    nx, ny, nz = n[:, 0] / ln, n[:, 1] / ln, n[:, 2] / ln
    # w = 1 + n_z, written without cancellation for n_z < 0 (|n| = 1)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(nz >= 0, 1.0 + nz, (nx * nx + ny * ny) / (1.0 - nz))
    x, y = -ny, nx
    flip = w <= 0
    w = np.where(flip, 0.0, w)
    x = np.where(flip, 1.0, x)
    y = np.where(flip, 0.0, y)
    lq = np.sqrt(w * w + x * x + y * y)
    return np.stack([w / lq, x / lq, y / lq, np.zeros_like(w)], axis=1)


def nearest_distance_sq(c):
    """Squared distance from each point to its nearest other point, brute force."""
    c = np.asarray(c, np.float32).astype(np.float64)
    K = c.shape[0]
    out = np.empty(K)
    for k0 in range(0, K, 512):
        a = c[k0:k0 + 512]
        dx = a[:, None, 0] - c[None, :, 0]
        dy = a[:, None, 1] - c[None, :, 1]
        dz = a[:, None, 2] - c[None, :, 2]
        d2 = dx * dx + dy * dy + dz * dz
        d2[np.arange(a.shape[0]), np.arange(k0, k0 + a.shape[0])] = np.inf
        out[k0:k0 + 512] = d2.min(axis=1)
    return out


def init_from_points(pts, nrm, sel, r_min: float = 1e-4):
    """Planes on the selected points (Sec. 3.1): float32 (center, quat, radii)."""
    sel = np.asarray(sel, np.int64)
    c = np.asarray(pts, np.float32)[sel]
    d = np.sqrt(nearest_distance_sq(c))
    r = np.maximum(0.5 * d, float(np.float32(r_min))).astype(np.float32)
    q = quat_from_normal(np.asarray(nrm, np.float32)[sel].astype(np.float64)).astype(np.float32)
    return c.copy(), q, np.repeat(r[:, None], 4, axis=1)


def bounding_sphere(pts):
    """(center [3], radius) of the points' box-centered bounding sphere, float64."""
    p = np.asarray(pts, np.float32).astype(np.float64)
    c = 0.5 * (p.min(axis=0) + p.max(axis=0))
    d = p - c
    return c, float(np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]).max()))


def init_sphere(pts, dirs, radius: float = 0.05):
    """Sphere initialisation (Sec. 4.3): float32 (center, quat, radii)."""
    c, R = bounding_sphere(pts)
    u = np.asarray(dirs, np.float32).astype(np.float64)
    lu = np.sqrt(u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1] + u[:, 2] * u[:, 2])
    u = u / lu[:, None]
    centers = c[None, :] + R * u
    q = quat_from_normal(-u)
    r = np.full((u.shape[0], 4), np.float32(radius), np.float32)
    return centers.astype(np.float32), q.astype(np.float32), r
