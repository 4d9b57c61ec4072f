"""Plane merge (oracle).  TEST INFRASTRUCTURE ONLY: see the package docstring.

Sec. 3.3 (plane merge paragraph): after the fit, primitives whose normals
differ by less than 25 degrees and whose offsets differ by less than 0.1 cm
are merged, the offset being the distance from the scene center to the plane
along its normal.  Readings:

* the normal of a plane is R(q) e_z with q normalised (Eq. 3); primitives
  are two-sided, so two planes are compared with the second one's normal
  turned towards the first's: with d = n_i . n_j, the pair is merged when
  |d| > cos(25 deg) and |o_i - sign(d) o_j| < 0.001 m, o = (p - c) . n;
* "merged" is transitive: plane instances are the connected components of
  that pair relation (no adjacency condition: the paper states none);
* the scene center c is an input; by default the middle of the axis-aligned
  box of the plane centers;
* every plane is labelled with the smallest plane index of its instance.

The pair test turns floats into a boolean, so it is written with one
rounding per operation in the order below (no fused multiply-add), in
float64 from the float32 parameters, and the kernel does the same.
"""

from __future__ import annotations

import math

import numpy as np


def normals_offsets(center, quat, scene_center):
    """Float64 normals [K,3] and offsets [K] in the pair test's arithmetic."""
    q = np.asarray(quat, np.float32).astype(np.float64)
    p = np.asarray(center, np.float32).astype(np.float64)
    c = np.asarray(scene_center, np.float32).astype(np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    qn = np.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / qn, x / qn, y / qn, z / qn
    n = np.stack([2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)], axis=1)
    o = (p[:, 0] - c[0]) * n[:, 0] + (p[:, 1] - c[1]) * n[:, 1] + (p[:, 2] - c[2]) * n[:, 2]
    return n, o


def default_center(center):
    """Middle of the axis-aligned box of the plane centers (float32)."""
    p = np.asarray(center, np.float32)
    return (0.5 * (p.min(axis=0).astype(np.float64) + p.max(axis=0).astype(np.float64))).astype(np.float32)


def merge_pairs(n, o, cos_thr: float, off_thr: float, rows=None):
    """Boolean [len(rows), K] pair relation (the diagonal included)."""
    K = n.shape[0]
    rows = np.arange(K) if rows is None else np.asarray(rows)
    d = (n[rows, None, 0] * n[None, :, 0] + n[rows, None, 1] * n[None, :, 1]) + n[rows, None, 2] * n[None, :, 2]
    oj = np.where(d >= 0.0, o[None, :], -o[None, :])
    return (np.abs(d) > cos_thr) & (np.abs(o[rows, None] - oj) < off_thr)


def merge_planes(center, quat, scene_center=None, angle_deg: float = 25.0, offset: float = 0.001):
    """int64 labels [K] (smallest index of each instance) and the instance count."""
    K = np.asarray(center).shape[0]
    if scene_center is None:
        scene_center = default_center(center)
    n, o = normals_offsets(center, quat, scene_center)
    cos_thr = math.cos(math.radians(angle_deg))
    off_thr = float(offset)
    label = -np.ones(K, np.int64)
    # breadth-first search over the pair relation, components found in index order
    for s in range(K):
        if label[s] >= 0:
            continue
        label[s] = s
        front = [s]
        while front:
            rel = merge_pairs(n, o, cos_thr, off_thr, rows=front)
            nxt = np.nonzero(rel.any(axis=0) & (label < 0))[0]
            label[nxt] = s
            front = list(nxt)
    return label, int(len(np.unique(label)))
