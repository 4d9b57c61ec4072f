"""Scene initialisation over the C ABI: planes from depth maps (Sec. 3.1)
and the sphere initialisation of the ablation (Sec. 4.3); the plane merge
after the fit (Sec. 3.3).

The random draws (which fused points become planes, the directions on the
sphere) are made here with a seeded numpy generator and passed to the
kernels; every computation runs in libplanesplat.so.  Typical use::

    c, q, r = init_from_depth(tgt_depth, tgt_normal, cams, K=2000, seed=0)
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import check
from .splat import _ptr, _stream, pack_cameras


def _cams_dev(cams, device):
    return cams if torch.is_tensor(cams) else pack_cameras(cams, device)


def depth_points(depth, normal, cams, stride: int = 4, voxel: float = 0.02, cap: int | None = None):
    """One point and normal per occupied voxel of the back-projected maps
    (depth_points).  depth [V,H,W], normal [V,3,H,W] on the device; returns
    (points [n',3], normals [n',3], n) with n' = min(n, cap)."""
    lib = _lib.load()
    V, H, W = (int(x) for x in depth.shape)
    assert tuple(normal.shape) == (V, 3, H, W), "normal must be [V, 3, H, W]"
    dev = depth.device
    depth = depth.contiguous().float()
    normal = normal.contiguous().float()
    n_cand = V * (-(-H // stride)) * (-(-W // stride))
    cap = n_cand if cap is None else int(cap)
    nbytes = int(lib.depth_points_ws_bytes(V, H, W, int(stride)))
    if nbytes == 0:
        raise ValueError("depth_points: unsupported sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    pts = torch.empty(max(cap, 1), 3, dtype=torch.float32, device=dev)
    nrm = torch.empty(max(cap, 1), 3, dtype=torch.float32, device=dev)
    n_out = torch.empty(1, dtype=torch.int32, device=dev)
    cd = _cams_dev(cams, dev)
    check(lib.depth_points(_ptr(depth), _ptr(normal), _ptr(cd), V, H, W, int(stride), float(voxel), _ptr(pts),
                           _ptr(nrm), cap, _ptr(n_out), _ptr(ws), nbytes, _stream()))
    n = int(n_out.item())
    m = min(n, cap)
    return pts[:m], nrm[:m], n


def init_from_points(points, normals, sel, r_min: float = 1e-4):
    """Planes on points[sel] (plane_init_points): (center, quat, radii)."""
    lib = _lib.load()
    dev = points.device
    sel = torch.as_tensor(np.asarray(sel, np.int32) if not torch.is_tensor(sel) else sel,
                          dtype=torch.int32).to(dev).contiguous()
    K = int(sel.shape[0])
    c = torch.empty(K, 3, dtype=torch.float32, device=dev)
    q = torch.empty(K, 4, dtype=torch.float32, device=dev)
    r = torch.empty(K, 4, dtype=torch.float32, device=dev)
    check(lib.plane_init_points(_ptr(points.contiguous()), _ptr(normals.contiguous()), int(points.shape[0]),
                                _ptr(sel), K, float(r_min), _ptr(c), _ptr(q), _ptr(r), _stream()))
    return c, q, r


def init_from_depth(depth, normal, cams, K: int = 2000, stride: int = 4, voxel: float = 0.02, seed: int = 0,
                    r_min: float = 1e-4):
    """Sec. 3.1: K planes on distinct random fused points (all of them when
    fewer), radii half the nearest-neighbour distance, rotation from the
    normal."""
    pts, nrm, n = depth_points(depth, normal, cams, stride, voxel)
    if n < 2:
        raise ValueError(f"init_from_depth: {n} fused points, need at least 2")
    sel = np.random.default_rng(seed).choice(n, min(K, n), replace=False).astype(np.int32)
    return init_from_points(pts, nrm, sel, r_min)


def sphere_directions(K: int, seed: int = 0) -> np.ndarray:
    """K seeded directions, uniform on the sphere once normalised."""
    return np.random.default_rng(seed).normal(size=(K, 3)).astype(np.float32)


def init_sphere(points, K: int = 2000, seed: int = 0, radius: float = 0.05, dirs=None):
    """Sec. 4.3: K planes of radius `radius` on the bounding sphere of the
    points, at seeded uniformly random directions (or `dirs` [K,3]), facing
    its center."""
    lib = _lib.load()
    dev = points.device
    if dirs is None:
        dirs = sphere_directions(K, seed)
    dirs = torch.as_tensor(np.asarray(dirs, np.float32) if not torch.is_tensor(dirs) else dirs,
                           dtype=torch.float32).to(dev).contiguous()
    K = int(dirs.shape[0])
    ws = torch.empty(8, dtype=torch.float64, device=dev)
    c = torch.empty(K, 3, dtype=torch.float32, device=dev)
    q = torch.empty(K, 4, dtype=torch.float32, device=dev)
    r = torch.empty(K, 4, dtype=torch.float32, device=dev)
    check(lib.plane_init_sphere(_ptr(points.contiguous()), int(points.shape[0]), _ptr(dirs), K, float(radius),
                                _ptr(c), _ptr(q), _ptr(r), _ptr(ws), _stream()))
    return c, q, r


def merge_planes(center, quat, scene_center=None, angle_deg: float = 25.0, offset: float = 0.001):
    """Plane instances (plane_merge): int32 labels [K] (smallest plane index
    of each instance) and the number of instances.  scene_center: [3]
    (device tensor or sequence); by default the middle of the box of the
    plane centers."""
    import math
    lib = _lib.load()
    dev = center.device
    center = center.contiguous().float()
    quat = quat.contiguous().float()
    K = int(center.shape[0])
    if scene_center is None:
        scene_center = 0.5 * (center.min(dim=0).values.double() + center.max(dim=0).values.double())
    sc = torch.as_tensor(scene_center, dtype=torch.float32).to(dev).contiguous()
    nbytes = int(lib.plane_merge_ws_bytes(K))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    label = torch.empty(K, dtype=torch.int32, device=dev)
    n_out = torch.empty(1, dtype=torch.int32, device=dev)
    check(lib.plane_merge(_ptr(center), _ptr(quat), K, _ptr(sc), math.cos(math.radians(angle_deg)), float(offset),
                          _ptr(label), _ptr(n_out), _ptr(ws), nbytes, _stream()))
    return label, int(n_out.item())
