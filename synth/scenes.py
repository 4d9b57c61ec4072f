"""Seeded scene generators: random rectangles, pinhole cameras, synthetic rooms.

Conventions shared by every consumer of these inputs:

* a plane is a rectangle with center p (3), unit quaternion q = (w, x, y, z)
  (Hamilton) and four radii (x+, x-, y+, y-), the double radii of Eq. 1;
  its local X / Y axes and normal are the columns of R(q) (Eq. 2-3);
* a camera maps world to camera coordinates as x_c = R x_w + t, with OpenCV
  axes (x right, y down, z forward) and a pinhole (fx, fy, cx, cy); the
  principal point of every generated camera is (W/2, H/2).

All outputs are float32 numpy arrays so that every consumer starts from the
same bits.  Random draws use numpy.random.default_rng(seed).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class PlaneSet:
    center: np.ndarray  # [K, 3] float32
    quat: np.ndarray    # [K, 4] float32, (w, x, y, z)
    radii: np.ndarray   # [K, 4] float32, (x+, x-, y+, y-)

    @property
    def K(self) -> int:
        return int(self.center.shape[0])

    def copy(self) -> "PlaneSet":
        return PlaneSet(self.center.copy(), self.quat.copy(), self.radii.copy())

    def subset(self, idx) -> "PlaneSet":
        return PlaneSet(self.center[idx].copy(), self.quat[idx].copy(), self.radii[idx].copy())


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))  # world->camera
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))

    def __post_init__(self):
        # every consumer (float64 oracle, float32 kernels) sees the same values
        self.fx, self.fy, self.cx, self.cy = (float(np.float32(v)) for v in (self.fx, self.fy, self.cx, self.cy))
        self.R = np.asarray(self.R, np.float32).reshape(3, 3)
        self.t = np.asarray(self.t, np.float32).reshape(3)

    def center(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


# ----------------------------------------------------------------------------
# quaternion helpers used to *generate* inputs (rotation noise, room layout)
# ----------------------------------------------------------------------------

def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a * b for arrays of shape [..., 4] (w, x, y, z)."""
    aw, ax, ay, az = np.moveaxis(np.asarray(a, np.float64), -1, 0)
    bw, bx, by, bz = np.moveaxis(np.asarray(b, np.float64), -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quat_from_matrix(Rm: np.ndarray) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of a proper rotation matrix (Shepperd)."""
    Rm = np.asarray(Rm, np.float64)
    tr = Rm[0, 0] + Rm[1, 1] + Rm[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (Rm[2, 1] - Rm[1, 2]) / s, (Rm[0, 2] - Rm[2, 0]) / s, (Rm[1, 0] - Rm[0, 1]) / s]
    elif Rm[0, 0] > Rm[1, 1] and Rm[0, 0] > Rm[2, 2]:
        s = math.sqrt(1.0 + Rm[0, 0] - Rm[1, 1] - Rm[2, 2]) * 2
        q = [(Rm[2, 1] - Rm[1, 2]) / s, 0.25 * s, (Rm[0, 1] + Rm[1, 0]) / s, (Rm[0, 2] + Rm[2, 0]) / s]
    elif Rm[1, 1] > Rm[2, 2]:
        s = math.sqrt(1.0 + Rm[1, 1] - Rm[0, 0] - Rm[2, 2]) * 2
        q = [(Rm[0, 2] - Rm[2, 0]) / s, (Rm[0, 1] + Rm[1, 0]) / s, 0.25 * s, (Rm[1, 2] + Rm[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + Rm[2, 2] - Rm[0, 0] - Rm[1, 1]) * 2
        q = [(Rm[1, 0] - Rm[0, 1]) / s, (Rm[0, 2] + Rm[2, 0]) / s, (Rm[1, 2] + Rm[2, 1]) / s, 0.25 * s]
    q = np.asarray(q)
    return q / np.linalg.norm(q)


# ----------------------------------------------------------------------------
# random rectangles (the tiny / differentiation-check workloads)
# ----------------------------------------------------------------------------

def random_planes(K: int, seed: int = 0, independent_radii: bool = False,
                  center_range: float = 1.0, extent_range=(0.05, 0.4)) -> PlaneSet:
    """K rectangles: centers U[-c, c]^3, q = normalise(N(0, I4)), half-extents U[lo, hi].

    With independent_radii the four radii are drawn independently, otherwise
    r^{x+} = r^{x-} = h_x and r^{y+} = r^{y-} = h_y.
    """
    rng = np.random.default_rng(seed)
    center = rng.uniform(-center_range, center_range, size=(K, 3))
    q = rng.normal(size=(K, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    lo, hi = extent_range
    if independent_radii:
        radii = rng.uniform(lo, hi, size=(K, 4))
    else:
        hx = rng.uniform(lo, hi, size=K)
        hy = rng.uniform(lo, hi, size=K)
        radii = np.stack([hx, hx, hy, hy], axis=1)
    return PlaneSet(center.astype(np.float32), q.astype(np.float32), radii.astype(np.float32))


def perturb_planes(ps: PlaneSet, seed: int, center_sigma: float, rot_sigma_deg: float,
                   extent_scale=None) -> PlaneSet:
    """Noisy copy: center + N(0, s^2); rotation by a uniform axis and an angle
    ~ N(0, rot_sigma^2), left-multiplied; optional per-radius scale U[lo, hi]."""
    rng = np.random.default_rng(seed)
    K = ps.K
    center = ps.center.astype(np.float64) + rng.normal(scale=center_sigma, size=(K, 3))
    axis = rng.normal(size=(K, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.normal(scale=math.radians(rot_sigma_deg), size=K)
    qn = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * axis], axis=1)
    q = quat_mul(qn, ps.quat.astype(np.float64))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    radii = ps.radii.astype(np.float64)
    if extent_scale is not None:
        lo, hi = extent_scale
        radii = radii * rng.uniform(lo, hi, size=(K, 4))
    return PlaneSet(center.astype(np.float32), q.astype(np.float32), radii.astype(np.float32))


def tiny_camera(width: int = 128, height: int = 96, f: float = 100.0) -> Camera:
    """Camera at (0, 0, -3) looking along +z (R = I, t = (0, 0, 3))."""
    return Camera(width, height, f, f, width / 2.0, height / 2.0,
                  np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 3.0], np.float32))


def scaled_camera(cam: Camera, width: int, height: int, f: float) -> Camera:
    return Camera(width, height, f, f, width / 2.0, height / 2.0, cam.R.copy(), cam.t.copy())


def degenerate_planes(seed: int = 11, n_random: int = 24) -> PlaneSet:
    """Planes in awkward positions for the tiny camera (center (0, 0, -3),
    looking along +z), followed by `n_random` random planes:
      0  a floor at y = 0.3 whose local Y axis runs along -z, reaching 2 m
         behind and 2 m in front of the camera;
      1  the plane x = 0, which contains the camera center;
      2  a plane at x = 0.15 whose normal is 80 degrees off the view axis;
      3  a small fronto-parallel plane 5 cm in front of the camera;
      4  a fronto-parallel plane 5 mm in front of the camera;
      5  a plane 1 m behind the camera;
      6  an oblique plane through a point 1 cm in front of the camera."""
    s = math.sqrt(0.5)
    c40, s40 = math.cos(math.radians(40.0)), math.sin(math.radians(40.0))
    quat = [[s, -s, 0, 0], [s, 0, s, 0], [c40, 0, s40, 0], [1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0],
            [0.95, 0.31, 0, 0]]
    center = [[0, 0.3, -3], [0, 0, 0], [0.15, 0, 0], [0.02, -0.01, -2.95], [0, 0, -2.995], [0, 0, -4],
              [0, 0, -2.99]]
    radii = [[2, 2, 2, 2], [1, 1, 1, 1], [0.5, 0.5, 1.0, 1.0], [0.01, 0.02, 0.015, 0.01], [0.3, 0.3, 0.3, 0.3],
             [2, 2, 2, 2], [1.0, 0.8, 1.0, 0.6]]
    base = random_planes(n_random, seed=seed, independent_radii=True)
    return PlaneSet(np.concatenate([np.array(center, np.float32), base.center]),
                    np.concatenate([np.array(quat, np.float32), base.quat]),
                    np.concatenate([np.array(radii, np.float32), base.radii]))


def stacked_planes(K: int, seed: int = 0) -> PlaneSet:
    """K small, nearly fronto-parallel rectangles stacked in depth in front of
    the tiny camera: centers (U[-0.2, 0.2], U[-0.2, 0.2], U[0, 5]), quaternions
    (1, N(0, 0.1^2) x 3), radii U[0.005, 0.02].  Seen through an 8x8 image at
    lambda(0) every one of them reaches every pixel through its fringe, so one
    tile lists all K."""
    rng = np.random.default_rng(seed)
    center = np.stack([rng.uniform(-0.2, 0.2, K), rng.uniform(-0.2, 0.2, K), rng.uniform(0.0, 5.0, K)], 1)
    quat = np.concatenate([np.ones((K, 1)), rng.normal(0.0, 0.1, (K, 3))], 1)
    radii = rng.uniform(0.005, 0.02, (K, 4))
    return PlaneSet(center.astype(np.float32), quat.astype(np.float32), radii.astype(np.float32))


# ----------------------------------------------------------------------------
# synthetic indoor room: box room + furniture boxes, faces split into cells
# ----------------------------------------------------------------------------

def _room_faces(rng, room, n_boxes):
    """List of rectangular faces (center, u, v, n, extent_u, extent_v) with
    u x v = n; room faces point inward, box faces outward, box bottoms omitted."""
    X, Y, Z = room
    e = np.eye(3)
    faces = []

    def add(c, u, n, eu, ev):
        u = np.asarray(u, np.float64)
        n = np.asarray(n, np.float64)
        v = np.cross(n, u)
        faces.append((np.asarray(c, np.float64), u, v, n, float(eu), float(ev)))

    add([X / 2, Y / 2, 0.0], e[0], e[2], X, Y)          # floor
    add([X / 2, Y / 2, Z], e[0], -e[2], X, Y)           # ceiling
    add([0.0, Y / 2, Z / 2], e[1], e[0], Y, Z)          # wall x = 0
    add([X, Y / 2, Z / 2], e[1], -e[0], Y, Z)           # wall x = X
    add([X / 2, 0.0, Z / 2], e[0], e[1], X, Z)          # wall y = 0
    add([X / 2, Y, Z / 2], e[0], -e[1], X, Z)           # wall y = Y
    boxes = []
    for _ in range(n_boxes):
        a, b = rng.uniform(0.3, 1.5, size=2)
        h = rng.uniform(0.3, 1.2)
        cx = rng.uniform(a / 2, X - a / 2)
        cy = rng.uniform(b / 2, Y - b / 2)
        boxes.append((cx, cy, a, b, h))
        add([cx, cy, h], e[0], e[2], a, b)                      # top
        add([cx + a / 2, cy, h / 2], e[1], e[0], b, h)          # +x side
        add([cx - a / 2, cy, h / 2], e[1], -e[0], b, h)         # -x side
        add([cx, cy + b / 2, h / 2], e[0], e[1], a, h)          # +y side
        add([cx, cy - b / 2, h / 2], e[0], -e[1], a, h)         # -y side
    return faces, boxes


def _cells(faces, s):
    out = []
    for (c, u, v, n, eu, ev) in faces:
        nu = max(1, int(math.ceil(eu / s - 1e-9)))
        nv = max(1, int(math.ceil(ev / s - 1e-9)))
        du, dv = eu / nu, ev / nv
        for i in range(nu):
            for j in range(nv):
                cc = c + ((i + 0.5) * du - eu / 2) * u + ((j + 0.5) * dv - ev / 2) * v
                out.append((cc, u, v, n, du / 2, dv / 2))
    return out


def room_planes(seed: int = 0, target_K: int = 2000, room=(6.0, 5.0, 3.0), n_boxes: int = 40):
    """Ground-truth rectangles of a synthetic room, about target_K of them.

    Returns (PlaneSet, info) where info holds the boxes and the cell size s
    chosen by bisection so that the face grid gives about target_K cells."""
    rng = np.random.default_rng(seed)
    faces, boxes = _room_faces(rng, room, n_boxes)
    lo, hi = 0.01, 10.0
    for _ in range(60):
        mid = math.sqrt(lo * hi)
        if len(_cells(faces, mid)) > target_K:
            lo = mid
        else:
            hi = mid
    s = hi
    cells = _cells(faces, s)
    K = len(cells)
    center = np.zeros((K, 3))
    quat = np.zeros((K, 4))
    radii = np.zeros((K, 4))
    for k, (cc, u, v, n, hu, hv) in enumerate(cells):
        center[k] = cc
        quat[k] = quat_from_matrix(np.stack([u, v, n], axis=1))
        radii[k] = [hu, hu, hv, hv]
    ps = PlaneSet(center.astype(np.float32), quat.astype(np.float32), radii.astype(np.float32))
    return ps, {"boxes": boxes, "cell": s, "room": room}


def _look_camera(pos, yaw, pitch, width, height, f) -> Camera:
    fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    Rm = np.stack([right, down, fwd], axis=0)
    t = -Rm @ np.asarray(pos, np.float64)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, Rm.astype(np.float32), t.astype(np.float32))


def room_trajectory(seed: int, n_views: int, info: dict, width: int = 640, height: int = 480,
                    f: float = 577.0, margin: float = 0.3, n_way: int = 8):
    """n_views cameras along a smooth random path inside the room.

    Waypoints lie in free space at height U[1.2, 1.8] m and at least `margin`
    from the walls; a Catmull-Rom spline joins them.  Yaw follows the path
    tangent (+- N(0, 20 deg)), pitch ~ U[-25, 10] deg, roll 0.  A camera over a
    box is lifted to at least `margin` above its top."""
    rng = np.random.default_rng(seed)
    X, Y, Z = info["room"]
    boxes = info["boxes"]
    way = np.stack([rng.uniform(margin, X - margin, n_way),
                    rng.uniform(margin, Y - margin, n_way),
                    rng.uniform(1.2, 1.8, n_way)], axis=1)
    P = np.concatenate([way[:1], way, way[-1:]], axis=0)
    pos, tan = [], []
    for i in range(n_views):
        s = i / max(1, n_views - 1) * (n_way - 1)
        k = min(int(s), n_way - 2)
        u = s - k
        p0, p1, p2, p3 = P[k], P[k + 1], P[k + 2], P[k + 3]
        pt = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                    + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
        dt = 0.5 * ((-p0 + p2) + 2 * (2 * p0 - 5 * p1 + 4 * p2 - p3) * u
                    + 3 * (-p0 + 3 * p1 - 3 * p2 + p3) * u * u)
        pt[0] = min(max(pt[0], margin), X - margin)
        pt[1] = min(max(pt[1], margin), Y - margin)
        zmin = 1.2
        for (bx, by, a, b, h) in boxes:
            if abs(pt[0] - bx) < a / 2 + margin and abs(pt[1] - by) < b / 2 + margin:
                zmin = max(zmin, h + margin)
        pt[2] = min(max(pt[2], zmin), Z - margin)
        pos.append(pt)
        tan.append(dt)
    cams = []
    for p, d in zip(pos, tan):
        yaw = math.atan2(d[1], d[0]) + rng.normal(scale=math.radians(20.0))
        pitch = math.radians(rng.uniform(-25.0, 10.0))
        cams.append(_look_camera(p, yaw, pitch, width, height, f))
    return cams


def room_init_planes(gt: PlaneSet, seed: int = 1) -> PlaneSet:
    """Noisy initialisation of a room fit: center sigma 0.1 m, rotation sigma
    10 deg, each radius scaled by U[0.7, 1.3]."""
    return perturb_planes(gt, seed, 0.1, 10.0, (0.7, 1.3))


def room_batch_specs(n_rooms: int, seed: int = 0, k_range=(200, 4000), view_range=(20, 100)):
    """Shapes of a batch of synthetic rooms: per room a seed, a plane count
    log-uniform in k_range, a view count uniform in view_range and, with
    probability 1/2 each, 320 x 240 (f = 288.5) or 640 x 480 (f = 577)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_rooms):
        K = int(round(math.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1])))))
        V = int(rng.integers(view_range[0], view_range[1] + 1))
        small = bool(rng.uniform() < 0.5)
        W, H, f = (320, 240, 288.5) if small else (640, 480, 577.0)
        out.append({"seed": seed + i, "K": K, "views": V, "width": W, "height": H, "f": f})
    return out


# ----------------------------------------------------------------------------
# random depth / normal maps (scene-initialisation checks)
# ----------------------------------------------------------------------------

def random_depth_maps(width: int, height: int, seed: int, bg_frac: float = 0.1):
    """Depth [H, W] and camera-frame normal [3, H, W] maps in the renderer's
    layout: per pixel a depth t ~ U[0.5, 4], a random unit normal n and a
    coverage w ~ U[0.3, 1] give D = w t and N = w n (a pixel partly covered by
    one plane); a fraction bg_frac of the pixels is background (D = 0)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.5, 4.0, size=(height, width))
    n = rng.normal(size=(3, height, width))
    n /= np.linalg.norm(n, axis=0, keepdims=True)
    w = rng.uniform(0.3, 1.0, size=(height, width))
    D = (w * t).astype(np.float32)
    N = (w[None] * n).astype(np.float32)
    D[rng.uniform(size=(height, width)) < bg_frac] = 0.0
    return D, N
