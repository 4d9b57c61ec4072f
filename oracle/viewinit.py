"""Geometry of the learned initializer's per-view form (oracle).  TEST
INFRASTRUCTURE ONLY: see the package docstring.

Not part of the paper (its Sec. 3.1 initialises planes from monocular depth);
the readings are ours, stated where each function is defined:

* the network's input of a view: candidate pixels (drawn by the caller) taken
  in order, the first N with depth > 0 kept, each back-projected through the
  pixel center to the camera frame with its depth scaled by (1 + sigma eps),
  eps a standard normal draw of the caller; fewer than N valid candidates
  repeat in order;
* a proposal (12 numbers) decodes as the set loss decodes it: center; unit
  quaternion of (o3 + 1, o4, o5, o6); radii softplus + 0.01; confidence
  sigmoid of the logit; it maps to the world by x_w = R^T (x_c - t) and the
  rotation R^T R(q), written as a unit quaternion by Shepperd's method;
* an initial plane takes the supporting plane of its nearest confident
  proposal (the set loss's distance, smallest index on ties) when that
  distance is at most d_max: normal turned to the initial side, center moved
  onto the plane along it, frame turned by the smallest rotation between the
  normals (Rodrigues' formula), radii kept.

Everything is float64 with one rounding per operation, in the order the
formulas are written, so that the choices (kept pixels, nearest proposal)
are the same as the kernels'.
"""

from __future__ import annotations

import math

import numpy as np

W_N = 0.25
W_E = 0.25
R_MIN = 0.01


def view_points(depth, cam, cand, eps, N: int, sigma: float):
    """depth [H, W]; cand, eps [n_cand]; returns X [N, 3] (float32) and the
    number of kept points."""
    H, W = depth.shape
    D = np.asarray(depth, np.float32).reshape(-1)
    pts = []
    for p, e in zip(np.asarray(cand).tolist(), np.asarray(eps, np.float32).tolist()):
        if len(pts) == N:
            break
        if not (0 <= p < H * W) or not (D[p] > 0):
            continue
        u = float(p % W) + 0.5
        v = float(p // W) + 0.5
        z = float(D[p]) * (1.0 + float(np.float32(sigma)) * float(e))
        dx = (u - float(cam.cx)) / float(cam.fx)
        dy = (v - float(cam.cy)) / float(cam.fy)
        pts.append((dx * z, dy * z, z))
    kept = len(pts)
    X = np.zeros((N, 3), np.float64)
    if kept:
        for i in range(N):
            X[i] = pts[i % kept]
    return X.astype(np.float32), kept


def quat_matrix(q):
    """Hamilton rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = q
    return np.array([[1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)],
                     [2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)],
                     [2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)]])


def matrix_quat(m):
    """Unit quaternion of a rotation matrix by Shepperd's method (the branch
    of the largest of the trace and the diagonal)."""
    tr = m[0, 0] + m[1, 1] + m[2, 2]
    if tr > 0.0:
        s = math.sqrt(tr + 1.0) * 2.0
        q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
    elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
        s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2.0
        q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
    elif m[1, 1] > m[2, 2]:
        s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2.0
        q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2.0
        q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
    n = math.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
    return [x / n for x in q]


def _softplus(a: float) -> float:
    return a if a > 30.0 else math.log1p(math.exp(a))


def proposals_to_world(out, cams_of_views, P: int):
    """out [B, 12 P] (float32) and one camera per view -> center [B P, 3],
    quat [B P, 4], radii [B P, 4], conf [B P] (float32)."""
    out = np.asarray(out, np.float32).reshape(-1, P, 12)
    B = out.shape[0]
    c_out = np.zeros((B * P, 3))
    q_out = np.zeros((B * P, 4))
    r_out = np.zeros((B * P, 4))
    f_out = np.zeros(B * P)
    for b in range(B):
        cam = cams_of_views[b]
        R = np.asarray(cam.R, np.float32).astype(np.float64)
        t = np.asarray(cam.t, np.float32).astype(np.float64)
        for j in range(P):
            o = [float(x) for x in out[b, j]]
            i = b * P + j
            c = [o[0] - t[0], o[1] - t[1], o[2] - t[2]]
            w, x, y, z = o[3] + 1.0, o[4], o[5], o[6]
            qn = math.sqrt(w * w + x * x + y * y + z * z)
            Rc = quat_matrix((w / qn, x / qn, y / qn, z / qn))
            Rw = np.zeros((3, 3))
            for r in range(3):
                for k in range(3):
                    Rw[r, k] = (R[0, r] * Rc[0, k] + R[1, r] * Rc[1, k]) + R[2, r] * Rc[2, k]
            for r in range(3):
                c_out[i, r] = (R[0, r] * c[0] + R[1, r] * c[1]) + R[2, r] * c[2]
            q_out[i] = matrix_quat(Rw)
            r_out[i] = [_softplus(o[7 + k]) + R_MIN for k in range(4)]
            f_out[i] = 1.0 / (1.0 + math.exp(-o[11]))
    f32 = lambda a: a.astype(np.float32)   # noqa: E731
    return f32(c_out), f32(q_out), f32(r_out), f32(f_out)


def _desc(c, q, r):
    w, x, y, z = (float(v) for v in q)
    qn = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / qn, x / qn, y / qn, z / qn
    n = (2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y))
    ex = 0.5 * (float(r[0]) + float(r[1]))
    ey = 0.5 * (float(r[2]) + float(r[3]))
    return [float(v) for v in c], n, max(ex, ey), min(ex, ey), (w, x, y, z)


def refine_planes(center, quat, radii, pc, pq, pr, pconf, conf_min: float, d_max: float):
    """Refined centers [K, 3] and quaternions [K, 4] (float32) and the
    matched proposal of each plane (-1: unchanged)."""
    K = np.asarray(center).shape[0]
    Q = np.asarray(pc).shape[0]
    props = [_desc(pc[j], pq[j], pr[j]) for j in range(Q)]
    confs = [float(x) for x in np.asarray(pconf, np.float32)]
    oc = np.asarray(center, np.float32).copy()
    oq = np.asarray(quat, np.float32).copy()
    match = np.full(K, -1, np.int64)
    for k in range(K):
        ck, nk, ak, bk, qk = _desc(center[k], quat[k], radii[k])
        best, bi = 0.0, -1
        for j, (cp, np_, ap, bp, _) in enumerate(props):
            if not (confs[j] >= conf_min):
                continue
            d0, d1, d2 = cp[0] - ck[0], cp[1] - ck[1], cp[2] - ck[2]
            dot = (np_[0] * nk[0] + np_[1] * nk[1]) + np_[2] * nk[2]
            da, db = ap - ak, bp - bk
            d = ((d0 * d0 + d1 * d1) + d2 * d2) + W_N * (1.0 - dot * dot) + W_E * (da * da + db * db)
            if bi < 0 or d < best:
                best, bi = d, j
        if bi < 0 or not (best <= d_max):
            continue
        match[k] = bi
        cp, np_, _, _, _ = props[bi]
        s = -1.0 if ((np_[0] * nk[0] + np_[1] * nk[1]) + np_[2] * nk[2]) < 0.0 else 1.0
        n = (s * np_[0], s * np_[1], s * np_[2])
        off = ((ck[0] - cp[0]) * n[0] + (ck[1] - cp[1]) * n[1]) + (ck[2] - cp[2]) * n[2]
        oc[k] = [ck[i] - off * n[i] for i in range(3)]
        R0 = quat_matrix(qk)
        v = (nk[1] * n[2] - nk[2] * n[1], nk[2] * n[0] - nk[0] * n[2], nk[0] * n[1] - nk[1] * n[0])
        sn = math.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
        cs = (nk[0] * n[0] + nk[1] * n[1]) + nk[2] * n[2]
        A = np.eye(3)
        if sn >= 1e-12:
            u = (v[0] / sn, v[1] / sn, v[2] / sn)
            ang = math.atan2(sn, cs)
            si, c1 = math.sin(ang), 1.0 - math.cos(ang)
            Kx = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
            for r in range(3):
                for cc in range(3):
                    kk = (Kx[r, 0] * Kx[0, cc] + Kx[r, 1] * Kx[1, cc]) + Kx[r, 2] * Kx[2, cc]
                    A[r, cc] = (A[r, cc] + si * Kx[r, cc]) + c1 * kk
        R1 = np.zeros((3, 3))
        for r in range(3):
            for cc in range(3):
                R1[r, cc] = (A[r, 0] * R0[0, cc] + A[r, 1] * R0[1, cc]) + A[r, 2] * R0[2, cc]
        oq[k] = matrix_quat(R1)
    return oc, oq, match
