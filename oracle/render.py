"""Brute-force FP64 renderer of rectangular plane primitives (oracle).

TEST INFRASTRUCTURE ONLY: see the package docstring.

Every pixel's ray is intersected with every plane; nothing is tiled, culled
or reordered beyond what the method states.  Readings of points the paper
leaves open:

* Eq. 4 prints the numerator as "(p - o . n)"; it is read as (p - o) . n.
* the pinhole ray of pixel (i, j) passes through the pixel center
  (i + 1/2, j + 1/2); the direction has camera-frame z component 1, so the
  ray parameter t of Eq. 4 is the camera z-depth, which is the "depth" t_j of
  Eq. 11.
* Eq. 7-8 print 2*sigmoid(.), which exceeds 1 inside the rectangle.  Mode "A"
  (default) keeps the printed weight and clamps it at 1: a point inside the
  rectangle is opaque (the primitives are described as solid).  Mode "B"
  uses sigmoid(.) without the factor 2.
* Eq. 9's "otherwise" gives w_Y on a tie, Eq. 7's "otherwise" takes r^{x-}
  at P_X = 0.
* mode "G", the Gaussian splat function of Eq. 5 (the paper's comparison):
  the covariance is planar with standard deviations equal to the radii on
  the hit's side, w = exp(-((P_X / r_X)^2 + (P_Y / r_Y)^2) / 2); no lambda,
  never opaque; the filter keeps w >= tau.
* intersections with |d . n| <= 1e-12 |d| or depth t <= z_near are no hits.
* the filter keeps w >= tau; the survivors are ordered by depth, ties broken
  by the plane index, and the first M are composited.  The order is an
  integer decided by floating point, so OracleParams.order states the
  precision it is decided in: "f32" (default), the depth rounded to float32,
  the precision the kernels decide it in; "f64", the exact float64 depth.
  The two differ only inside runs of hits whose depths round to the same
  float32 value, and tests bound what that changes.
* the products with the camera rotation (ray directions, camera-frame
  normals) are written out as three-term sums, so every pixel's value comes
  from the same operations whichever batch of pixels or planes it is
  evaluated in: the tiled evaluation below equals the brute force bit for
  bit.
* the rendered normal is the plane normal in the camera frame, flipped to
  face the camera (two-sided); with two_sided=False it is R(q) e_z as is.
* a pixel with no surviving intersection renders depth 0 and normal 0.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64


@dataclass
class OracleParams:
    M: int = 30             # nearest intersections composited per ray (Sec. 3.2)
    tau: float = 1e-4       # weight filter threshold (Sec. 3.2)
    z_near: float = 0.01    # near clip in metres (not in the paper)
    weight_mode: str = "A"  # "A": min(1, 2 sigmoid(5 lambda a)); "B": sigmoid(5 lambda a);
    #                         "G": the Gaussian of Eq. 5 (the ablation's splat function)
    two_sided: bool = True
    order: str = "f32"      # precision the per-ray depth order is decided in: "f32" or "f64"


def lambda_at(ite: int) -> float:
    """Eq. 10: lambda = min(20 e^{-(1 - 0.001 ite)}, 300), ite counted from 0."""
    return min(20.0 * math.exp(-(1.0 - 0.001 * ite)), 300.0)


def gauss_bound(prm: OracleParams) -> float:
    """Q such that the Gaussian weight exp(-q/2) >= tau  <=>  q <= Q."""
    return 2.0 * math.log(1.0 / prm.tau)


def fringe_margin(lam: float, prm: OracleParams) -> float:
    """delta such that w >= tau  <=>  min(a_X, a_Y) >= -delta (closed form)."""
    if prm.weight_mode == "A":
        return math.log(2.0 / prm.tau - 1.0) / (5.0 * lam)
    return math.log(1.0 / prm.tau - 1.0) / (5.0 * lam)


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(F64)
    return torch.as_tensor(np.asarray(x), dtype=F64)


def quat_to_frame(q: torch.Tensor):
    """Eq. 2-3: v_x = R(q) e_x, v_y = R(q) e_y, n = R(q) e_z, with q normalised
    first and R the Hamilton rotation matrix of q = (w, x, y, z)."""
    qn = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = qn.unbind(-1)
    vx = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], dim=-1)
    vy = torch.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], dim=-1)
    n = torch.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)], dim=-1)
    return vx, vy, n


def camera_rays(cam, pix: torch.Tensor):
    """Origin o (world) and world directions d of the rays through the pixel
    centers of the flat pixel indices `pix` (row-major, index = j*W + i)."""
    Rcw = _t(cam.R)
    tcw = _t(cam.t)
    o = -(Rcw.T @ tcw)
    i = (pix % cam.width).to(F64)
    j = torch.div(pix, cam.width, rounding_mode="floor").to(F64)
    dc = torch.stack([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, torch.ones_like(i)], dim=-1)
    d = _rot_t(Rcw, dc)  # R^T d_c
    return o, d, Rcw


def _rot(Rm, v):
    """R v for vectors v [..., 3], each component a sum of three products in a fixed order."""
    return torch.stack([v[..., 0] * Rm[a, 0] + v[..., 1] * Rm[a, 1] + v[..., 2] * Rm[a, 2] for a in range(3)], -1)


def _rot_t(Rm, v):
    """R^T v for vectors v [..., 3], written out like _rot."""
    return torch.stack([v[..., 0] * Rm[0, a] + v[..., 1] * Rm[1, a] + v[..., 2] * Rm[2, a] for a in range(3)], -1)


def _pairs(center, quat, radii, cam, lam, pix, prm: OracleParams, cand=None):
    """All (pixel, plane) quantities of Sec. 3.2 for the pixels `pix`.

    Parameters have shape [K, .] (shared) or [P, K, .] (one copy per pixel, used
    to read per-pixel gradients).  Returns a dict of [P, K] tensors."""
    o, d, Rcw = camera_rays(cam, pix)
    if center.dim() == 2:
        center, quat, radii = center[None], quat[None], radii[None]
    vx, vy, n = quat_to_frame(quat)                       # [., K, 3]
    dd = d[:, None, :]                                    # [P, 1, 3]
    den = (dd * n).sum(-1)                                # d . n
    num = ((center - o) * n).sum(-1)                      # (p - o) . n   (Eq. 4, reading of the numerator)
    ok = den.abs() > 1e-12 * dd.norm(dim=-1)
    t = num / torch.where(ok, den, torch.ones_like(den))  # Eq. 4 ray parameter = z-depth
    valid = ok & (t > prm.z_near)
    x = o + t[..., None] * dd                             # intersection x^r_pi (Eq. 4)
    rel = x - center
    PX = (rel * vx).sum(-1)                               # Eq. 6
    PY = (rel * vy).sum(-1)
    rX = torch.where(PX > 0, radii[..., 0], radii[..., 1])  # Eq. 7: r^{x+} if P_X > 0 else r^{x-}
    rY = torch.where(PY > 0, radii[..., 2], radii[..., 3])  # Eq. 8
    zX = 5 * lam * (rX - PX.abs())
    zY = 5 * lam * (rY - PY.abs())
    # 1 - w is formed from the same argument by an identity instead of a
    # subtraction (1 - s(z) = s(-z), 1 - 2 s(z) = tanh(-z/2)), so the
    # transmittance behind a nearly opaque layer keeps its precision.
    if prm.weight_mode == "G":
        # Eq. 5: exp(-(x - p)^T Sigma^-1 (x - p) / 2) with the planar covariance
        # of standard deviations r along v_x and v_y (the radius on the hit's
        # side, as Eq. 7-8 pick it): q = (P_X / r_X)^2 + (P_Y / r_Y)^2
        qg = (PX / rX) ** 2 + (PY / rY) ** 2
        w = torch.exp(-qg / 2)
        omw = -torch.expm1(-qg / 2)
        keep = valid & (qg <= gauss_bound(prm))       # filter: exp(-q/2) >= tau
        if cand is not None:
            keep = keep & cand
        n_cam = _rot(Rcw, n)
        if prm.two_sided:
            n_cam = n_cam * (-torch.sign(num))[..., None]
        return dict(t=t, w=w, omw=omw, keep=keep, n=n_cam, PX=PX, PY=PY, rX=rX, rY=rY, num=num, den=den, a=qg)
    if prm.weight_mode == "A":
        wX, wY = 2 * torch.sigmoid(zX), 2 * torch.sigmoid(zY)
        oX, oY = torch.tanh(-zX / 2), torch.tanh(-zY / 2)
    else:
        wX, wY = torch.sigmoid(zX), torch.sigmoid(zY)
        oX, oY = torch.sigmoid(-zX), torch.sigmoid(-zY)
    w = torch.where(wX < wY, wX, wY)                      # Eq. 9
    omw = torch.where(wX < wY, oX, oY)
    if prm.weight_mode == "A":
        opaque = w >= 1
        w = torch.where(opaque, torch.ones_like(w), w)    # solid primitive: weight at most 1
        omw = torch.where(opaque, torch.zeros_like(omw), omw)
    keep = valid & (w >= prm.tau)                         # filter (Sec. 3.2)
    if cand is not None:
        keep = keep & cand
    # rendered normal: camera frame, facing the camera
    n_cam = _rot(Rcw, n)
    if prm.two_sided:
        s = -torch.sign(num)
        n_cam = n_cam * s[..., None]
    a = torch.where(wX < wY, rX - PX.abs(), rY - PY.abs())   # a* of the branch Eq. 9 takes
    return dict(t=t, w=w, omw=omw, keep=keep, n=n_cam, PX=PX, PY=PY, rX=rX, rY=rY, num=num, den=den, a=a)


def order_key(t: torch.Tensor, prm: OracleParams) -> torch.Tensor:
    """Sort key of a hit's depth in the precision the per-ray order is decided
    in (OracleParams.order)."""
    if prm.order == "f64":
        return t
    if prm.order != "f32":
        raise ValueError(f"order must be 'f32' or 'f64', not {prm.order!r}")
    return t.to(torch.float32).to(F64)


def _composite(q, prm: OracleParams):
    """Sort the kept intersections of each ray near to far, keep the first M,
    composite depth and normal front to back (Eq. 11-13)."""
    t, w, keep, n = q["t"], q["w"], q["keep"], q["n"]
    P, K = t.shape
    key = torch.where(keep, order_key(t.detach(), prm), torch.full_like(t, math.inf))
    order = torch.sort(key, dim=1, stable=True).indices   # stable: ties keep plane order
    Msel = min(prm.M, K)
    sel = order[:, :Msel]
    ks = keep.gather(1, sel)
    w_s = torch.where(ks, w.gather(1, sel), torch.zeros((), dtype=F64))
    o_s = torch.where(ks, q["omw"].gather(1, sel), torch.ones((), dtype=F64))   # 1 - w_s
    t_s = torch.where(ks, t.gather(1, sel), torch.zeros((), dtype=F64))
    if n.shape[0] == 1:
        n = n.expand(P, K, 3)
    n_s = n.gather(1, sel[..., None].expand(P, Msel, 3))
    T = torch.ones(P, dtype=F64)
    D = torch.zeros(P, dtype=F64)
    N = torch.zeros(P, 3, dtype=F64)
    cov = torch.zeros(P, dtype=F64)
    for j in range(Msel):
        Tw = T * w_s[:, j]
        D = D + Tw * t_s[:, j]                            # Eq. 11
        N = N + Tw[:, None] * n_s[:, j]                   # Eq. 12
        cov = cov + Tw
        T = T * o_s[:, j]                                 # Eq. 13, (1 - w_j)
    ids = torch.where(ks, sel, torch.full_like(sel, -1))
    # the hits a ray needs, without the cap of M: every kept hit up to and
    # including the first opaque one (all kept hits if none is opaque)
    kept_sorted = keep.gather(1, order)
    opq = kept_sorted & (w.gather(1, order) >= 1)
    first = torch.where(opq.any(1), opq.int().argmax(1) + 1, kept_sorted.sum(1))
    need = torch.minimum(first, kept_sorted.sum(1))
    return D, N, dict(count=ks.sum(1), coverage=cov.detach(), ids=ids, T=T.detach(), need=need)


def render_pixels(center, quat, radii, cam, lam, pix, prm: OracleParams = OracleParams(),
                  chunk: int = 4096, cand=None):
    """Depth [P] and camera-frame normal [P, 3] for flat pixel indices `pix`."""
    center, quat, radii = _t(center), _t(quat), _t(radii)
    pix = torch.as_tensor(np.asarray(pix), dtype=torch.int64)
    Ds, Ns, aux = [], [], []
    for s in range(0, pix.numel(), chunk):
        pc = pix[s:s + chunk]
        args = (center, quat, radii)
        if center.dim() == 3:   # per-pixel parameter copies
            args = tuple(a[s:s + chunk] for a in args)
        cc = None if cand is None else cand[s:s + chunk]
        q = _pairs(*args, cam, lam, pc, prm, cand=cc)
        D, N, a = _composite(q, prm)
        Ds.append(D)
        Ns.append(N)
        aux.append(a)
    D = torch.cat(Ds)
    N = torch.cat(Ns)
    merged = {k: torch.cat([a[k] for a in aux]) for k in aux[0]}
    return D, N, merged


def render(center, quat, radii, cam, lam, prm: OracleParams = OracleParams(), tiles=None, chunk: int = 4096):
    """Full image: depth [H, W] and normal [3, H, W] (camera frame).

    With tiles=(tw, th) the "tiled mode" is used: a plane is a candidate for
    the pixels of a tile only if its expanded footprint (footprint_tiles)
    touches the tile; the result must be identical to the untiled one."""
    W, H = cam.width, cam.height
    pix = torch.arange(W * H)
    cand = None
    if tiles is not None:
        tw, th = tiles
        rects = footprint_tiles(center, quat, radii, cam, lam, prm, tw, th)
        ti = (pix % W) // tw
        tj = (pix // W) // th
        r = torch.as_tensor(rects)
        cand = ((ti[:, None] >= r[None, :, 0]) & (ti[:, None] <= r[None, :, 2])
                & (tj[:, None] >= r[None, :, 1]) & (tj[:, None] <= r[None, :, 3]))
    D, N, aux = render_pixels(center, quat, radii, cam, lam, pix, prm, chunk, cand=cand)
    aux = {k: v.reshape(H, W, *v.shape[1:]) for k, v in aux.items()}
    return D.reshape(H, W), N.T.reshape(3, H, W), aux


def render_tiled(center, quat, radii, cam, lam, prm: OracleParams = OracleParams(), tiles=(16, 16),
                 max_pairs: int = 1 << 21):
    """The full image like render(), evaluating each pixel only against the
    planes whose grown footprint (footprint_tiles) touches its tile.

    Outside that footprint every plane has w < tau at every pixel of the tile
    (the footprint is the exact filter region, grown, clipped and projected),
    so it is never kept; each pixel gets its candidates as its own parameter
    copies, in ascending plane order, and every per-pixel value comes from
    the same operations as in the brute force.  The result equals render()
    bit for bit (a test pins it) at a fraction of the cost on large scenes.
    Returns depth [H, W], normal [3, H, W] and the aux maps of render(), with
    plane ids in the ids map."""
    center, quat, radii = _t(center), _t(quat), _t(radii)
    W, H = cam.width, cam.height
    tw, th = tiles
    rects = torch.as_tensor(footprint_tiles(center, quat, radii, cam, lam, prm, tw, th))
    ntx, nty = (W + tw - 1) // tw, (H + th - 1) // th
    tx = torch.arange(ntx * nty) % ntx
    ty = torch.arange(ntx * nty) // ntx
    cand = ((tx[:, None] >= rects[None, :, 0]) & (tx[:, None] <= rects[None, :, 2])
            & (ty[:, None] >= rects[None, :, 1]) & (ty[:, None] <= rects[None, :, 3]))   # [tiles, K]
    ncand = cand.sum(1)
    D = torch.zeros(H * W, dtype=F64)
    N = torch.zeros(H * W, 3, dtype=F64)
    Msel = min(prm.M, center.shape[0])
    aux = dict(count=torch.zeros(H * W, dtype=torch.int64), coverage=torch.zeros(H * W, dtype=F64),
               ids=torch.full((H * W, Msel), -1, dtype=torch.int64), T=torch.ones(H * W, dtype=F64),
               need=torch.zeros(H * W, dtype=torch.int64))
    order = torch.argsort(ncand, descending=True, stable=True)
    i = 0
    while i < order.numel():
        kc = max(1, int(ncand[order[i]]))
        # tiles with at most kc candidates, up to max_pairs pairs per evaluation
        n_t = max(1, max_pairs // (kc * tw * th))
        grp = order[i:i + n_t]
        i += grp.numel()
        if int(ncand[grp[0]]) == 0:
            continue   # no candidate: depth and normal 0, T = 1
        pix, idx, ok = [], [], []
        for t in grp.tolist():
            x0, y0 = int(tx[t]) * tw, int(ty[t]) * th
            ks = torch.nonzero(cand[t]).flatten()
            pad = torch.zeros(kc - ks.numel(), dtype=torch.int64)
            row = torch.cat([ks, pad])
            rok = torch.cat([torch.ones(ks.numel(), dtype=torch.bool), torch.zeros(pad.numel(), dtype=torch.bool)])
            for y in range(y0, min(y0 + th, H)):
                for x in range(x0, min(x0 + tw, W)):
                    pix.append(y * W + x)
            n_pix = (min(y0 + th, H) - y0) * (min(x0 + tw, W) - x0)
            idx.append(row[None].expand(n_pix, kc))
            ok.append(rok[None].expand(n_pix, kc))
        pix = torch.tensor(pix, dtype=torch.int64)
        idx = torch.cat(idx)
        ok = torch.cat(ok)
        d, n, a = render_pixels(center[idx], quat[idx], radii[idx], cam, lam, pix, prm, chunk=pix.numel(), cand=ok)
        D[pix] = d
        N[pix] = n
        aux["count"][pix] = a["count"]
        aux["coverage"][pix] = a["coverage"]
        aux["T"][pix] = a["T"]
        aux["need"][pix] = a["need"]
        ids = a["ids"]
        mapped = torch.where(ids >= 0, idx.gather(1, ids.clamp_min(0)), ids)
        aux["ids"][pix, :mapped.shape[1]] = mapped
    aux = {k: v.reshape(H, W, *v.shape[1:]) for k, v in aux.items()}
    return D.reshape(H, W), N.T.reshape(3, H, W), aux


def footprint_tiles(center, quat, radii, cam, lam, prm: OracleParams, tw: int, th: int):
    """Inclusive tile rectangle [tx0, ty0, tx1, ty1] per plane that contains
    every pixel whose ray can give w >= tau, or an empty rectangle.

    w >= tau holds exactly when -(r^{x-} + delta) <= P_X <= r^{x+} + delta and
    likewise for P_Y (delta = fringe_margin), i.e. inside the rectangle grown
    by delta.  The grown rectangle is clipped to z > z_near in the camera frame,
    projected, and its bounding box (plus one pixel) is converted to tiles."""
    center = _t(center).detach().numpy()
    vx, vy, _ = (a.detach().numpy() for a in quat_to_frame(_t(quat)))
    radii = _t(radii).detach().numpy()
    Rcw = np.asarray(cam.R, np.float64)
    tcw = np.asarray(cam.t, np.float64)
    gauss = prm.weight_mode == "G"
    dl = 0.0 if gauss else fringe_margin(lam, prm)
    ext = math.sqrt(gauss_bound(prm)) if gauss else 1.0   # the Gaussian's footprint: |P| <= r sqrt(Q)
    ntx = (cam.width + tw - 1) // tw
    nty = (cam.height + th - 1) // th
    out = np.zeros((center.shape[0], 4), np.int64)
    for k in range(center.shape[0]):
        xp, xm, yp, ym = radii[k] * ext + dl
        corners = [center[k] + a * vx[k] + b * vy[k] for a, b in ((xp, yp), (-xm, yp), (-xm, -ym), (xp, -ym))]
        cc = [Rcw @ c + tcw for c in corners]
        poly = []
        for a, b in zip(cc, cc[1:] + cc[:1]):       # clip the polygon to z >= z_near
            ina, inb = a[2] >= prm.z_near, b[2] >= prm.z_near
            if ina:
                poly.append(a)
            if ina != inb:
                s = (prm.z_near - a[2]) / (b[2] - a[2])
                poly.append(a + s * (b - a))
        if not poly:
            out[k] = [1, 1, 0, 0]
            continue
        us = [cam.fx * p[0] / p[2] + cam.cx for p in poly]
        vs = [cam.fy * p[1] / p[2] + cam.cy for p in poly]
        # pixel i is inside when u0 <= i + 1/2 <= u1; one pixel of guard
        i0 = max(0, math.floor(min(us) - 0.5) - 1)
        i1 = min(cam.width - 1, math.ceil(max(us) - 0.5) + 1)
        j0 = max(0, math.floor(min(vs) - 0.5) - 1)
        j1 = min(cam.height - 1, math.ceil(max(vs) - 0.5) + 1)
        if i0 > i1 or j0 > j1:
            out[k] = [1, 1, 0, 0]
            continue
        out[k] = [i0 // tw, j0 // th, min(i1 // tw, ntx - 1), min(j1 // th, nty - 1)]
    return out
