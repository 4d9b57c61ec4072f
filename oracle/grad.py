"""Reverse-mode gradient of the rendered maps (oracle).  TEST INFRASTRUCTURE ONLY.

The gradient is plain torch autograd of the float64 forward definition in
render.py; nothing about the adjoint is written by hand here.  Given upstream
gradients gD = dL/dD and gN = dL/dN (any source), the returned gradient is
that of sum_r gD(r) D(r) + gN(r) . N(r) with respect to center, quat, radii.

per_pixel_abs_grad also returns, per parameter coordinate, the sum over
pixels of the absolute value of each pixel's contribution.  It is obtained by
giving every pixel its own copy of the parameters, so one backward pass
yields the per-pixel Jacobian rows.  The GPU's float32 sums over pixels are
compared against this scale where the pixel contributions cancel.

weight_path_magnitude is the matching scale for cancellation inside one
pixel.  The adjoint of the front-to-back composite (Eq. 11-13) with respect
to a hit's weight is dL/dw_j = T_j (g . c_j - g . S_{j+1}), c_j the hit's
depth or normal and S_{j+1} the composite of what lies behind it; where a
hit sits just in front of a similar one the two terms nearly cancel, and a
float32 evaluation is off by a few roundoffs of the terms, not of their
difference.  Per coordinate it returns the sum over pixels and hits of
|dw_j/dtheta| T_j (|g_D| (|t_j| + A_{j+1}) + sum_c |g_N,c| (|n_j,c| + A_{j+1,c})),
with A the composite of |t| and |n| behind the hit (the same recurrence
with every value replaced by its magnitude).
"""

from __future__ import annotations

import numpy as np
import torch

from .render import OracleParams, _pairs, _t, order_key, render_pixels

F64 = torch.float64


def _upstream(cam, gD, gN):
    P = cam.width * cam.height
    gD = _t(gD).reshape(P)
    gN = _t(gN).reshape(3, P).T
    return gD, gN


def render_backward(center, quat, radii, cam, lam, gD, gN, prm: OracleParams = OracleParams(), pix=None):
    """(g_center [K,3], g_quat [K,4], g_radii [K,4]) in float64."""
    c = _t(center).clone().requires_grad_(True)
    q = _t(quat).clone().requires_grad_(True)
    r = _t(radii).clone().requires_grad_(True)
    gD, gN = _upstream(cam, gD, gN)
    if pix is None:
        pix = torch.arange(cam.width * cam.height)
    pix = torch.as_tensor(pix, dtype=torch.int64)
    D, N, _ = render_pixels(c, q, r, cam, lam, pix, prm)
    s = (gD[pix] * D).sum() + (gN[pix] * N).sum()
    s.backward()
    return c.grad.detach(), q.grad.detach(), r.grad.detach()


def per_pixel_abs_grad(center, quat, radii, cam, lam, gD, gN, prm: OracleParams = OracleParams(),
                       chunk: int = 2048, pix=None):
    """(grad, abs_sum) for each of center, quat, radii: grad is the plain
    gradient, abs_sum the per-coordinate sum over pixels of |contribution|.
    pix: the pixels to sum over (flat indices; all by default), for upstream
    gradients that vanish elsewhere."""
    center, quat, radii = _t(center), _t(quat), _t(radii)
    gD, gN = _upstream(cam, gD, gN)
    P = cam.width * cam.height
    K = center.shape[0]
    allpix = torch.arange(P) if pix is None else torch.as_tensor(np.asarray(pix), dtype=torch.int64)
    grads = [torch.zeros(K, 3, dtype=F64), torch.zeros(K, 4, dtype=F64), torch.zeros(K, 4, dtype=F64)]
    abss = [torch.zeros(K, 3, dtype=F64), torch.zeros(K, 4, dtype=F64), torch.zeros(K, 4, dtype=F64)]
    for s in range(0, allpix.numel(), chunk):
        pix = allpix[s:s + chunk]
        n = pix.numel()
        cc = center[None].expand(n, K, 3).clone().requires_grad_(True)
        qq = quat[None].expand(n, K, 4).clone().requires_grad_(True)
        rr = radii[None].expand(n, K, 4).clone().requires_grad_(True)
        D, N, _ = render_pixels(cc, qq, rr, cam, lam, pix, prm, chunk=n)
        tot = (gD[pix] * D).sum() + (gN[pix] * N).sum()
        tot.backward()
        for i, leaf in enumerate((cc, qq, rr)):
            grads[i] += leaf.grad.sum(0)
            abss[i] += leaf.grad.abs().sum(0)
    return grads, abss


def weight_path_magnitude(center, quat, radii, cam, lam, gD, gN, prm: OracleParams = OracleParams(),
                          chunk: int = 2048, pix=None):
    """Per-coordinate magnitude of the weight path of the gradient (module
    docstring), as [K,3], [K,4], [K,4] float64 tensors."""
    center, quat, radii = _t(center), _t(quat), _t(radii)
    gD, gN = _upstream(cam, gD, gN)
    P = cam.width * cam.height
    K = center.shape[0]
    allpix = torch.arange(P) if pix is None else torch.as_tensor(np.asarray(pix), dtype=torch.int64)
    mags = [torch.zeros(K, 3, dtype=F64), torch.zeros(K, 4, dtype=F64), torch.zeros(K, 4, dtype=F64)]
    for s in range(0, allpix.numel(), chunk):
        pc = allpix[s:s + chunk]
        n = pc.numel()
        cc = center[None].expand(n, K, 3).clone().requires_grad_(True)
        qq = quat[None].expand(n, K, 4).clone().requires_grad_(True)
        rr = radii[None].expand(n, K, 4).clone().requires_grad_(True)
        q = _pairs(cc, qq, rr, cam, lam, pc, prm)
        # the hits each pixel composites, near to far (the forward's selection)
        key = torch.where(q["keep"], order_key(q["t"].detach(), prm), torch.full_like(q["t"], np.inf))
        sel = torch.sort(key, dim=1, stable=True).indices[:, :min(prm.M, K)]
        ks = q["keep"].gather(1, sel)
        w_s = torch.where(ks, q["w"].gather(1, sel), torch.zeros((), dtype=F64))
        with torch.no_grad():
            wv = w_s.detach()
            t_abs = torch.where(ks, q["t"].gather(1, sel), torch.zeros((), dtype=F64)).abs()
            n_abs = q["n"].gather(1, sel[..., None].expand(n, sel.shape[1], 3)).abs() * ks[..., None]
            J = sel.shape[1]
            T = torch.ones(n, J, dtype=F64)
            for j in range(1, J):
                T[:, j] = T[:, j - 1] * (1.0 - wv[:, j - 1])
            A_d = torch.zeros(n, J + 1, dtype=F64)
            A_n = torch.zeros(n, J + 1, 3, dtype=F64)
            for j in range(J - 1, -1, -1):
                A_d[:, j] = wv[:, j] * t_abs[:, j] + (1.0 - wv[:, j]) * A_d[:, j + 1]
                A_n[:, j] = wv[:, j, None] * n_abs[:, j] + (1.0 - wv[:, j, None]) * A_n[:, j + 1]
            gd = gD[pc].abs()[:, None]
            gn = gN[pc].abs()[:, None, :]
            M = T * (gd * (t_abs + A_d[:, 1:]) + (gn * (n_abs + A_n[:, 1:])).sum(-1))
        # each plane appears at most once in a pixel's list, so the gradient of
        # sum_j M_j w_j per pixel copy is M_j dw_j/dtheta with no cross terms
        (M * w_s).sum().backward()
        for i, leaf in enumerate((cc, qq, rr)):
            mags[i] += leaf.grad.abs().sum(0)
    return mags
