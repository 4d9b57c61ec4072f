"""Reverse-mode gradient of the rendered maps (oracle).  TEST INFRASTRUCTURE ONLY.

The gradient is plain torch autograd of the float64 forward definition in
render.py; nothing about the adjoint is written by hand here.  Given upstream
gradients gD = dL/dD and gN = dL/dN (any source), the returned gradient is
that of sum_r gD(r) D(r) + gN(r) . N(r) with respect to center, quat, radii.

per_pixel_abs_grad also returns, per parameter coordinate, the sum over
pixels of the absolute value of each pixel's contribution.  It is obtained by
giving every pixel its own copy of the parameters, so one backward pass
yields the per-pixel Jacobian rows.  The GPU's float32 sums over pixels are
judged against this scale where the pixel contributions cancel.
"""

from __future__ import annotations

import numpy as np
import torch

from .render import OracleParams, _t, render_pixels

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
