"""Learned plane initializer (oracle).  TEST INFRASTRUCTURE ONLY.

The paper initialises planes from monocular depth (Sec. 3.3, initialisation
paragraph).  The learned initializer is not in the paper; its network, loss
and matching are readings of this project, each marked below, and the GPU
kernels are checked against these definitions.

Network (per view; N back-projected depth points in the camera frame):
    pre1 = X W1 + b1,   h1 = bf16(relu(pre1))            3 -> 256
    pre2 = h1 W2 + b2,  h2 = bf16(relu(pre2))          256 -> 256
    pre3 = h2 W3 + b3,  h3 = bf16(relu(pre3))          256 -> 256
    g[c] = max_n h3[n, c],  arg[c] = smallest n attaining it
    out  = g Wh + bh                                   256 -> P * 12
Weights W*, Wh are bfloat16 values, biases float32, X float32.  Products are
exact in float64 and sums are float64; bf16(.) rounds to float32 and then to
bfloat16 (round to nearest even), which is what the kernels store.  In the
backward the rounding passes gradients through unchanged.

Proposal j of a view (out[j*12 : j*12+12] = o):
    center = o[0:3] (metres, camera frame)
    quat   = normalise(o[3:7] + (1, 0, 0, 0))
    radii  = softplus(o[7:11]) + 0.01
    conf   = o[11] (logit)
Plane descriptors used by the loss: the unit normal n (third column of R(q),
Eq. 2-3) and the half-extents a >= b of the rectangle, a = max(ex, ey),
b = min(ex, ey) with ex = (r_x+ + r_x-) / 2, ey = (r_y+ + r_y-) / 2.

Set loss of a view with targets t = 1..T (the fitted planes visible in the
view, camera frame):
    d(p, t) = |c_p - c_t|^2 + w_n (1 - (n_p . n_t)^2) + w_e ((a_p - a_t)^2 + (b_p - b_t)^2)
    L = (1/T) sum_t min_p d(p, t)  +  (1/P) sum_p BCE(conf_p, y_p)
y_p = 1 if p is the nearest proposal of some target (ties: smallest p),
else 0.  (n_p . n_t)^2 makes the loss blind to the normal's sign, which
the facing rule of the renderer fixes.  w_n = w_e = 0.25.
"""

from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64
P_PROPOSALS = 256
WIDTH = 256
OUT_PER = 12
W_N = 0.25
W_E = 0.25
R_MIN = 0.01


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round float64 values to float32, then to bfloat16 (nearest even)."""
    return x.to(torch.float32).to(torch.bfloat16).to(F64)


def _bf16_st(x: torch.Tensor) -> torch.Tensor:
    # forward: rounded value; backward: identity
    return x + (bf16(x.detach()) - x.detach())


def init_params(seed: int = 0, width: int = WIDTH, n_prop: int = P_PROPOSALS):
    """He-normal weights rounded to bfloat16, zero biases (float64 tensors)."""
    rng = np.random.default_rng(seed)

    def w(cin, cout, scale=None):
        s = np.sqrt(2.0 / cin) if scale is None else scale
        return bf16(torch.tensor(rng.normal(scale=s, size=(cin, cout)), dtype=F64))

    return {
        "W1": w(3, width), "b1": torch.zeros(width, dtype=F64),
        "W2": w(width, width), "b2": torch.zeros(width, dtype=F64),
        "W3": w(width, width), "b3": torch.zeros(width, dtype=F64),
        "Wh": w(width, n_prop * OUT_PER, scale=0.01 / np.sqrt(width)), "bh": torch.zeros(n_prop * OUT_PER, dtype=F64),
    }


def forward(X, prm, round_bf16: bool = True):
    """X [B, N, 3] -> dict of pre1, h1, pre2, h2, pre3, h3 [B, N, C], g [B, C],
    arg [B, C] (int64) and out [B, P*12], all float64 (differentiable in prm
    and X).  round_bf16=False keeps the activations exact (for derivative
    checks of the composition)."""
    rnd = _bf16_st if round_bf16 else (lambda x: x)
    X = torch.as_tensor(X).to(F64)
    pre1 = X @ prm["W1"] + prm["b1"]
    h1 = rnd(torch.relu(pre1))
    pre2 = h1 @ prm["W2"] + prm["b2"]
    h2 = rnd(torch.relu(pre2))
    pre3 = h2 @ prm["W3"] + prm["b3"]
    h3 = rnd(torch.relu(pre3))
    g, arg = pool_max(h3)
    out = g @ prm["Wh"] + prm["bh"]
    return {"pre1": pre1, "h1": h1, "pre2": pre2, "h2": h2, "pre3": pre3, "h3": h3, "g": g, "arg": arg, "out": out}


def pool_max(h):
    """Max over the point axis and the smallest index attaining it."""
    B, N, C = h.shape
    g = h.max(dim=1).values
    hit = h.detach() == g.detach()[:, None, :]
    idx = torch.arange(N)[None, :, None].expand(B, N, C)
    arg = torch.where(hit, idx, torch.full_like(idx, N)).min(dim=1).values
    g = torch.gather(h, 1, arg[:, None, :]).squeeze(1)
    return g, arg


def quat_to_R(q):
    """Rotation matrices of unit quaternions (w, x, y, z), [..., 3, 3]; the
    columns are the plane's X axis, Y axis and normal (Eq. 2-3)."""
    w, x, y, z = q.unbind(-1)
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def decode(out):
    """out [B, P*12] -> center [B,P,3], quat [B,P,4] (unit), radii [B,P,4], conf [B,P]."""
    o = out.reshape(out.shape[0], -1, OUT_PER)
    center = o[..., 0:3]
    qr = o[..., 3:7] + torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=out.dtype)
    quat = qr / qr.norm(dim=-1, keepdim=True)
    radii = torch.nn.functional.softplus(o[..., 7:11]) + R_MIN
    conf = o[..., 11]
    return center, quat, radii, conf


def descriptors(quat, radii):
    """Unit normal and half-extents (a >= b) of planes."""
    n = quat_to_R(quat)[..., :, 2]
    ex = 0.5 * (radii[..., 0] + radii[..., 1])
    ey = 0.5 * (radii[..., 2] + radii[..., 3])
    a = torch.maximum(ex, ey)
    b = torch.minimum(ex, ey)
    return n, a, b


def pair_dist(cp, np_, ap, bp, ct, nt, at, bt):
    """d(p, t) for all pairs: [P, T]."""
    dc = ((cp[:, None, :] - ct[None, :, :]) ** 2).sum(-1)
    dn = 1.0 - ((np_[:, None, :] * nt[None, :, :]).sum(-1)) ** 2
    de = (ap[:, None] - at[None, :]) ** 2 + (bp[:, None] - bt[None, :]) ** 2
    return dc + W_N * dn + W_E * de


def set_loss(out, targets):
    """Mean over views of the set loss; targets[b] = (center [T,3], quat [T,4],
    radii [T,4]) of the view's target planes in its camera frame."""
    center, quat, radii, conf = decode(out)
    n_p, a_p, b_p = descriptors(quat, radii)
    total = 0.0
    for b, (ct, qt, rt) in enumerate(targets):
        ct, qt, rt = (torch.as_tensor(x).to(F64) for x in (ct, qt, rt))
        n_t, a_t, b_t = descriptors(qt / qt.norm(dim=-1, keepdim=True), rt)
        D = pair_dist(center[b], n_p[b], a_p[b], b_p[b], ct, n_t, a_t, b_t)
        T = D.shape[1]
        P = D.shape[0]
        if T > 0:
            best = nearest(D)
            geo = D[best, torch.arange(T)].mean()
            y = torch.zeros(P, dtype=F64)
            y[best] = 1.0
        else:
            geo = torch.zeros((), dtype=F64)
            y = torch.zeros(P, dtype=F64)
        s = conf[b]
        bce = (torch.nn.functional.softplus(s) - y * s).mean()   # BCE with logits
        total = total + geo + bce
    return total / len(targets)


def nearest(D):
    """Index of the nearest proposal of each target (smallest index on ties)."""
    P = D.shape[0]
    m = D.detach().min(dim=0).values
    idx = torch.arange(P)[:, None].expand_as(D)
    return torch.where(D.detach() == m[None, :], idx, torch.full_like(idx, P)).min(dim=0).values


def grads_given_arg(X, prm, arg, d_out):
    """Gradient of sum(d_out * out) with respect to every parameter, with the
    pooled point of each channel fixed to arg [B, C] (the forward's choice).
    Returns a dict of float64 tensors shaped like prm."""
    p = {k: v.detach().clone().requires_grad_(True) for k, v in prm.items()}
    X = torch.as_tensor(X).to(F64)
    pre1 = X @ p["W1"] + p["b1"]
    h1 = _bf16_st(torch.relu(pre1))
    pre2 = h1 @ p["W2"] + p["b2"]
    h2 = _bf16_st(torch.relu(pre2))
    pre3 = h2 @ p["W3"] + p["b3"]
    h3 = _bf16_st(torch.relu(pre3))
    arg = torch.as_tensor(arg).to(torch.int64)
    g = torch.gather(h3, 1, arg[:, None, :]).squeeze(1)
    out = g @ p["Wh"] + p["bh"]
    (out * torch.as_tensor(d_out).to(F64)).sum().backward()
    return {k: v.grad.detach() for k, v in p.items()}
