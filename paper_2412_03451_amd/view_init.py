"""Learned initialisation of a fit, per-view form: a point-set network reads
4096 back-projected depth samples of one view and proposes 256 planes in that
view's camera frame; a scene's initial planes take the supporting planes of
their nearest confident proposals (the plain initialisation stays the
fallback).  The network and its kernels are in initnet.py; the geometry
(back-projection, proposal decoding and mapping to the world, refinement)
runs in the library's kernels (include/initnet.h).

Training data come from the plain method: rooms are fitted by the batched
fitting loop from their noisy initialisation, and each view's targets are the
fitted planes that take part in its render (a plane whose gradient in that
view is not zero), in the view's camera frame.
"""

from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from ._lib import check
from .fit import BatchFit, FitConfig, Scene
from .initnet import InitNet
from .splat import Job, Renderer, _ptr, _stream, pack_cameras

N_POINTS = 4096      # depth samples per view
N_PROPOSALS = 256    # proposals per view
SIGMA = 0.01         # multiplicative depth noise of the samples


# ---------------------------------------------------------------- rotations (torch, float64)
def quat_to_matrix(q: torch.Tensor) -> torch.Tensor:
    q = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def matrix_to_quat(m: torch.Tensor) -> torch.Tensor:
    """Unit quaternions of rotation matrices [..., 3, 3] (Shepperd's method,
    every branch evaluated and the largest of the trace and the diagonal kept)."""
    m00, m11, m22 = m[..., 0, 0], m[..., 1, 1], m[..., 2, 2]
    tr = m00 + m11 + m22
    cands = []
    s = torch.sqrt((tr + 1).clamp_min(1e-12)) * 2
    cands.append(torch.stack([0.25 * s, (m[..., 2, 1] - m[..., 1, 2]) / s, (m[..., 0, 2] - m[..., 2, 0]) / s,
                              (m[..., 1, 0] - m[..., 0, 1]) / s], -1))
    s = torch.sqrt((1 + m00 - m11 - m22).clamp_min(1e-12)) * 2
    cands.append(torch.stack([(m[..., 2, 1] - m[..., 1, 2]) / s, 0.25 * s, (m[..., 0, 1] + m[..., 1, 0]) / s,
                              (m[..., 0, 2] + m[..., 2, 0]) / s], -1))
    s = torch.sqrt((1 + m11 - m00 - m22).clamp_min(1e-12)) * 2
    cands.append(torch.stack([(m[..., 0, 2] - m[..., 2, 0]) / s, (m[..., 0, 1] + m[..., 1, 0]) / s, 0.25 * s,
                              (m[..., 1, 2] + m[..., 2, 1]) / s], -1))
    s = torch.sqrt((1 + m22 - m00 - m11).clamp_min(1e-12)) * 2
    cands.append(torch.stack([(m[..., 1, 0] - m[..., 0, 1]) / s, (m[..., 0, 2] + m[..., 2, 0]) / s,
                              (m[..., 1, 2] + m[..., 2, 1]) / s, 0.25 * s], -1))
    pick = torch.stack([tr, m00, m11, m22], -1).argmax(-1)
    q = torch.stack(cands, -2).gather(-2, pick[..., None, None].expand(*pick.shape, 1, 4)).squeeze(-2)
    return q / q.norm(dim=-1, keepdim=True)


# ---------------------------------------------------------------- network input
def view_points(tD: torch.Tensor, cams_dev: torch.Tensor, V: int, H: int, W: int, n: int = N_POINTS,
                sigma: float = SIGMA, seed: int = 0):
    """X [V, n, 3]: depth samples of every view back-projected to its camera
    frame (initnet_view_points), candidate pixels and noise drawn here."""
    from . import _lib
    lib = _lib.load()
    dev = tD.device
    rng = np.random.default_rng(seed)
    n_cand = 2 * n
    cand = torch.as_tensor(rng.integers(0, H * W, (V, n_cand)).astype(np.int32), device=dev)
    eps = torch.as_tensor(rng.standard_normal((V, n_cand)).astype(np.float32), device=dev)
    X = torch.empty(V, n, 3, dtype=torch.float32, device=dev)
    kept = torch.empty(V, dtype=torch.int32, device=dev)
    depth = tD.contiguous()   # held until the call returns
    check(lib.initnet_view_points(_ptr(depth), _ptr(cams_dev), V, H, W, _ptr(cand), _ptr(eps), n_cand, n,
                                  float(sigma), _ptr(X), _ptr(kept), _stream()))
    return X, kept


# ---------------------------------------------------------------- training targets
def visible_planes(planes, cams, tile=(16, 16), chunk: int = 20, device="cuda") -> torch.Tensor:
    """[V, K] bool: plane k takes part in the render of view v (its gradient
    in that view, for upstream gradients of one on every pixel, is not zero).
    Each view renders its own copy of the planes, so one backward gives every
    view's gradients."""
    c, q, r = (_dev32(x, device) for x in planes)
    K = c.shape[0]
    W, H = int(cams[0].width), int(cams[0].height)
    out = []
    lt = torch.tensor([300.0], device=device)
    for s in range(0, len(cams), chunk):
        vs = list(range(s, min(len(cams), s + chunk)))
        n = len(vs)
        jobs = [Job(i * K, (i + 1) * K, v, W, H, tile) for i, v in enumerate(vs)]
        rend = Renderer(jobs, cams, device=device, pair_capacity=1 << 20)
        cc, qq, rr = c.repeat(n, 1), q.repeat(n, 1), r.repeat(n, 1)
        rend.render(cc, qq, rr, lt)
        gD = torch.ones(rend.n_pixels, device=device)
        gN = torch.ones(3 * rend.n_pixels, device=device)
        gc, gq, gr = rend.backward(cc, qq, rr, lt, gD, gN)
        g = torch.cat([gc, gq, gr], 1).view(n, K, 11)
        out.append((g != 0).any(-1))
    return torch.cat(out)


def camera_frame_targets(planes, cams, visible: torch.Tensor, device="cuda"):
    """Rows [T, 11] (center, quaternion, radii in each view's camera frame)
    of the visible planes, view after view, and their offsets [V + 1]."""
    c = torch.as_tensor(np.asarray(planes[0], np.float64), device=device)
    Rq = quat_to_matrix(torch.as_tensor(np.asarray(planes[1], np.float64), device=device))
    r = torch.as_tensor(np.asarray(planes[2], np.float64), device=device)
    rows, off = [], [0]
    for v, cam in enumerate(cams):
        sel = torch.nonzero(visible[v]).squeeze(1)
        R = torch.as_tensor(np.asarray(cam.R, np.float64), device=device)
        t = torch.as_tensor(np.asarray(cam.t, np.float64), device=device)
        cc = c[sel] @ R.T + t
        qc = matrix_to_quat(R @ Rq[sel])
        rows.append(torch.cat([cc, qc, r[sel]], 1).float())
        off.append(off[-1] + int(sel.numel()))
    return torch.cat(rows).contiguous(), torch.tensor(off, dtype=torch.int32, device=device)


def _dev32(x, device):
    if torch.is_tensor(x):
        return x.detach().to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=device)


def render_targets(planes, cams, tile=(16, 16), lam: float = 300.0, device="cuda"):
    """Depth [V, H*W] and normal [V, 3*H*W] of the planes seen from every camera."""
    c, q, r = (_dev32(x, device) for x in planes)
    W, H = int(cams[0].width), int(cams[0].height)
    rt = Renderer([Job(0, c.shape[0], v, W, H, tile) for v in range(len(cams))], cams, device=device,
                  pair_capacity=1 << 22)
    D, N = rt.render(c, q, r, torch.tensor([lam], device=device))
    return D.view(len(cams), -1).clone(), N.view(len(cams), -1).clone()


def fit_rooms(rooms, iters: int, cfg: FitConfig | None = None, device="cuda"):
    """Plain batched fit of rooms (dicts with init, cams, tD, tN); the fitted
    planes of each room (numpy)."""
    scenes = [Scene(rm["init"].center, rm["init"].quat, rm["init"].radii, rm["cams"], rm["tD"], rm["tN"])
              for rm in rooms]
    fit = BatchFit(scenes, cfg=cfg or FitConfig(check_every=250), device=device)
    fit.size_capacity()
    fit.run(iters, graph=True)
    out = []
    for i in range(len(rooms)):
        c, q, r = fit.planes(i)
        out.append((c.cpu().numpy(), q.cpu().numpy(), r.cpu().numpy()))
    return out


class ViewData:
    """Training samples: X [S, N, 3] and, per sample, its target rows."""

    def __init__(self, device="cuda"):
        self.X = []
        self.rows = []
        self.off = []
        self.device = device

    def add_room(self, room, fitted, seed: int):
        cams = room["cams"]
        V = len(cams)
        W, H = int(cams[0].width), int(cams[0].height)
        X, _ = view_points(room["tD"], pack_cameras(cams, self.device), V, H, W, seed=seed)
        vis = visible_planes(fitted, cams, device=self.device)
        rows, off = camera_frame_targets(fitted, cams, vis, device=self.device)
        for v in range(V):
            self.X.append(X[v])
            self.rows.append(rows[int(off[v]):int(off[v + 1])])

    def batch(self, idx):
        X = torch.stack([self.X[i] for i in idx]).contiguous()
        rows = [self.rows[i] for i in idx]
        off = np.cumsum([0] + [r.shape[0] for r in rows]).astype(np.int32)
        return X, torch.cat(rows).contiguous(), torch.as_tensor(off, device=X.device)


def train(net: InitNet, data: ViewData, steps: int, batch: int = 32, lr: float = 1e-3, seed: int = 0, log=None):
    rng = np.random.default_rng(seed)
    S = len(data.X)
    hist = []
    for it in range(steps):
        idx = rng.choice(S, size=batch, replace=S < batch)
        X, tgt, off = data.batch(idx)
        g, arg, out = net.forward(X)
        loss, d_out = net.set_loss(out, tgt, off)
        net.adam_step(net.backward(X, g, arg, d_out), lr=lr)
        if it % 200 == 0 or it == steps - 1:
            hist.append((it, float(loss.mean())))
            if log:
                log(f"initnet step {it}: set loss {hist[-1][1]:.5f}")
    return hist


# ---------------------------------------------------------------- use
def proposals(net: InitNet, X: torch.Tensor, cams_dev: torch.Tensor, batch: int = 32):
    """World-frame proposals of every view: center [V P, 3], quat, radii, conf."""
    from . import _lib
    lib = _lib.load()
    V = X.shape[0]
    P = net.P
    dev = X.device
    outs = []
    for s in range(0, V, batch):
        Xb = X[s:s + batch]
        if Xb.shape[0] % 2:
            Xb = torch.cat([Xb, Xb[-1:]])
        _, _, o = net.forward(Xb)
        outs.append(o[:min(batch, V - s)])
    out = torch.cat(outs).contiguous()
    view_cam = torch.arange(V, dtype=torch.int32, device=dev)
    c = torch.empty(V * P, 3, device=dev)
    q = torch.empty(V * P, 4, device=dev)
    r = torch.empty(V * P, 4, device=dev)
    f = torch.empty(V * P, device=dev)
    check(lib.initnet_proposals_to_world(_ptr(out), V, P, _ptr(cams_dev), _ptr(view_cam), _ptr(c), _ptr(q), _ptr(r),
                                         _ptr(f), _stream()))
    return c, q, r, f


def refine(init, props, conf_min: float = 0.5, d_max: float = 0.1, device="cuda"):
    """initnet_refine_planes: initial planes take the supporting planes of
    their nearest confident proposals.  Returns (center, quat, radii) device
    tensors and the number of planes changed."""
    from . import _lib
    lib = _lib.load()
    c0, q0, r0 = (_dev32(x, device) for x in init)
    K = c0.shape[0]
    pc, pq, pr, pf = props
    oc = torch.empty_like(c0)
    oq = torch.empty_like(q0)
    match = torch.empty(K, dtype=torch.int32, device=device)
    check(lib.initnet_refine_planes(_ptr(c0), _ptr(q0), _ptr(r0), K, _ptr(pc), _ptr(pq), _ptr(pr), _ptr(pf),
                                    int(pc.shape[0]), float(conf_min), float(d_max), _ptr(oc), _ptr(oq),
                                    _ptr(match), _stream()))
    return (oc, oq, r0), int((match >= 0).sum())


def depth_l1(planes, cams, tD, device="cuda") -> float:
    D, _ = render_targets(planes, cams, device=device)
    return float((D - tD).abs().mean())


def learned_init(net: InitNet, init, cams, tD, seed: int = 0, conf_min: float = 0.5, d_max: float = 0.1,
                 device="cuda"):
    """Scene initialisation refined by the network's proposals, with the plain
    one as the fallback (used when the refined planes render a larger depth
    L1 over the views).  Returns (planes, info)."""
    V = len(cams)
    W, H = int(cams[0].width), int(cams[0].height)
    cams_dev = pack_cameras(cams, device)
    X, _ = view_points(tD, cams_dev, V, H, W, seed=seed)
    props = proposals(net, X, cams_dev)
    refined, moved = refine(init, props, conf_min, d_max, device)
    e_plain = depth_l1(init, cams, tD, device=device)
    e_ref = depth_l1(refined, cams, tD, device=device)
    use = e_ref < e_plain
    planes = refined if use else tuple(_dev32(x, device) for x in init)
    return planes, {"planes_refined": moved, "planes": int(np.asarray(init[0]).shape[0]),
                    "depth_l1_plain_init": e_plain, "depth_l1_learned_init": e_ref,
                    "used": "learned" if use else "plain (fallback)"}
