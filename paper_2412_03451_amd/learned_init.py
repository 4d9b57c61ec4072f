"""Learned initialisation of a fit: data, training, proposals and the
refined scene initialisation (the network and its kernels are in initnet.py).

The network reads the depth samples around one plane of the plain (noisy)
initialisation, expressed in that plane's frame (x, y along its axes, z
along its normal), and proposes the plane that the plain method would
converge to, in the same frame: one proposal per plane (P = 1).  Depth
samples come from the observed depth maps of the views, back-projected with
multiplicative noise; the samples of a plane are those within its grown
footprint and near its surface.

Training data come from the plain method itself: rooms are fitted by the
batched fitting loop from their noisy initialisation, and every initial
plane with enough samples pairs its samples with its converged plane.

At initialisation time each plane with enough samples takes the proposed
center and normal (its in-plane axes follow the normal by the smallest
rotation, its radii are kept); the others keep the plain values.  The plain
initialisation stays the fallback: the refined one is used only if its depth
error on the observed views is lower.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from .fit import BatchFit, FitConfig, Scene
from .initnet import InitNet
from .splat import Job, Renderer


# ---------------------------------------------------------------- rotations (numpy, float64)
def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def matrix_to_quat(R: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z) of rotation matrices [..., 3, 3]."""
    R = np.asarray(R, np.float64)
    shp = R.shape[:-2]
    R = R.reshape(-1, 3, 3)
    out = np.empty((R.shape[0], 4))
    for i, m in enumerate(R):
        tr = m[0, 0] + m[1, 1] + m[2, 2]
        if tr > 0:
            s = math.sqrt(tr + 1.0) * 2
            q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif m[0, 0] > m[1, 1] and m[0, 0] > m[2, 2]:
            s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
            q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif m[1, 1] > m[2, 2]:
            s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
        out[i] = np.asarray(q) / np.linalg.norm(q)
    return out.reshape(*shp, 4)


def _align(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Rotation matrices taking unit vectors a [n,3] to b [n,3] (smallest angle)."""
    v = np.cross(a, b)
    c = np.sum(a * b, -1)
    out = np.tile(np.eye(3), (a.shape[0], 1, 1))
    for i in range(a.shape[0]):
        s = np.linalg.norm(v[i])
        if s < 1e-12:
            continue
        k = v[i] / s
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        ang = math.atan2(s, c[i])
        out[i] = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)
    return out


# ---------------------------------------------------------------- data
def backproject(depth: torch.Tensor, cam, n: int, gen: torch.Generator, noise: float = 0.01) -> torch.Tensor:
    """n depth samples of a depth map [H, W] (pixels with depth > 0, drawn
    with replacement) back-projected to the camera frame [n, 3], depth
    scaled by (1 + noise N(0, 1))."""
    H, W = depth.shape
    idx = torch.nonzero(depth.reshape(-1) > 0).squeeze(1)
    if idx.numel() == 0:
        return torch.zeros(n, 3, device=depth.device)
    pick = idx[torch.randint(0, idx.numel(), (n,), generator=gen, device=depth.device)]
    z = depth.reshape(-1)[pick] * (1 + noise * torch.randn(n, generator=gen, device=depth.device))
    u = (pick % W).float() + 0.5
    v = (pick // W).float() + 0.5
    return torch.stack([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z], 1).contiguous()


def render_targets(planes, cams, tile=(16, 16), lam: float = 300.0, device="cuda"):
    """Depth [V, H*W] and normal [V, 3*H*W] of the planes seen from every camera."""
    c, q, r = (torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=device) for x in planes)
    W, H = int(cams[0].width), int(cams[0].height)
    rt = Renderer([Job(0, c.shape[0], v, W, H, tile) for v in range(len(cams))], cams, device=device,
                  pair_capacity=1 << 20)
    D, N = rt.render(c, q, r, torch.tensor([lam], device=device))
    return D.view(len(cams), -1).clone(), N.view(len(cams), -1).clone()


def fit_rooms(rooms, iters: int, cfg: FitConfig | None = None, device="cuda"):
    """Plain batched fit of rooms (each: dict with gt, init, cams); returns
    the fitted planes of each room (numpy) and the targets used."""
    scenes = []
    for rm in rooms:
        tD, tN = render_targets((rm["gt"].center, rm["gt"].quat, rm["gt"].radii), rm["cams"], device=device)
        rm["tD"], rm["tN"] = tD, tN
        init = rm["init"]
        scenes.append(Scene(init.center, init.quat, init.radii, rm["cams"], tD, tN))
    fit = BatchFit(scenes, cfg=cfg or FitConfig(check_every=250), device=device)
    fit.size_capacity()
    fit.run(iters, graph=True)
    out = []
    for i in range(len(rooms)):
        c, q, r = fit.planes(i)
        out.append((c.cpu().numpy(), q.cpu().numpy(), r.cpu().numpy()))
    return out


def world_samples(tD, cams, per_view: int = 4096, seed: int = 0, device="cuda") -> torch.Tensor:
    """Depth samples of every view back-projected to the world frame [V*per_view, 3]."""
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    W, H = int(cams[0].width), int(cams[0].height)
    pts = []
    for v, cam in enumerate(cams):
        Xc = backproject(tD[v].view(H, W), cam, per_view, gen).double()
        R = torch.tensor(np.asarray(cam.R, np.float64), device=device)
        t = torch.tensor(np.asarray(cam.t, np.float64), device=device)
        pts.append((Xc - t) @ R)   # R^T (x_c - t)
    return torch.cat(pts)


def plane_samples(planes, pts: torch.Tensor, n: int = 128, margin: float = 0.15, depth_tol: float = 0.3,
                  min_count: int = 16, seed: int = 0):
    """Samples around every plane in its own frame: X [K, n, 3] (float32) and
    the mask of planes with at least min_count samples (others are zeros).
    A world point belongs to plane k if its offset along the normal is within
    depth_tol and its in-plane offsets are within the grown radii."""
    dev = pts.device
    c = torch.as_tensor(np.asarray(planes[0], np.float64), device=dev)
    R = torch.as_tensor(quat_to_matrix(np.asarray(planes[1])), device=dev)
    r = torch.as_tensor(np.asarray(planes[2], np.float64), device=dev)
    K = c.shape[0]
    X = torch.zeros(K, n, 3, dtype=torch.float32, device=dev)
    ok = torch.zeros(K, dtype=torch.bool, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    for s in range(0, K, 64):
        e = min(K, s + 64)
        loc = torch.einsum("kmi,kij->kmj", pts[None] - c[s:e, None], R[s:e])   # [k, M, 3] local coordinates
        x, y, z = loc[..., 0], loc[..., 1], loc[..., 2]
        rr = r[s:e]
        inside = (z.abs() < depth_tol) & (x < rr[:, None, 0] + margin) & (x > -rr[:, None, 1] - margin) \
            & (y < rr[:, None, 2] + margin) & (y > -rr[:, None, 3] - margin)
        good = inside.sum(1) >= min_count
        if bool(good.any()):
            idx = torch.multinomial(inside[good].double(), n, replacement=True, generator=gen)
            Xs = torch.gather(loc[good], 1, idx[..., None].expand(-1, -1, 3)).float()
            gi = torch.nonzero(good).squeeze(1) + s
            X[gi] = Xs
        ok[s:e] = good
    return X, ok


def local_targets(init, fitted) -> np.ndarray:
    """Converged planes in the frame of their initial planes, [K, 11]."""
    c0 = np.asarray(init[0], np.float64)
    R0 = quat_to_matrix(np.asarray(init[1]))
    c1 = np.asarray(fitted[0], np.float64)
    R1 = quat_to_matrix(np.asarray(fitted[1]))
    cl = np.einsum("kij,ki->kj", R0, c1 - c0)            # R0^T (c1 - c0)
    Rl = np.einsum("kji,kjl->kil", R0, R1)               # R0^T R1
    return np.concatenate([cl, matrix_to_quat(Rl), np.asarray(fitted[2], np.float64)], 1).astype(np.float32)


@dataclass
class PlaneBatch:
    X: torch.Tensor        # [K, n, 3] samples in each plane's frame
    targets: np.ndarray    # [K, 11] converged planes in the same frames


def training_planes(rooms, fitted, n: int = 128, seed: int = 0, device="cuda") -> PlaneBatch:
    """Samples and targets of every initial plane with enough samples."""
    Xs, Ts = [], []
    for i, (rm, fit_planes) in enumerate(zip(rooms, fitted)):
        init = (rm["init"].center, rm["init"].quat, rm["init"].radii)
        pts = world_samples(rm["tD"], rm["cams"], seed=seed + i, device=device)
        X, ok = plane_samples(init, pts, n=n, seed=seed + i)
        T = local_targets(init, fit_planes)
        sel = torch.nonzero(ok).squeeze(1)
        Xs.append(X[sel])
        Ts.append(T[sel.cpu().numpy()])
    return PlaneBatch(torch.cat(Xs).contiguous(), np.concatenate(Ts))


def train_planes(net: InitNet, data: PlaneBatch, steps: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
                 log=None):
    """Adam on the set loss (one proposal per plane) over random batches of planes."""
    rng = np.random.default_rng(seed)
    dev = net.device
    K = data.X.shape[0]
    hist = []
    tgt_all = torch.tensor(data.targets, device=dev)
    off = torch.arange(batch + 1, dtype=torch.int32, device=dev)
    for it in range(steps):
        pick = torch.tensor(rng.choice(K, size=batch, replace=K < batch), device=dev)
        X = data.X[pick].contiguous()
        g, arg, out = net.forward(X)
        loss, d_out = net.set_loss(out, tgt_all[pick].contiguous(), off)
        net.adam_step(net.backward(X, g, arg, d_out), lr=lr)
        if it % 100 == 0 or it == steps - 1:
            hist.append((it, float(loss.mean())))
            if log:
                log(f"initnet step {it}: set loss {hist[-1][1]:.5f}")
    return hist


def refine(net: InitNet, init, X: torch.Tensor, ok: torch.Tensor):
    """Planes with samples take the proposed center and normal (world frame)."""
    c0 = np.asarray(init[0], np.float64)
    q0 = np.asarray(init[1], np.float64)
    R0 = quat_to_matrix(q0)
    sel = torch.nonzero(ok).squeeze(1)
    c, q = c0.copy(), q0.copy()
    if sel.numel() == 0:
        return (c.astype(np.float32), q.astype(np.float32), np.asarray(init[2], np.float32)), 0
    outs = []
    for s in range(0, sel.numel(), 1024):
        part = sel[s:s + 1024]
        Xb = X[part]
        if Xb.shape[0] % 2:
            Xb = torch.cat([Xb, Xb[-1:]])
        _, _, o = net.forward(Xb.contiguous())
        outs.append(o[:part.numel()].cpu().numpy().astype(np.float64))
    o = np.concatenate(outs)
    k = sel.cpu().numpy()
    n_loc = quat_to_matrix(o[:, 3:7] + np.array([1.0, 0, 0, 0]))[:, :, 2]
    n_loc *= np.where(n_loc[:, 2:3] < 0, -1.0, 1.0)      # keep the initial facing
    c[k] = c0[k] + np.einsum("kij,kj->ki", R0[k], o[:, 0:3])
    n_w = np.einsum("kij,kj->ki", R0[k], n_loc)
    Ra = _align(R0[k][:, :, 2], n_w / np.linalg.norm(n_w, axis=1, keepdims=True))
    q[k] = matrix_to_quat(Ra @ R0[k])
    return (c.astype(np.float32), q.astype(np.float32), np.asarray(init[2], np.float32)), int(k.size)


def learned_init(net: InitNet, init, cams, tD, n: int = 128, seed: int = 0, device="cuda"):
    """Scene initialisation refined by the network, with the plain one as the
    fallback.  Returns (planes, info)."""
    pts = world_samples(tD, cams, seed=seed, device=device)
    X, ok = plane_samples(init, pts, n=n, seed=seed)
    refined, moved = refine(net, init, X, ok)
    e_plain = depth_l1(init, cams, tD, device=device)
    e_ref = depth_l1(refined, cams, tD, device=device)
    use = e_ref < e_plain
    return (refined if use else tuple(np.asarray(x, np.float32) for x in init)), {
        "planes_refined": moved, "planes": int(np.asarray(init[0]).shape[0]), "depth_l1_plain_init": e_plain,
        "depth_l1_learned_init": e_ref, "used": "learned" if use else "plain (fallback)"}


def depth_l1(planes, cams, tD, tile=(16, 16), device="cuda") -> float:
    """Mean |D - D^| over the views (render at lambda = 300)."""
    D, _ = render_targets(planes, cams, tile=tile, device=device)
    return float((D - tD).abs().mean())


def iterations_to_target(planes, cams, tD, tN, target: float, max_iters: int, check_every: int = 50,
                         cfg: FitConfig | None = None, device="cuda"):
    """Fit from `planes` until the depth L1 (lambda = 300 renders of every
    view) is <= target; (iterations, fit seconds excluding the checks,
    final depth L1)."""
    fit = BatchFit([Scene(planes[0], planes[1], planes[2], cams, tD, tN)],
                   cfg=cfg or FitConfig(check_every=check_every), device=device)
    fit.size_capacity()
    done, secs = 0, 0.0
    err = fit.depth_l1(0, lam=300.0)
    while err > target and done < max_iters:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit.run(check_every, graph=True)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        done += check_every
        err = fit.depth_l1(0, lam=300.0)
    return done, secs, err
