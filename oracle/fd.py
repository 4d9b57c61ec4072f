"""Central finite differences of the oracle's render, one parameter coordinate
at a time.  TEST INFRASTRUCTURE ONLY: see the package docstring.

The objective is L(theta) = sum_p gD_p D_p + gN_p . N_p with fixed upstream
gradients, the functional whose gradient plane_render_bwd computes.  Moving
one coordinate of plane k changes only the pixels inside plane k's filter
footprint (oracle.footprint_tiles: outside it the plane's weight is below
tau), so each evaluation covers those tiles only, each pixel against the
planes whose footprint touches its tile (the tiled evaluation, which equals
the brute force bit for bit).  The difference is formed pixel by pixel before
summing, so pixels the move leaves unchanged cancel exactly.

A coordinate is reported as discontinuous when the +-h moves change any
affected pixel's ordered hit list, which hits are opaque (the kink of the
clamped weight at a* = 0), the branch Eq. 9 takes, or the side Eq. 7 takes
(P_X, P_Y > 0): a finite difference across a jump or a kink is meaningless.
"""

from __future__ import annotations

import numpy as np
import torch

from .render import OracleParams, _composite, _pairs, _t, footprint_tiles


class FdObjective:
    def __init__(self, center, quat, radii, cam, lam, gD, gN, prm: OracleParams = OracleParams(), tiles=(8, 8)):
        self.base = [_t(center).clone(), _t(quat).clone(), _t(radii).clone()]
        self.cam, self.lam, self.prm = cam, lam, prm
        self.tw, self.th = tiles
        P = cam.width * cam.height
        self.gD = _t(gD).reshape(P)
        self.gN = _t(gN).reshape(3, P).T.contiguous()
        self.ntx = (cam.width + self.tw - 1) // self.tw
        self.nty = (cam.height + self.th - 1) // self.th
        self.rects = torch.as_tensor(footprint_tiles(*self.base, cam, lam, prm, self.tw, self.th))

    def _rect(self, params, k):
        r = footprint_tiles(params[0][k:k + 1], params[1][k:k + 1], params[2][k:k + 1], self.cam, self.lam,
                                   self.prm, self.tw, self.th)[0]
        return [int(x) for x in r]

    def _tile_pixels(self, tx, ty):
        key = (tx, ty)
        cache = self.__dict__.setdefault("_tp", {})
        if key not in cache:
            W, H = self.cam.width, self.cam.height
            ys = torch.arange(ty * self.th, min(ty * self.th + self.th, H))
            xs = torch.arange(tx * self.tw, min(tx * self.tw + self.tw, W))
            cache[key] = (ys[:, None] * W + xs[None, :]).reshape(-1)
        return cache[key]

    def _eval(self, params, k, tiles, cand_k):
        """Per-pixel objective terms, ordered hit lists and branch flags on
        the pixels of `tiles`; plane k is a candidate on the tiles cand_k."""
        rects = self.rects
        tt = torch.tensor(tiles, dtype=torch.int64)
        inr = ((rects[None, :, 0] <= tt[:, 0:1]) & (rects[None, :, 2] >= tt[:, 0:1])
               & (rects[None, :, 1] <= tt[:, 1:2]) & (rects[None, :, 3] >= tt[:, 1:2]))   # [tiles, K]
        inr[:, k] = torch.tensor([t in cand_k for t in tiles])
        kc = max(1, int(inr.sum(1).max()))
        # candidates of each tile in ascending plane order, padded with -1
        order = torch.argsort((~inr).to(torch.int8), dim=1, stable=True)[:, :kc]
        rows = torch.where(inr.gather(1, order), order, torch.full_like(order, -1))
        pix, idx = [], []
        for i, (tx, ty) in enumerate(tiles):
            tp = self._tile_pixels(tx, ty)
            pix.append(tp)
            idx.append(rows[i][None].expand(tp.numel(), kc))
        pix = torch.cat(pix)
        idx = torch.cat(idx)
        ok = idx >= 0
        idx = idx.clamp_min(0)
        q = _pairs(params[0][idx], params[1][idx], params[2][idx], self.cam, self.lam, pix, self.prm, cand=ok)
        D, N, aux = _composite(q, self.prm)
        f = self.gD[pix] * D + (self.gN[pix] * N).sum(-1)
        ids = aux["ids"]
        sel = ids.clamp_min(0)
        taken = ids >= 0
        opaque = (q["w"].gather(1, sel) >= 1) & taken
        PXp = (q["PX"].gather(1, sel) > 0) & taken
        PYp = (q["PY"].gather(1, sel) > 0) & taken
        if self.prm.weight_mode == "G":
            xb = torch.zeros_like(taken)
        else:
            aX = q["rX"] - q["PX"].abs()
            aY = q["rY"] - q["PY"].abs()
            xb = (aX.gather(1, sel) < aY.gather(1, sel)) & taken
        plane_ids = torch.where(taken, idx.gather(1, sel), torch.full_like(sel, -1))
        sig = torch.cat([plane_ids, opaque.long(), PXp.long(), PYp.long(), xb.long()], 1)
        return f, sig

    def central_difference(self, which: int, k: int, comp: int, h: float = 1e-6):
        """(fd, err, absd, continuous): the central difference of L along
        the coordinate, a bound of its float64 rounding error, the sum over
        pixels of |per-pixel difference| / 2h (the scale its truncation error
        is relative to when pixel terms cancel), and whether the moves stay
        on one smooth piece."""
        params = {}
        rect = None
        for s in (+1, -1, 0):
            p = [b.clone() for b in self.base]
            p[which][k, comp] += s * h
            params[s] = p
            r = self._rect(p, k)
            if r[0] <= r[2] and r[1] <= r[3]:
                rect = r if rect is None else [min(rect[0], r[0]), min(rect[1], r[1]), max(rect[2], r[2]),
                                               max(rect[3], r[3])]
        if rect is None:
            return 0.0, 0.0, 0.0, True   # the plane reaches no pixel
        tiles = [(tx, ty) for ty in range(rect[1], rect[3] + 1) for tx in range(rect[0], rect[2] + 1)]
        cand_k = set(tiles)
        f, sig = {}, {}
        for s in (+1, -1, 0):
            f[s], sig[s] = self._eval(params[s], k, tiles, cand_k)
        cont = torch.equal(sig[1], sig[0]) and torch.equal(sig[-1], sig[0])
        d = f[1] - f[-1]
        fd = float(d.sum()) / (2 * h)
        changed = d != 0
        err = float(((f[1].abs() + f[-1].abs()) * changed).sum()) * 2.0 ** -52 / (2 * h) + abs(fd) * 2.0 ** -50
        absd = float(d.abs().sum()) / (2 * h)
        return fd, err, absd, cont


def random_coordinates(K: int, n: int, seed: int):
    """n distinct (group, plane, component) coordinates, uniform over the
    11 K parameters (center 3, quaternion 4, radii 4 per plane)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(11 * K, size=n, replace=False)
    out = []
    for x in flat.tolist():
        if x < 3 * K:
            out.append((0, x // 3, x % 3))
        elif x < 7 * K:
            out.append((1, (x - 3 * K) // 4, (x - 3 * K) % 4))
        else:
            out.append((2, (x - 7 * K) // 4, (x - 7 * K) % 4))
    return out
