"""Fitting loop of the method (Sec. 3.3): Adam on the plane parameters against
target depth and normal maps, with the loss of Eq. 14 and lambda of Eq. 10.

One iteration is: ps_fit_schedule (device-side iteration counter, lambda,
Adam step and the view of each job) -> plane_project -> tile_bin ->
plane_render_fwd -> loss_depth_normal_cam -> plane_render_bwd ->
adam_step_planes; by default (FitConfig.one_launch) the last four are one
call, plane_render_step: one render launch for each 8x8 block's forward, loss
and backward, then the per-plane reduction, which also applies Adam when it
has a workgroup per plane.  Every step runs in the library's kernels and nothing in it
reads back to the host, so the iteration can be captured once in a HIP graph
(torch.cuda.CUDAGraph) and replayed.

Pair-list capacity: binning raises a device flag when the (tile, plane) pairs
exceed the workspace; the flag is sticky until the workspace is re-initialised.
The loop checks it after every run of `check_every` replays; on overflow it
restores the state saved before that run, grows the workspace, captures again
and repeats the run, so no iteration is ever applied with a truncated list.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, replace

import numpy as np
import torch

from ._lib import check
from .splat import (Job, Renderer, SplatParams, _ptr, _stream, adam_step, check_finite, grad_accumulate, split_planes,
                    tie_radii)


def view_schedule(n_views: int, n_rows: int, per_step: int = 1, seed: int = 0) -> np.ndarray:
    """[n_rows][per_step] camera indices: concatenated random permutations of
    the views (every view is used once per epoch)."""
    rng = np.random.default_rng(seed)
    need = n_rows * per_step
    out = []
    while sum(len(p) for p in out) < need:
        out.append(rng.permutation(n_views))
    return np.concatenate(out)[:need].reshape(n_rows, per_step).astype(np.int32)


@dataclass
class FitConfig:
    tile: tuple = (16, 16)
    views_per_step: int = 1
    lr: tuple = (1e-3, 1e-3, 1e-3)     # center, quaternion, radii
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-8
    r_min: float = 1e-4
    loss_w: tuple = (5.0, 5.0, 1.0)    # alpha_cos, alpha_nl1, alpha_d (Eq. 14)
    schedule_rows: int = 5000
    seed: int = 0
    check_every: int = 100
    grow: float = 1.5
    split_every: int = 0                # plane splitting every n iterations (Sec. 3.3: 1000); 0: off
    split_thresh: float = 0.2           # average |dL/dr| over a pair of radii that triggers a split
    single_radii: bool = False          # ablation (Sec. 4.3): one radius per axis, r+ = r- (from their mean)
    one_launch: bool = True             # plain step: forward, loss and backward in one render launch
    check_finite: bool = False          # before a run and after every checked run of steps, fail on NaN or
                                        # infinity in the planes (the kernels do not test their inputs)


@dataclass
class Scene:
    """One scene of a batch: planes (numpy or tensors, [K,3] / [K,4] / [K,4]),
    its cameras (all of one size) and per-view targets tgt_depth [V, H*W],
    tgt_normal [V, 3*H*W] (device tensors).  tile and pending (render
    pending-buffer size) may be set per scene (the autotuner's choice)."""
    center: object
    quat: object
    radii: object
    cams: list
    tgt_depth: torch.Tensor
    tgt_normal: torch.Tensor
    tile: tuple | None = None
    mask: torch.Tensor | None = None
    sched_seed: int | None = None   # seed of the scene's view schedule (None: cfg.seed + its index)


class BatchFit:
    """Fit of one or many scenes at once: every step advances all scenes by
    one iteration (views_per_step views each) in one launch per phase."""

    def __init__(self, scenes, cfg: FitConfig | None = None, params: SplatParams | None = None,
                 pair_capacity: int | None = None, size_capacity: bool = True, device="cuda"):
        self.cfg = cfg or FitConfig()
        self.device = torch.device(device)
        dev = self.device
        self.scenes = list(scenes)

        def T(x):
            if torch.is_tensor(x):
                return x.detach().to(device=dev, dtype=torch.float32).contiguous().clone()
            return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev).clone()

        cs = [T(sc.center).reshape(-1, 3) for sc in self.scenes]
        self.c = torch.cat(cs).contiguous()
        self.q = torch.cat([T(sc.quat).reshape(-1, 4) for sc in self.scenes]).contiguous()
        self.r = torch.cat([T(sc.radii).reshape(-1, 4) for sc in self.scenes]).contiguous()
        if self.cfg.single_radii:
            # one radius per axis: both directions start from their mean
            mx = 0.5 * (self.r[:, 0] + self.r[:, 1])
            my = 0.5 * (self.r[:, 2] + self.r[:, 3])
            self.r = torch.stack([mx, mx, my, my], dim=1).contiguous()
        self.K = int(self.c.shape[0])
        self.k_off = np.cumsum([0] + [int(x.shape[0]) for x in cs])
        self.m = torch.zeros(11 * self.K, device=dev)
        self.v = torch.zeros(11 * self.K, device=dev)
        self.ite = torch.zeros(1, dtype=torch.int32, device=dev)
        self.lam = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step_no = torch.zeros(1, dtype=torch.int32, device=dev)
        S = self.cfg.views_per_step
        cams, jobs, tables, tgt_off, tD, tN, masks = [], [], [], [], [], [], []
        self.v_off = [0]
        self.size = []
        pix = 0
        for si, sc in enumerate(self.scenes):
            W, H = int(sc.cams[0].width), int(sc.cams[0].height)
            if any(int(cm.width) != W or int(cm.height) != H for cm in sc.cams):
                raise ValueError(f"scene {si}: all views must have the same size")
            V = len(sc.cams)
            self.size.append((W, H))
            seed = self.cfg.seed + si if sc.sched_seed is None else sc.sched_seed
            table = view_schedule(V, self.cfg.schedule_rows, S, seed) + self.v_off[-1]
            tables.append(table)
            tile = tuple(sc.tile or self.cfg.tile)
            for j in range(S):
                jobs.append(Job(int(self.k_off[si]), int(self.k_off[si + 1]), int(table[0, j]), W, H, tile, si))
            for _ in range(V):
                tgt_off.append(pix)
                pix += W * H
            cams += list(sc.cams)
            tD.append(sc.tgt_depth.reshape(-1))
            tN.append(sc.tgt_normal.reshape(-1))
            masks.append(sc.mask)
            self.v_off.append(self.v_off[-1] + V)
        self.table = torch.as_tensor(np.concatenate(tables, axis=1), device=dev).contiguous()
        self.tgt_depth = torch.cat(tD).contiguous()
        self.tgt_normal = torch.cat(tN).contiguous()
        if all(mk is None for mk in masks):
            self.mask = None
        else:
            self.mask = torch.cat([mk.reshape(-1).to(torch.uint8) if mk is not None else
                                   torch.ones(sc.tgt_depth.numel(), dtype=torch.uint8, device=dev)
                                   for mk, sc in zip(masks, self.scenes)]).contiguous()
        self.tgt_off = torch.tensor(tgt_off, dtype=torch.int64, device=dev)
        self.params = params or SplatParams()
        self.jobs = jobs
        self.rend = Renderer(jobs, cams, device=dev, pair_capacity=pair_capacity or (1 << 16), params=self.params)
        self.acc = torch.zeros(self.K, 4, device=dev)   # sum of |dL/dr| since the last split
        self.cnt = torch.zeros(self.K, dtype=torch.int32, device=dev)   # iterations with a radii gradient
        self.since_split = 0
        self.splits = []                                  # (iteration, planes before, planes after)
        self.graph = None
        self.last_loss = None
        if size_capacity:
            self._size_capacity()

    # ------------------------------------------------------------------ capacity
    def _size_capacity(self):
        """Bin the current state (views of the next iteration) and grow the
        workspace to fit with margin."""
        lib = self.rend.lib
        ite = self.ite.clone()
        check(lib.ps_fit_schedule(C.byref(self.rend.L), _ptr(self.rend.ws), _ptr(ite), _ptr(self.table),
                                  int(self.table.shape[0]), _ptr(self.lam), _ptr(self.step_no), _stream()))
        self.rend.project(self.c, self.q, self.r, self.lam)
        self.rend.bin(check_capacity=True, grow=2.0)

    def size_capacity(self, rows: int | None = None, margin: float = 1.5):
        """Size the pair lists for the views of the first `rows` schedule rows
        (every view of the largest scene by default) at the current state."""
        lib = self.rend.lib
        if rows is None:
            rows = max(self.v_off[i + 1] - self.v_off[i] for i in range(len(self.scenes)))
        rows = min(rows, int(self.table.shape[0]))
        need_max = 0
        for row in range(rows):
            ite = torch.tensor([int(self.ite.item()) + row], dtype=torch.int32, device=self.device)
            check(lib.ps_fit_schedule(C.byref(self.rend.L), _ptr(self.rend.ws), _ptr(ite), _ptr(self.table),
                                      int(self.table.shape[0]), _ptr(self.lam), _ptr(self.step_no), _stream()))
            self.rend.project(self.c, self.q, self.r, self.lam)
            need = C.c_int64(0)
            self.rend.lib.tile_bin(C.byref(self.rend.L), _ptr(self.rend.ws), C.byref(need), _stream())
            need_max = max(need_max, int(need.value))
        cap = int(need_max * margin) + 1024
        if cap != self.rend.L.pair_capacity:
            self.rend._make_layout(cap)
            self.graph = None
        return need_max

    def _grow(self):
        cap = int(self.rend.L.pair_capacity * self.cfg.grow) + 1024
        self.rend._make_layout(cap)
        self.graph = None

    # ------------------------------------------------------------------ one step
    def _step(self, mark=None, ite=None):
        """One iteration; mark() (if given) is called between the phases
        (schedule + project, bin, forward + loss, backward, Adam), ite (if
        given) replaces the state's iteration counter."""
        cfg = self.cfg
        rend = self.rend
        m = mark or (lambda: None)
        m()
        check(rend.lib.ps_fit_schedule(C.byref(rend.L), _ptr(rend.ws), _ptr(self.ite if ite is None else ite),
                                       _ptr(self.table), int(self.table.shape[0]), _ptr(self.lam),
                                       _ptr(self.step_no), _stream()))
        rend.project(self.c, self.q, self.r, self.lam)
        m()
        rend.bin(check_capacity=False)
        m()
        fused = not cfg.single_radii and not cfg.split_every
        if fused and cfg.one_launch:
            # the plain step's forward, loss, backward and Adam with one render
            # launch (plane_render_step); its time counts as the forward phase
            loss = torch.empty(len(rend.jobs), 4, dtype=torch.float32, device=self.device)
            rend.step(self.tgt_depth, self.tgt_normal, self.m, self.v, self.step_no, self.tgt_off, mask=self.mask,
                      a_cos=cfg.loss_w[0], a_nl1=cfg.loss_w[1], a_d=cfg.loss_w[2], lr=cfg.lr, betas=cfg.betas,
                      eps=cfg.eps, r_min=cfg.r_min, loss=loss, maps=False)
            m()
            m()
            m()
            return loss
        # forward and render loss in one pass (plane_render_fwd_loss); in the
        # plain step the loss sums and Adam ride on the backward's launches
        # (plane_render_bwd_adam)
        D, N, loss, gD, gN = rend.forward_loss(self.tgt_depth, self.tgt_normal, self.tgt_off, mask=self.mask,
                                               a_cos=cfg.loss_w[0], a_nl1=cfg.loss_w[1], a_d=cfg.loss_w[2],
                                               reduce=not fused)
        m()
        if fused:
            loss = torch.empty(len(rend.jobs), 4, dtype=torch.float32, device=self.device)
            rend.backward_adam(self.c, self.q, self.r, self.lam, gD, gN, self.m, self.v, self.step_no, lr=cfg.lr,
                               betas=cfg.betas, eps=cfg.eps, r_min=cfg.r_min, loss=loss)
            m()
            m()
            return loss
        gc, gq, gr = rend.backward(self.c, self.q, self.r, self.lam, gD, gN)
        if cfg.single_radii:
            tie_radii(gr)
        if cfg.split_every:
            grad_accumulate(gr, self.acc, self.cnt)
        m()
        adam_step(self.c, self.q, self.r, gc, gq, gr, self.m, self.v, self.step_no, lr=cfg.lr, betas=cfg.betas,
                  eps=cfg.eps, r_min=cfg.r_min)
        m()
        return loss

    def diagnose(self):
        """Render statistics of the next iteration's views at the current
        state (no state change): the render counters with walk statistics,
        composited hits and the loss."""
        cfg = self.cfg
        rend = self.rend
        ite = self.ite.clone()
        check(rend.lib.ps_fit_schedule(C.byref(rend.L), _ptr(rend.ws), _ptr(ite), _ptr(self.table),
                                       int(self.table.shape[0]), _ptr(self.lam), _ptr(self.step_no), _stream()))
        rend.project(self.c, self.q, self.r, self.lam)
        rend.bin(check_capacity=False)
        D, N, Tr, Cn = rend.forward(diagnostics=True)
        loss, gD, gN = rend.loss_cam(D, N, self.tgt_depth, self.tgt_normal, self.tgt_off, mask=self.mask,
                                     a_cos=cfg.loss_w[0], a_nl1=cfg.loss_w[1], a_d=cfg.loss_w[2])
        rend.backward(self.c, self.q, self.r, self.lam, gD, gN, diagnostics=True)
        torch.cuda.synchronize()
        cnt = rend.counters()
        cnt["composited_hits"] = int(Cn.sum().item())
        cnt["loss"] = loss.sum(0).cpu().tolist()
        return cnt

    def _capture(self):
        # every kernel has run eagerly (capacity sizing, warm-up step) before capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._graph_loss = self._step()
        self.graph = g

    def state(self):
        return [t.clone() for t in (self.c, self.q, self.r, self.m, self.v, self.ite, self.acc, self.cnt)]

    def restore(self, st):
        for dst, src in zip((self.c, self.q, self.r, self.m, self.v, self.ite, self.acc, self.cnt), st):
            dst.copy_(src)

    def _split_scale(self):
        """Per plane: 1 / pixels per view of its scene, the factor from the
        summed loss of loss_depth_normal to the per-pixel mean that the
        splitting threshold is read against."""
        sc = np.empty(self.K, np.float32)
        for i, (W, H) in enumerate(self.size):
            sc[int(self.k_off[i]):int(self.k_off[i + 1])] = 1.0 / (W * H)
        return torch.from_numpy(sc).to(self.device)

    def _split(self):
        """Plane splitting (Sec. 3.3) of every scene; the plane set, the Adam
        moments (kept for planes that are not cut, zero for new children),
        the jobs' plane ranges and the workspace are rebuilt, and the step is
        captured again at the next run."""
        K0 = self.K
        c, q, r, parent, first = split_planes(self.c, self.q, self.r, self.acc, self.cnt, self._split_scale(),
                                              self.cfg.split_thresh)
        K1 = int(c.shape[0])
        self.splits.append((int(self.ite.item()), K0, K1))
        self.since_split = 0
        if K1 == K0:
            # same plane set: the captured step keeps its buffers
            self.acc.zero_()
            self.cnt.zero_()
            return
        self.acc = torch.zeros(K1, 4, device=self.device)
        self.cnt = torch.zeros(K1, dtype=torch.int32, device=self.device)
        first_h = first.cpu().numpy()
        pl = parent.long()
        single = ((first[1:] - first[:-1])[pl] == 1).to(torch.float32)

        def moments(x):
            xc, xq, xr = x[:3 * K0].view(K0, 3), x[3 * K0:7 * K0].view(K0, 4), x[7 * K0:].view(K0, 4)
            return torch.cat([(xc[pl] * single[:, None]).reshape(-1), (xq[pl] * single[:, None]).reshape(-1),
                              (xr[pl] * single[:, None]).reshape(-1)]).contiguous()

        self.m, self.v = moments(self.m), moments(self.v)
        self.c, self.q, self.r = c, q, r
        self.K = K1
        self.k_off = np.array([first_h[k] for k in self.k_off])
        self.jobs = [Job(int(self.k_off[j.scene]), int(self.k_off[j.scene + 1]), j.cam, j.width, j.height, j.tile,
                         j.scene) for j in self.jobs]
        self.rend = Renderer(self.jobs, self.rend.cams, device=self.device, pair_capacity=self.rend.L.pair_capacity,
                             params=self.params)
        self._eval = {}
        self.graph = None
        self.size_capacity()

    def overflowed(self) -> bool:
        return bool(self.rend.counters()["overflow_since_init"])

    # ------------------------------------------------------------------ checkpoint
    def save(self, path: str):
        """Write a checkpoint: plane parameters, Adam moments, the iteration
        counter (lambda of Eq. 10, the Adam step and the view of the next step
        follow from it), the split accumulators, the scenes' plane ranges and
        the split history.  A file of tensors only (read back with
        torch.load(weights_only=True))."""
        torch.cuda.synchronize()
        splits = torch.tensor(self.splits, dtype=torch.int64).reshape(-1, 3)
        torch.save({"c": self.c.cpu(), "q": self.q.cpu(), "r": self.r.cpu(), "m": self.m.cpu(), "v": self.v.cpu(),
                    "ite": self.ite.cpu(), "acc": self.acc.cpu(), "cnt": self.cnt.cpu(),
                    "k_off": torch.as_tensor(np.asarray(self.k_off, np.int64)),
                    "since_split": torch.tensor([self.since_split], dtype=torch.int64), "splits": splits}, path)

    def load(self, path: str):
        """Resume from a checkpoint of a fit over the same scenes (targets,
        cameras and configuration); continuing gives the same bits as the
        uninterrupted fit.  If splitting changed the plane counts, the jobs and
        the workspace are rebuilt for them."""
        d = torch.load(path, map_location="cpu", weights_only=True)
        k_off = d["k_off"].numpy()
        if len(k_off) != len(self.k_off):
            raise ValueError(f"checkpoint holds {len(k_off) - 1} scenes, this fit {len(self.k_off) - 1}")
        dev = self.device
        if np.array_equal(k_off, np.asarray(self.k_off)):
            # same plane set: copy into the buffers a captured step uses
            for dst, key in ((self.c, "c"), (self.q, "q"), (self.r, "r"), (self.m, "m"), (self.v, "v"),
                             (self.ite, "ite"), (self.acc, "acc"), (self.cnt, "cnt")):
                dst.copy_(d[key].to(dev))
        else:
            self.c, self.q, self.r = (d[k].to(dev).contiguous() for k in ("c", "q", "r"))
            self.m, self.v = d["m"].to(dev).contiguous(), d["v"].to(dev).contiguous()
            self.acc, self.cnt = d["acc"].to(dev).contiguous(), d["cnt"].to(dev).contiguous()
            self.ite.copy_(d["ite"].to(dev))
            self.K = int(self.c.shape[0])
            self.k_off = k_off
            self.jobs = [Job(int(k_off[j.scene]), int(k_off[j.scene + 1]), j.cam, j.width, j.height, j.tile, j.scene)
                         for j in self.jobs]
            self.rend = Renderer(self.jobs, self.rend.cams, device=dev, pair_capacity=self.rend.L.pair_capacity,
                                 params=self.params)
            self._eval = {}
            self.graph = None
            self.size_capacity()
        self.since_split = int(d["since_split"][0])
        self.splits = [tuple(int(x) for x in row) for row in d["splits"].tolist()]
        return self

    def run(self, n_steps: int, graph: bool = True, callback=None):
        """Advance n_steps iterations.  callback(fit, done) runs after every
        checked run of steps (host side, after a synchronisation)."""
        done = 0
        grows = 0
        if self.cfg.check_finite:
            bad = check_finite(self.c, self.q, self.r)
            if bad:
                raise FloatingPointError(f"{bad} non-finite plane parameters before the run")
        while done < n_steps:
            if grows > 8:
                raise RuntimeError("pair lists keep overflowing after growing the workspace: a tile list "
                                   "probably exceeds the per-tile limit (use smaller tiles)")
            chunk = min(self.cfg.check_every, n_steps - done)
            if self.cfg.split_every:
                chunk = min(chunk, self.cfg.split_every - self.since_split)
            saved = self.state()
            if graph and self.graph is None:
                # one eager step (loads every kernel), then capture
                self.restore(saved)
                self._step()
                torch.cuda.synchronize()
                if self.overflowed():
                    self.restore(saved)
                    self._grow()
                    grows += 1
                    continue
                self.restore(saved)
                self._capture()
                self.restore(saved)
            for _ in range(chunk):
                if graph:
                    self.graph.replay()
                    self.last_loss = self._graph_loss
                else:
                    self.last_loss = self._step()
            torch.cuda.synchronize()
            if self.overflowed():
                self.restore(saved)
                self._grow()
                grows += 1
                continue
            done += chunk
            if self.cfg.check_finite:
                bad = check_finite(self.c, self.q, self.r)
                if bad:
                    # back to the state saved before this run of steps (it was checked)
                    self.restore(saved)
                    raise FloatingPointError(f"{bad} non-finite plane parameters after {done} steps of this run; "
                                             f"state restored to step {done - chunk}")
            if self.cfg.split_every:
                self.since_split += chunk
                if self.since_split >= self.cfg.split_every:
                    self._split()
            if callback is not None:
                callback(self, done)
        return self

    # ------------------------------------------------------------------ evaluation
    def planes(self, scene: int = 0):
        a, b = int(self.k_off[scene]), int(self.k_off[scene + 1])
        return self.c[a:b], self.q[a:b], self.r[a:b]

    def subset(self, keep) -> "BatchFit":
        """A batch of the scenes `keep` (indices into this batch) that carries
        on from the current state: planes, Adam moments, the iteration
        counter and each scene's view schedule, so every kept scene follows
        the trajectory it had in this batch (a batch gives each scene the
        bits it gets alone).  Scenes that have reached their goal leave the
        batch this way.  Splitting statistics are not carried."""
        keep = list(keep)
        scenes = []
        for i in keep:
            c, q, r = self.planes(i)
            sc = self.scenes[i]
            scenes.append(replace(sc, center=c, quat=q, radii=r,
                                  sched_seed=self.cfg.seed + i if sc.sched_seed is None else sc.sched_seed))
        nf = BatchFit(scenes, cfg=self.cfg, params=self.params, pair_capacity=self.rend.L.pair_capacity,
                      size_capacity=False, device=self.device)
        for j, i in enumerate(keep):
            a0, a1 = int(self.k_off[i]), int(self.k_off[i + 1])
            b0 = int(nf.k_off[j])
            n = a1 - a0
            # moments laid out center (3K) | quat (4K) | radii (4K)
            for o_old, o_new, w in ((0, 0, 3), (3 * self.K, 3 * nf.K, 4), (7 * self.K, 7 * nf.K, 4)):
                nf.m[o_new + w * b0:o_new + w * (b0 + n)] = self.m[o_old + w * a0:o_old + w * a1]
                nf.v[o_new + w * b0:o_new + w * (b0 + n)] = self.v[o_old + w * a0:o_old + w * a1]
        nf.ite.copy_(self.ite)
        nf.step_no.copy_(self.step_no)
        nf.lam.copy_(self.lam)
        nf.size_capacity()
        return nf

    def render_view(self, view: int, scene: int = 0, lam: float | None = None):
        """Depth [H, W] and normal [3, H, W] of one view of a scene at the
        current state (lambda of the current iteration unless given)."""
        W, H = self.size[scene]
        a, b = int(self.k_off[scene]), int(self.k_off[scene + 1])
        tile = tuple(self.scenes[scene].tile or self.cfg.tile)
        r = Renderer([Job(a, b, self.v_off[scene] + view, W, H, tile)], self.rend.cams, device=self.device,
                     pair_capacity=self.rend.L.pair_capacity, params=self.params)
        lt = torch.tensor([lam if lam is not None else float(self.lam.item())], device=self.device)
        D, N = r.render(self.c, self.q, self.r, lt)
        return D.view(H, W), N.view(3, H, W)

    def depth_l1(self, scene: int = 0, views=None, lam: float | None = None, chunk: int = 20) -> float:
        """Mean |D - D^| over the pixels of the given views of a scene (all by
        default), rendered `chunk` views at a time.  The evaluation renderers
        are kept per (scene, views) and start from at most 2^20 pairs,
        growing only if a chunk needs more."""
        W, H = self.size[scene]
        V = self.v_off[scene + 1] - self.v_off[scene]
        views = list(range(V)) if views is None else list(views)
        a, b = int(self.k_off[scene]), int(self.k_off[scene + 1])
        tile = tuple(self.scenes[scene].tile or self.cfg.tile)
        cache = getattr(self, "_eval", {})
        self._eval = cache
        lt = torch.tensor([lam if lam is not None else float(self.lam.item())], device=self.device)
        total = torch.zeros((), dtype=torch.float64, device=self.device)
        for s0 in range(0, len(views), chunk):
            part = views[s0:s0 + chunk]
            key = (scene, tuple(part))
            if key not in cache:
                cache[key] = Renderer([Job(a, b, self.v_off[scene] + v, W, H, tile) for v in part], self.rend.cams,
                                      device=self.device, pair_capacity=min(self.rend.L.pair_capacity, 1 << 20),
                                      params=self.params)
            D, _ = cache[key].render(self.c, self.q, self.r, lt)
            offs = [int(self.tgt_off[self.v_off[scene] + v].item()) for v in part]
            Dt = torch.cat([self.tgt_depth[o:o + W * H] for o in offs])
            total += (D - Dt).abs().double().sum()
        return float(total.item()) / (len(views) * W * H)


class SceneFit(BatchFit):
    """Plain fit of one scene: planes (K), cameras (V views) and per-view
    targets tgt_depth [V, H*W], tgt_normal [V, 3*H*W] on the device."""

    def __init__(self, center, quat, radii, cams, tgt_depth, tgt_normal, mask=None, cfg: FitConfig | None = None,
                 params: SplatParams | None = None, pair_capacity: int | None = None, size_capacity: bool = True,
                 device="cuda"):
        cams = list(cams)
        super().__init__([Scene(center, quat, radii, cams, tgt_depth, tgt_normal, mask=mask)], cfg=cfg,
                         params=params, pair_capacity=pair_capacity, size_capacity=size_capacity, device=device)
        self.V = len(cams)
        self.W, self.H = self.size[0]


def jsonl_logger(path: str, depth_l1: bool = False):
    """A run() callback that appends one JSON line per checked run of steps:
    the iteration, lambda, the plane count, the loss terms of the last step
    per job (Eq. 14: normal cosine, normal L1, depth L1 sums), the pair count
    and overflow flag of the last binning, the pixels that took the exact
    fallback ordering path, and (with depth_l1) the mean depth error of every
    scene over all its views at the current lambda."""
    import json

    def cb(fit, done):
        cnt = fit.rend.counters()
        rec = {"iteration": int(fit.ite.item()), "lambda": float(fit.lam.item()), "planes": int(fit.K),
               "loss": None if fit.last_loss is None else fit.last_loss.detach().double().cpu().tolist(),
               "pairs": int(cnt["pairs"]), "overflow_since_init": int(cnt["overflow_since_init"]),
               "fallback_pixels": int(cnt["slow_pixels"])}
        if depth_l1:
            rec["depth_l1"] = [fit.depth_l1(s) for s in range(len(fit.scenes))]
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")
    return cb
