"""Python front end of the splatting library: torch tensors in, C ABI calls out.

torch provides device memory and the current HIP stream; every computation
is a call into libplanesplat.so.  A `Renderer` owns one batch layout and its
workspace.  Typical use::

    r = Renderer.single_scene(cams, K, tile=(16, 16))
    depth, normal = r.render(center, quat, radii, lam)
    loss, gD, gN = r.loss(depth, normal, tgt_depth, tgt_normal)
    gc, gq, gr = r.backward(center, quat, radii, lam, gD, gN)
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import PsCamera, PsLayout, PsParams, PsSlot, check


@dataclass
class SplatParams:
    """Method constants (Sec. 3.2) and readings; see include/planesplat.h."""
    M: int = 30
    tau: float = 1e-4
    z_near: float = 0.01
    weight_mode: int = 0   # 0: min(1, 2 sigmoid), 1: sigmoid, 2: Gaussian of Eq. 5
    two_sided: int = 1
    flags: int = 0         # bit 0: exact fallback path; bits 4-5: pending size; bit 6: walk statistics

    def c(self) -> PsParams:
        return PsParams(self.M, self.tau, self.z_near, self.weight_mode, self.two_sided, self.flags)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def pack_cameras(cams, device="cuda") -> torch.Tensor:
    """Cameras (objects with width, height, fx, fy, cx, cy, R[3x3], t[3]) as a
    device byte tensor of ps_camera structs."""
    arr = (PsCamera * len(cams))()
    for i, cm in enumerate(cams):
        arr[i].width, arr[i].height = int(cm.width), int(cm.height)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(cm.fx), float(cm.fy), float(cm.cx), float(cm.cy)
        R = np.asarray(cm.R, np.float32).reshape(9)
        t = np.asarray(cm.t, np.float32).reshape(3)
        for j in range(9):
            arr[i].R[j] = float(R[j])
        for j in range(3):
            arr[i].t[j] = float(t[j])
    buf = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return buf.to(device)


@dataclass
class Job:
    plane_begin: int
    plane_end: int
    cam: int
    width: int
    height: int
    tile: tuple = (16, 16)
    scene: int = 0


class Renderer:
    """One batch of render jobs (views / scenes) with its device workspace."""

    def __init__(self, jobs: Sequence[Job], cams, device="cuda", pair_capacity: int | None = None,
                 params: SplatParams | None = None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.jobs = list(jobs)
        self.params = params or SplatParams()
        self.cams_host = list(cams) if not isinstance(cams, torch.Tensor) else None
        self.cams = cams if isinstance(cams, torch.Tensor) else pack_cameras(cams, self.device)
        self.n_cams = self.cams.numel() // C.sizeof(PsCamera)
        if pair_capacity is None:
            pair_capacity = 1 << 16
        self._make_layout(int(pair_capacity))
        self.last_pairs = 0
        self.generation = 0   # bumped by every project(): identifies the workspace contents

    @classmethod
    def single_scene(cls, cams, K: int, tile=(16, 16), **kw):
        jobs = [Job(0, K, i, int(c.width), int(c.height), tile) for i, c in enumerate(cams)]
        return cls(jobs, cams, **kw)

    # ------------------------------------------------------------------ layout
    def _make_layout(self, capacity: int):
        S = len(self.jobs)
        slots = (PsSlot * S)()
        for i, j in enumerate(self.jobs):
            s = slots[i]
            s.plane_begin, s.plane_end, s.cam = j.plane_begin, j.plane_end, j.cam
            s.width, s.height = j.width, j.height
            s.tile_w, s.tile_h = j.tile
            s.scene = j.scene
        L = PsLayout()
        check(self.lib.ps_layout_init(slots, S, capacity, C.byref(L)))
        self.slots = slots
        self.L = L
        self.ws = torch.empty(int(L.ws_bytes), dtype=torch.uint8, device=self.device)
        check(self.lib.ps_workspace_init(C.byref(L), slots, _ptr(self.ws), _stream()))
        # offsets of each job's outputs
        self.pix_off = [int(slots[i].pix_off) for i in range(S)]

    @property
    def n_pixels(self) -> int:
        return int(self.L.n_pixels)

    @property
    def n_planes(self) -> int:
        return int(self.L.n_planes)

    def region(self, i: int, dtype, count: int) -> torch.Tensor:
        """View of workspace region i (for tests and diagnostics)."""
        off = int(self.L.region[i])
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + count * itemsize].view(dtype)

    # ------------------------------------------------------------------ steps
    def project(self, center, quat, radii, lam):
        self._inputs = (center, quat, radii, lam)
        self.generation = getattr(self, "generation", 0) + 1
        prm = self.params.c()
        check(self.lib.plane_project(C.byref(self.L), _ptr(self.ws), _ptr(center), _ptr(quat), _ptr(radii),
                                     int(center.shape[0]), _ptr(self.cams), self.n_cams, _ptr(lam),
                                     C.byref(prm), _stream()))

    def bin(self, check_capacity: bool = True, grow: float = 1.5):
        if not check_capacity:
            check(self.lib.tile_bin(C.byref(self.L), _ptr(self.ws), None, _stream()))
            return
        need = C.c_int64(0)
        rc = self.lib.tile_bin(C.byref(self.L), _ptr(self.ws), C.byref(need), _stream())
        if rc == _lib.PS_ERR_CAPACITY and need.value > self.L.pair_capacity:
            self._make_layout(int(need.value * grow) + 1024)
            self.project(*self._inputs)
            rc = self.lib.tile_bin(C.byref(self.L), _ptr(self.ws), C.byref(need), _stream())
        check(rc)
        self.last_pairs = int(need.value)

    def forward(self, diagnostics: bool = False, mark_fallback: bool = False):
        """Depth [n_pixels] and normal [3 n_pixels]; with diagnostics also the
        final transmittance and the number of composited hits per pixel (with
        mark_fallback, plus 256 where the pixel took the exact fallback
        ordering path)."""
        depth = torch.empty(self.n_pixels, dtype=torch.float32, device=self.device)
        normal = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=self.device)
        trans = count = None
        if diagnostics:
            trans = torch.empty(self.n_pixels, dtype=torch.float32, device=self.device)
            count = torch.empty(self.n_pixels, dtype=torch.int32, device=self.device)
        prm = self.params.c()
        if diagnostics:
            prm.flags |= 64 | (128 if mark_fallback else 0)
        _, _, _, lam = self._inputs
        check(self.lib.plane_render_fwd(C.byref(self.L), _ptr(self.ws), _ptr(self.cams), self.n_cams, _ptr(lam),
                                        C.byref(prm), _ptr(depth), _ptr(normal), _ptr(trans), _ptr(count),
                                        _stream()))
        if diagnostics:
            return depth, normal, trans, count
        return depth, normal

    def forward_lists(self):
        """Forward that also stores the per-pixel lists (list-storing
        variant): depth, normal and (pos, a*, T) [M, n_pixels] plus count."""
        M = int(self.params.M)
        P = self.n_pixels
        depth = torch.empty(P, dtype=torch.float32, device=self.device)
        normal = torch.empty(3 * P, dtype=torch.float32, device=self.device)
        pos = torch.empty(M, P, dtype=torch.int32, device=self.device)
        a = torch.empty(M, P, dtype=torch.float32, device=self.device)
        T = torch.empty(M, P, dtype=torch.float32, device=self.device)
        cnt = torch.empty(P, dtype=torch.int32, device=self.device)
        prm = self.params.c()
        _, _, _, lam = self._inputs
        check(self.lib.plane_render_fwd_lists(C.byref(self.L), _ptr(self.ws), _ptr(self.cams), self.n_cams, _ptr(lam),
                                              C.byref(prm), _ptr(depth), _ptr(normal), _ptr(pos), _ptr(a), _ptr(T),
                                              _ptr(cnt), _stream()))
        return depth, normal, (pos, a, T, cnt)

    def backward_lists(self, center, quat, radii, lam, g_depth, g_normal, lists):
        """Gradients from the stored per-pixel lists (list-storing variant)."""
        pos, a, _, cnt = lists
        K = int(center.shape[0])
        gc = torch.empty(K, 3, dtype=torch.float32, device=self.device)
        gq = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        gr = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        prm = self.params.c()
        check(self.lib.plane_render_bwd_lists(C.byref(self.L), _ptr(self.ws), _ptr(center), _ptr(quat), _ptr(radii), K,
                                              _ptr(self.cams), self.n_cams, _ptr(lam), C.byref(prm),
                                              _ptr(g_depth.contiguous()), _ptr(g_normal.contiguous()), _ptr(pos),
                                              _ptr(a), _ptr(cnt), _ptr(gc), _ptr(gq), _ptr(gr), _stream()))
        return gc, gq, gr

    def render(self, center, quat, radii, lam):
        self.project(center, quat, radii, lam)
        self.bin()
        return self.forward()

    def render_diag(self, center, quat, radii, lam):
        """render() with the diagnostics: depth, normal, final transmittance
        and hit count per pixel, plus 256 where the pixel took the exact
        fallback ordering path."""
        self.project(center, quat, radii, lam)
        self.bin()
        return self.forward(diagnostics=True, mark_fallback=True)

    def loss(self, depth, normal, tgt_depth, tgt_normal, mask=None, a_cos=5.0, a_nl1=5.0, a_d=1.0):
        loss = torch.empty(len(self.jobs), 4, dtype=torch.float32, device=self.device)
        gD = torch.empty_like(depth)
        gN = torch.empty_like(normal)
        check(self.lib.loss_depth_normal(C.byref(self.L), _ptr(self.ws), _ptr(depth), _ptr(normal),
                                         _ptr(tgt_depth), _ptr(tgt_normal), _ptr(mask), a_cos, a_nl1, a_d,
                                         _ptr(loss), _ptr(gD), _ptr(gN), _stream()))
        return loss, gD, gN

    def loss_cam(self, depth, normal, tgt_depth, tgt_normal, tgt_off, mask=None, a_cos=5.0, a_nl1=5.0, a_d=1.0):
        """Loss against per-camera targets (tgt_off: device int64 pixel offset of each camera's target)."""
        loss = torch.empty(len(self.jobs), 4, dtype=torch.float32, device=self.device)
        gD = torch.empty_like(depth)
        gN = torch.empty_like(normal)
        check(self.lib.loss_depth_normal_cam(C.byref(self.L), _ptr(self.ws), _ptr(depth), _ptr(normal),
                                             _ptr(tgt_depth), _ptr(tgt_normal), _ptr(mask), _ptr(tgt_off),
                                             int(tgt_off.numel()), a_cos, a_nl1, a_d, _ptr(loss), _ptr(gD), _ptr(gN),
                                             _stream()))
        return loss, gD, gN

    def forward_loss(self, tgt_depth, tgt_normal, tgt_off=None, mask=None, a_cos=5.0, a_nl1=5.0, a_d=1.0,
                     reduce: bool = True):
        """Forward that forms the render loss as it composites
        (plane_render_fwd_loss): depth, normal, loss [jobs, 4], g_depth,
        g_normal, the bits of forward() followed by loss_cam() / loss().
        With reduce=False loss is None: the per-block partial sums stay in the
        workspace for backward_adam(loss=...)."""
        P = self.n_pixels
        depth = torch.empty(P, dtype=torch.float32, device=self.device)
        normal = torch.empty(3 * P, dtype=torch.float32, device=self.device)
        loss = torch.empty(len(self.jobs), 4, dtype=torch.float32, device=self.device)
        gD = torch.empty_like(depth)
        gN = torch.empty_like(normal)
        prm = self.params.c()
        _, _, _, lam = self._inputs
        n_tgt = 0 if tgt_off is None else int(tgt_off.numel())
        check(self.lib.plane_render_fwd_loss(C.byref(self.L), _ptr(self.ws), _ptr(self.cams), self.n_cams, _ptr(lam),
                                             C.byref(prm), _ptr(depth), _ptr(normal), _ptr(tgt_depth),
                                             _ptr(tgt_normal), _ptr(mask), _ptr(tgt_off), n_tgt, a_cos, a_nl1, a_d,
                                             _ptr(loss if reduce else None), _ptr(gD), _ptr(gN), _stream()))
        return depth, normal, (loss if reduce else None), gD, gN

    def backward(self, center, quat, radii, lam, g_depth, g_normal, diagnostics: bool = False):
        K = int(center.shape[0])
        gc = torch.empty(K, 3, dtype=torch.float32, device=self.device)
        gq = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        gr = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        prm = self.params.c()
        if diagnostics:
            prm.flags |= 64
        check(self.lib.plane_render_bwd(C.byref(self.L), _ptr(self.ws), _ptr(center), _ptr(quat), _ptr(radii), K,
                                        _ptr(self.cams), self.n_cams, _ptr(lam), C.byref(prm),
                                        _ptr(g_depth.contiguous()), _ptr(g_normal.contiguous()),
                                        _ptr(gc), _ptr(gq), _ptr(gr), _stream()))
        return gc, gq, gr

    def backward_adam(self, center, quat, radii, lam, g_depth, g_normal, m, v, step, lr=(1e-3, 1e-3, 1e-3),
                      betas=(0.9, 0.999), eps=1e-8, r_min=1e-4, loss=None):
        """backward() followed by adam_step_planes in the same launches
        (plane_render_bwd_adam): center, quat, radii, m and v are updated in
        place, the gradients returned; with loss ([jobs, 4] float32 device)
        also the loss sums of the last forward_loss(reduce=False)."""
        K = int(center.shape[0])
        gc = torch.empty(K, 3, dtype=torch.float32, device=self.device)
        gq = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        gr = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        prm = self.params.c()
        check(self.lib.plane_render_bwd_adam(C.byref(self.L), _ptr(self.ws), _ptr(center), _ptr(quat), _ptr(radii), K,
                                             _ptr(self.cams), self.n_cams, _ptr(lam), C.byref(prm),
                                             _ptr(g_depth.contiguous()), _ptr(g_normal.contiguous()), _ptr(gc),
                                             _ptr(gq), _ptr(gr), _ptr(m), _ptr(v), _ptr(step), lr[0], lr[1], lr[2],
                                             betas[0], betas[1], eps, r_min, _ptr(loss), _stream()))
        return gc, gq, gr

    def step(self, tgt_depth, tgt_normal, m, v, step, tgt_off=None, mask=None, a_cos=5.0, a_nl1=5.0, a_d=1.0,
             lr=(1e-3, 1e-3, 1e-3), betas=(0.9, 0.999), eps=1e-8, r_min=1e-4, loss=None, maps: bool = True):
        """forward_loss(reduce=False) then backward_adam(loss=...) in one
        render launch (plane_render_step), on the planes last projected:
        planes, m and v updated in place; returns depth, normal, g_depth,
        g_normal and the gradients, the bits of the two calls.  maps=False:
        depth, normal, g_depth and g_normal are not written (None)."""
        center, quat, radii, lam = self._inputs
        K = int(center.shape[0])
        P = self.n_pixels
        depth = torch.empty(P, dtype=torch.float32, device=self.device) if maps else None
        normal = torch.empty(3 * P, dtype=torch.float32, device=self.device) if maps else None
        gD = torch.empty_like(depth) if maps else None
        gN = torch.empty_like(normal) if maps else None
        gc = torch.empty(K, 3, dtype=torch.float32, device=self.device)
        gq = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        gr = torch.empty(K, 4, dtype=torch.float32, device=self.device)
        prm = self.params.c()
        n_tgt = 0 if tgt_off is None else int(tgt_off.numel())
        check(self.lib.plane_render_step(C.byref(self.L), _ptr(self.ws), _ptr(center), _ptr(quat), _ptr(radii), K,
                                         _ptr(self.cams), self.n_cams, _ptr(lam), C.byref(prm), _ptr(depth),
                                         _ptr(normal), _ptr(tgt_depth), _ptr(tgt_normal), _ptr(mask), _ptr(tgt_off),
                                         n_tgt, a_cos, a_nl1, a_d, _ptr(gD), _ptr(gN), _ptr(gc), _ptr(gq), _ptr(gr),
                                         _ptr(m), _ptr(v), _ptr(step), lr[0], lr[1], lr[2], betas[0], betas[1], eps,
                                         r_min, _ptr(loss), _stream()))
        return depth, normal, gD, gN, gc, gq, gr

    def counters(self):
        out = (C.c_int64 * 20)()
        check(self.lib.ps_read_counters(C.byref(self.L), _ptr(self.ws), out, _stream()))
        return dict(pairs=out[0], overflow=out[1], max_tile=out[2], slow_pixels=out[3], big_tiles=out[4],
                    bwd_extra_passes=out[5], evals=out[6], commits=out[7], steps=out[8], max_steps=out[9],
                    wave_ticks=out[10], max_wave_ticks=out[11], bwd_ticks_setup=out[12], bwd_ticks_walk=out[13],
                    bwd_ticks_sort=out[14], bwd_ticks_grad=out[15], bwd_grad_candidates=out[16],
                    bwd_grad_groups=out[17], overflow_since_init=out[18], bwd_max_block_ticks=out[19])

    def block_stats(self) -> torch.Tensor:
        """Per-8x8-block statistics of the last renders run with diagnostics
        [n_items, 16] int64: evals, commits, steps, forward ticks, backward
        set-up / walk / sort / gradient ticks, gradient candidates and groups,
        backward ticks (100 MHz ticks)."""
        n = int(self.L.n_items)
        return self.region(18, torch.int64, 16 * n).view(n, 16)

    # ------------------------------------------------------------------ image views
    def job_depth(self, depth, s):
        j = self.jobs[s]
        o = self.pix_off[s]
        return depth[o:o + j.width * j.height].view(j.height, j.width)

    def job_normal(self, normal, s):
        j = self.jobs[s]
        o = self.pix_off[s]
        return normal[3 * o:3 * (o + j.width * j.height)].view(3, j.height, j.width)


def adam_step(center, quat, radii, g_center, g_quat, g_radii, m, v, step, lr=(1e-3, 1e-3, 1e-3),
              betas=(0.9, 0.999), eps=1e-8, r_min=1e-4):
    """In-place Adam on the plane parameters (adam_step_planes)."""
    lib = _lib.load()
    check(lib.adam_step_planes(_ptr(center), _ptr(quat), _ptr(radii), _ptr(g_center), _ptr(g_quat),
                               _ptr(g_radii), _ptr(m), _ptr(v), int(center.shape[0]), _ptr(step),
                               lr[0], lr[1], lr[2], betas[0], betas[1], eps, r_min, _stream()))


def tie_radii(g_radii):
    """Single-direction radii: g[x+] = g[x-] = their sum, likewise y
    (plane_tie_radii), in place."""
    lib = _lib.load()
    check(lib.plane_tie_radii(_ptr(g_radii), int(g_radii.shape[0]), _stream()))


def grad_accumulate(g_radii, acc, cnt):
    """acc += |g_radii|, cnt += 1 where the radii gradient is not all zero
    (plane_grad_accumulate)."""
    lib = _lib.load()
    check(lib.plane_grad_accumulate(_ptr(g_radii), _ptr(acc), _ptr(cnt), int(g_radii.shape[0]), _stream()))


def split_planes(center, quat, radii, acc, cnt, scale=None, thresh: float = 0.2):
    """Plane splitting (plane_split): (center, quat, radii, parent, first) of
    the new plane set, trimmed to its size (one host read of the count).
    scale: per-plane device float tensor (summed loss -> per-pixel mean), or
    None for 1."""
    lib = _lib.load()
    K = int(center.shape[0])
    dev = center.device
    oc = torch.empty(4 * K, 3, dtype=torch.float32, device=dev)
    oq = torch.empty(4 * K, 4, dtype=torch.float32, device=dev)
    orr = torch.empty(4 * K, 4, dtype=torch.float32, device=dev)
    parent = torch.empty(4 * K, dtype=torch.int32, device=dev)
    first = torch.empty(K + 1, dtype=torch.int32, device=dev)
    k_out = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(K + 1, dtype=torch.int32, device=dev)
    check(lib.plane_split(_ptr(center), _ptr(quat), _ptr(radii), _ptr(acc), _ptr(cnt), _ptr(scale), float(thresh), K,
                          _ptr(oc), _ptr(oq), _ptr(orr), _ptr(parent), _ptr(first), _ptr(k_out), _ptr(ws),
                          _stream()))
    n = int(k_out.item())
    return oc[:n].contiguous(), oq[:n].contiguous(), orr[:n].contiguous(), parent[:n].contiguous(), first


def valu_probe(kind: int, blocks: int = 8192, iters: int = 4096, reps: int = 3):
    """Measured vector-ALU issue rate in T lane-op/s (ps_valu_probe; kind 0
    fp32, 1 fp64): the best of `reps` timed launches on the current stream,
    after one untimed launch.  Returns (rate, sink tensor)."""
    lib = _lib.load()
    dt = torch.float32 if kind == 0 else torch.float64
    sink = torch.empty(blocks * 256, dtype=dt, device="cuda")
    nbytes = sink.numel() * sink.element_size()
    st = torch.cuda.current_stream()
    check(lib.ps_valu_probe(kind, blocks, iters, _ptr(sink), nbytes, _stream()))
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        check(lib.ps_valu_probe(kind, blocks, iters, _ptr(sink), nbytes, _stream()))
        e1.record(st)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return blocks * 256 * iters * 8 / best / 1e12, sink


def check_finite(*tensors) -> int:
    """Number of NaN or infinite values in the given float32 device tensors
    (ps_check_finite; synchronises the stream)."""
    lib = _lib.load()
    if not tensors:
        return 0
    d = torch.empty(1, dtype=torch.int64, device=tensors[0].device)
    total = 0
    for t in tensors:
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("check_finite: contiguous float32 tensors only")
        h = C.c_int64(0)
        check(lib.ps_check_finite(_ptr(t), int(t.numel()), _ptr(d), C.byref(h), _stream()))
        total += int(h.value)
    return total
