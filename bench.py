"""Benchmark of the plane-splatting fitting step on one MI355X.

Workload (single synthetic room, the configuration the headline metric is
quoted on): a 6 x 5 x 3 m box room with 40 furniture boxes whose faces are
split into ~2000 ground-truth rectangles; the fitted planes start from the
ground truth with center noise 0.1 m, rotation noise 10 deg and radii scaled
U[0.7, 1.3]; 100 views of 640 x 480 px (f = 577) on a random path; targets are
the ground truth rendered at lambda = 300.  One step = one fitting iteration
on `--views` views: plane_project -> tile_bin -> plane_render_fwd ->
loss_depth_normal -> plane_render_bwd -> adam_step_planes, lambda(ite) from
Eq. 10, every view used once per 100/views steps (shuffled cycle).

Metric: fwd+bwd Mpixel.planes/s = (pixels of the step) * K / step time / 1e6,
with the whole step (Adam included) inside the timed region and all inputs
resident in HBM.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
MI355X_FP64_VECTOR_TFLOPS = 78.6   # = non-packed fp32 FMA rate; packed fp32 is not used

# Algorithmic flops per composited (pixel, plane) hit (Sec. 3.2 arithmetic):
#   ray-plane intersection and in-plane coordinates (Eq. 4, 6): den (2 FMA),
#   t = h/den (1 div), x = o + t d (3 FMA), x - p (3), P_X, P_Y (2 x 3 FMA) -> 26
#   splat weight (Eq. 7-9): 2 |P|, 2 subtractions, min, sigmoid (exp, add, div) -> 8
#   compositing (Eq. 11-13): T w, D += T w t, N += T w n (3 FMA), T *= 1 - w -> 12
FLOPS_FWD_PER_HIT = 46
# backward per composited hit: recompute (46) + suffix walk (4) + chain to 13
# accumulators (~30) -> 80, plus the wave reduction of the accumulators
FLOPS_BWD_PER_HIT = 80


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(n_views: int, seed: int = 0):
    import synth
    gt, info = synth.room_planes(seed=seed, target_K=2000)
    init = synth.room_init_planes(gt, seed=seed + 1)
    cams = synth.room_trajectory(seed=seed, n_views=n_views, info=info)
    return gt, init, cams, info


def cpu_baseline(init, cams, lam, budget_s: float = 20.0):
    """The float64 oracle on a bounded sample of one view: forward + loss +
    backward for a block of pixel rows, timed on the host cores."""
    import torch
    import oracle
    torch.set_num_threads(os.cpu_count() or 1)
    cam = cams[0]
    rows = 2
    rng = np.random.default_rng(0)
    P = cam.width * cam.height
    Dt = torch.as_tensor(rng.uniform(1, 4, size=P))
    Nt = torch.as_tensor(rng.normal(size=(P, 3)))
    done_px = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        j0 = (done_px // cam.width) % cam.height
        pix = torch.arange(j0 * cam.width, min(P, (j0 + rows) * cam.width))
        c, q, r = (torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in (init.center, init.quat, init.radii))
        D, N, _ = oracle.render_pixels(c, q, r, cam, lam, pix)
        L = (D - Dt[pix]).abs().sum() + 5 * (1 - (N * Nt[pix]).sum(1)).abs().sum() + 5 * (N - Nt[pix]).abs().sum()
        L.backward()
        done_px += pix.numel()
    dt = time.perf_counter() - t0
    return {
        "value": done_px * init.K / dt / 1e6,
        "unit": "Mpixel*planes/s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": f"{done_px} pixels (rows of view 0, 640x480) x {init.K} planes, float64 forward+loss+backward, "
                  f"{dt:.1f} s on {os.cpu_count()} host cores ({platform.processor() or platform.machine()})",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--views", type=int, default=1, help="views per fitting step")
    ap.add_argument("--tile", type=int, nargs=2, default=(16, 16))
    ap.add_argument("--start-ite", type=int, default=0)
    ap.add_argument("--pending", type=int, default=6, choices=(4, 6, 8, 12),
                    help="pending-hit buffer size of the render kernels")
    ap.add_argument("--force-rounds", action="store_true",
                    help="send every pixel through the exact round-based ordering path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): scenes shard across GPUs "
              f"without communication, so the per-GPU number is the whole story", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_03451_amd.splat import Job, Renderer, SplatParams, adam_step
    import oracle  # noqa: F401  (only for lambda_at and the cpu baseline leg)
    from oracle import lambda_at

    n_views = 100
    V = args.views
    assert n_views % V == 0
    log(f"building room workload ({n_views} views)")
    gt, init, cams, info = build_workload(n_views)
    K = init.K
    W, H = cams[0].width, cams[0].height
    rng = np.random.default_rng(0)
    order = rng.permutation(n_views)
    cams_sched = [cams[i] for i in order]
    dev = torch.device("cuda")

    def T(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)

    # targets: ground truth rendered at lambda = 300 by the parity-tested forward
    log("rendering targets")
    tr = Renderer([Job(0, K, i, W, H, tuple(args.tile)) for i in range(n_views)], cams_sched,
                  pair_capacity=1 << 22)
    lam300 = torch.tensor([300.0], device=dev)
    tgt_d, tgt_n = tr.render(T(gt.center), T(gt.quat), T(gt.radii), lam300)
    tgt_d = tgt_d.view(n_views, H * W)
    tgt_n = tgt_n.view(n_views, 3 * H * W)
    del tr

    # fitting state
    c, q, r = T(init.center), T(init.quat), T(init.radii)
    m = torch.zeros(11 * K, device=dev)
    v = torch.zeros(11 * K, device=dev)
    step_t = torch.zeros(1, dtype=torch.int32, device=dev)
    lam_t = torch.zeros(1, device=dev)
    view_t = torch.zeros(V, dtype=torch.int32, device=dev)
    sched = torch.arange(n_views, dtype=torch.int32, device=dev)
    rend = Renderer([Job(0, K, s, W, H, tuple(args.tile)) for s in range(V)], cams_sched,
                    pair_capacity=1 << 20,
                    params=SplatParams(flags=({6: 0, 4: 1, 8: 2, 12: 3}[args.pending] << 4)
                                       | (1 if args.force_rounds else 0)))
    lib = rend.lib
    import ctypes as C
    from paper_2412_03451_amd.splat import _ptr, _stream

    ev = {k: [] for k in ("project", "bin", "fwd", "loss", "bwd", "adam")}

    def one_step(it, timed):
        blk = (it * V) % n_views
        view_t.copy_(sched[blk:blk + V])
        lam_t.fill_(lambda_at(args.start_ite + it))
        step_t.fill_(it + 1)
        lib.ps_set_cameras(C.byref(rend.L), _ptr(rend.ws), _ptr(view_t), _stream())
        marks = []

        def mark():
            if timed:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                marks.append(e)
        mark()
        rend.project(c, q, r, lam_t)
        mark()
        rend.bin(check_capacity=False)
        mark()
        D, N = rend.forward()
        mark()
        loss, gD, gN = rend.loss(D, N, tgt_d[blk:blk + V].reshape(-1), tgt_n[blk:blk + V].reshape(-1))
        mark()
        gc, gq, gr = rend.backward(c, q, r, lam_t, gD, gN)
        mark()
        adam_step(c, q, r, gc, gq, gr, m, v, step_t)
        mark()
        return marks, loss

    # capacity: size the pair buffers once (the first step checks and grows)
    view_t.copy_(sched[0:V])
    lib.ps_set_cameras(C.byref(rend.L), _ptr(rend.ws), _ptr(view_t), _stream())
    lam_t.fill_(lambda_at(args.start_ite))
    rend.project(c, q, r, lam_t)
    rend.bin(check_capacity=True, grow=2.0)
    log(f"pairs {rend.last_pairs}, capacity {rend.L.pair_capacity}")

    log(f"warmup {args.warmup} steps")
    for it in range(args.warmup):
        one_step(it, False)
    torch.cuda.synchronize()
    cnt = rend.counters()
    if cnt["overflow"]:
        raise RuntimeError(f"pair capacity exceeded during warmup: {cnt}")
    # reset the fit so the timed steps start at the same state
    c.copy_(T(init.center)); q.copy_(T(init.quat)); r.copy_(T(init.radii))
    m.zero_(); v.zero_()

    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    all_marks = []
    start.record()
    for it in range(args.steps):
        marks, loss = one_step(it, True)
        all_marks.append(marks)
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    ms_step = total_ms / args.steps
    names = list(ev)
    for marks in all_marks:
        for i, n in enumerate(names):
            ev[n].append(marks[i].elapsed_time(marks[i + 1]))
    phase_ms = {n: float(np.mean(x)) for n, x in ev.items()}
    cnt = rend.counters()
    if cnt["overflow"]:
        raise RuntimeError(f"pair capacity exceeded: {cnt}")

    # diagnostics pass (untimed): composited hits of the last step's views
    D, N, Tr, Cn = rend.forward(diagnostics=True)
    torch.cuda.synchronize()
    hits = int(Cn.sum().item())
    cnt = rend.counters()
    evals = int(cnt["evals"])

    pix = V * W * H
    value = pix * K / (ms_step * 1e-3) / 1e6
    # roofline of the dominant kernel
    dom = max(("fwd", "bwd"), key=lambda n: phase_ms[n])
    per_hit = FLOPS_FWD_PER_HIT if dom == "fwd" else FLOPS_BWD_PER_HIT
    achieved = hits * per_hit / (phase_ms[dom] * 1e-3) / 1e12
    roof = {
        "kernel": "render_fwd_kernel" if dom == "fwd" else "render_bwd_kernel+bwd_reduce_kernel",
        "bound": "alu",
        "achieved": round(achieved, 4),
        "peak": MI355X_FP64_VECTOR_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / MI355X_FP64_VECTOR_TFLOPS, 5),
        "traffic": None,
        "algorithmic_units": f"{hits} composited hits x {per_hit} flops",
        "pairs_evaluated": evals,
    }
    out = {
        "metric": "fwd+bwd Mpixel*planes/s",
        "value": round(value, 1),
        "unit": "Mpixel*planes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 ray-plane geometry)",
        "data": "synthetic",
        "config": {"workload": f"single room, K={K} planes, {V} view(s)/step of 640x480, f=577, "
                               f"tile {args.tile[0]}x{args.tile[1]}, lambda from ite {args.start_ite}",
                   "planes": K, "views_per_step": V, "width": W, "height": H,
                   "pairs_per_step": int(cnt["pairs"])},
        "phase_ms": {k: round(x, 4) for k, x in phase_ms.items()},
        "render_stats": {"pending": args.pending, "composited_hits": hits, "pairs_evaluated": evals,
                         "round_path_pixels": int(cnt["slow_pixels"]),
                         "bwd_extra_passes": int(cnt["bwd_extra_passes"])},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (float64 oracle on a pixel sample)")
        out["cpu_baseline"] = cpu_baseline(init, cams, lambda_at(args.start_ite), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
