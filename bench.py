"""Benchmark of the plane-splatting fitting step on one MI355X.

Workload (single synthetic room, the configuration the headline metric is
quoted on): a 6 x 5 x 3 m box room with 40 furniture boxes whose faces are
split into ~2000 ground-truth rectangles; the fitted planes start from the
ground truth with center noise 0.1 m, rotation noise 10 deg and radii scaled
U[0.7, 1.3]; 100 views of 640 x 480 px (f = 577) on a random path; targets are
the ground truth rendered at lambda = 300.  One step = one fitting iteration
on `--views` views: ps_fit_schedule (device-side lambda of Eq. 10, Adam step,
view of the step from a shuffled cycle) -> plane_project -> tile_bin ->
plane_render_step (forward, loss of Eq. 14, backward and the Adam update of
the planes: one render launch, then the per-plane reduction that applies the
update), captured once in a HIP graph and replayed.  --separate-calls times
the same step as plane_render_fwd_loss + plane_render_bwd_adam.

Metric: fwd+bwd Mpixel.planes/s = (pixels of the step) * K / step time / 1e6,
with the whole replayed step (Adam included) inside the timed region and all
inputs resident in HBM.  By default the timed steps are the room's whole
5000-iteration fit from its start (lambda rising from 7.4 to 300 by Eq. 10);
the first 200 steps, the slowest (widest fringes), are reported beside it.
Per-kernel durations come from steps sampled evenly over the same
trajectory, run eagerly with events between the phases.  Prints one JSON
line.
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
# Vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane
# operations per second (one non-packed fp32 or fp64 operation per lane per
# cycle; packed fp32 is not used; an FMA counts as one operation).
MI355X_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work of the render kernels, in lane operations (Sec. 3.2):
#   per evaluated (pixel, candidate) pair: three affine forms in the pixel
#   (den, and the numerators of P_X, P_Y), the reciprocal of den, t, P_X, P_Y,
#   branch radii, |P|, two differences, the minimum, the filter test
#   -> about 16 operations and 1 transcendental
OPS_PER_EVAL = 17
#   per composited hit: the weight (exp, reciprocal, ~4 operations), the
#   compositing of depth, normal and transmittance (~6), the ordered insertion (~4)
OPS_PER_HIT_FWD = 16
#   backward: the forward's work twice (the walk that recomputes the
#   committed sequence, then every committed hit evaluated again for its
#   gradient), 2 x 17 per evaluated pair and 2 x 16 per composited hit, plus
#   the chain rule to the 13 per-pair accumulators (~40 per hit)
OPS_PER_EVAL_BWD = 2 * OPS_PER_EVAL
OPS_PER_HIT_BWD = 2 * OPS_PER_HIT_FWD + 40


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(n_views: int, seed: int = 0):
    import synth
    gt, info = synth.room_planes(seed=seed, target_K=2000)
    init = synth.room_init_planes(gt, seed=seed + 1)
    cams = synth.room_trajectory(seed=seed, n_views=n_views, info=info)
    return gt, init, cams, info


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_rate(init, cam, lam, budget_s: float, threads: int):
    """Pixels x planes per second of the float64 oracle (forward + loss +
    backward) on blocks of two pixel rows of one view, for `budget_s`."""
    import torch
    import oracle
    torch.set_num_threads(threads)
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
    return done_px * init.K / dt, done_px, dt, torch.get_num_threads()


def oracle_small_step_s(reps: int = 3, K: int = 64, width: int = 128, height: int = 96, f: float | None = None):
    """Seconds of one whole float64 oracle step on a small configuration
    (default 64 planes, 128x96; 256 planes at 256x192, f = 200, for the
    differentiation-check configuration), lambda(0): render, Eq. 14 loss
    against the perturbed scene's render, backward and one Adam step; best
    of `reps`."""
    import torch
    import oracle
    import synth
    ps = synth.random_planes(K, seed=0, independent_radii=True)
    tgt = synth.perturb_planes(ps, seed=1, center_sigma=0.05, rot_sigma_deg=5.0)
    cam = synth.tiny_camera() if f is None else synth.tiny_camera(width, height, f)
    lam = float(np.float32(oracle.lambda_at(0)))
    Dt, Nt, _ = oracle.render(tgt.center, tgt.quat, tgt.radii, cam, 300.0)
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        c, q, r = (torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in (ps.center, ps.quat, ps.radii))
        D, N, _ = oracle.render(c, q, r, cam, lam)
        oracle.render_loss(D, N, Dt, Nt).backward()
        for x in (c, q, r):
            z = np.zeros(tuple(x.shape))
            oracle.adam_step(x.detach().numpy(), x.grad.numpy(), z, z, 1)
        best = min(best, time.perf_counter() - t0)
    return best


def small_config_rates():
    """The oracle's whole step, in full, on the two small configurations:
    64 planes at 128x96 and 256 planes at 256x192 (f = 200), as
    Mpixel*planes/s with the GPU's formula."""
    out = {}
    for name, K, W, H, f in (("64 planes, 128x96", 64, 128, 96, None), ("256 planes, 256x192", 256, 256, 192, 200.0)):
        t = oracle_small_step_s(reps=2, K=K, width=W, height=H, f=f)
        out[name] = {"step_s": round(t, 3), "value": round(W * H * K / t / 1e6, 2), "unit": "Mpixel*planes/s"}
    return out


def cpu_baseline(init, cams, lam, budget_s: float = 20.0):
    """The float64 oracle on a bounded sample of one view: forward + loss +
    backward for blocks of pixel rows, timed on the host cores (three
    quarters of the budget on every core, the rest on one core)."""
    import torch
    cam = cams[0]
    n = os.cpu_count() or 1
    rate, px, dt, used = _oracle_rate(init, cam, lam, 0.75 * budget_s, n)
    rate1, px1, dt1, _ = _oracle_rate(init, cam, lam, 0.25 * budget_s, 1)
    torch.set_num_threads(n)
    step_s = cam.width * cam.height * init.K / rate
    return {
        "value": rate / 1e6,
        "unit": "Mpixel*planes/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{px} pixels (rows of view 0, {cam.width}x{cam.height}) x {init.K} planes, float64 "
                  f"forward+loss+backward, {dt:.1f} s on {used} threads of {n} host cores ({cpu_model()})",
        "value_1_thread": rate1 / 1e6,
        "sample_1_thread": f"{px1} pixels in {dt1:.1f} s on one thread",
        "fit_5000_steps_s_extrapolated": round(5000 * step_s, 1),
        "small_config_step_s": round(oracle_small_step_s(), 3),
        "configs": small_config_rates(),
    }


def culling_efficiency(init, cams, lam, tile, n_pix: int = 4096, seed: int = 0):
    """Culling efficiency N_need / N_eval of the forward on view 0 at the
    start state: N_eval is the forward's own count of evaluated (pixel,
    plane) pairs over the whole view (its diagnostics), N_need the pairs a
    ray needs (every kept hit up to and including its first opaque one, from
    the float64 oracle) on a seeded uniform sample of n_pix pixels, scaled to
    the view."""
    import torch
    import oracle
    from paper_2412_03451_amd.splat import Job, Renderer
    cam = cams[0]
    W, H = cam.width, cam.height
    rend = Renderer([Job(0, init.K, 0, W, H, tuple(tile))], cams, pair_capacity=1 << 22)
    T = [torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")
         for x in (init.center, init.quat, init.radii)]
    rend.render_diag(*T, torch.tensor([lam], dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    n_eval = int(rend.counters()["evals"])
    del rend
    pix = np.sort(np.random.default_rng(seed).choice(W * H, size=n_pix, replace=False))
    t0 = time.perf_counter()
    _, _, aux = oracle.render_pixels(init.center, init.quat, init.radii, cam, float(np.float32(lam)), pix)
    need = float(aux["need"].double().mean()) * W * H
    return {"n_need": round(need), "n_eval": n_eval, "frac": round(need / max(1, n_eval), 4),
            "sample": f"view 0 ({W}x{H}) at iteration 0; N_need from the float64 oracle on {n_pix} seeded "
                      f"uniform pixels ({time.perf_counter() - t0:.1f} s), scaled to the view; N_eval over every "
                      f"pixel of the view"}


KERNEL_SOURCES = ("paper_2412_03451_amd/csrc/render.hip", "paper_2412_03451_amd/csrc/ps_internal.h",
                  "paper_2412_03451_amd/csrc/adam.hip")
TRAFFIC_FILES = {"fwd": "profiles/render_fwd_room640_hbm_traffic.txt",
                 "bwd": "profiles/render_bwd_room640_hbm_traffic.txt",
                 "step": "profiles/render_step_room640_hbm_traffic.txt"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_key(args) -> str:
    """The bench arguments that decide the render launches of the timed steps."""
    return (f"--steps {args.steps} --start-ite {args.start_ite} --views {args.views} "
            f"--tile {args.tile[0]} {args.tile[1]} --pending {args.pending}"
            + (" --force-rounds" if args.force_rounds else "")
            + (" --separate-calls" if getattr(args, "separate_calls", False) else ""))


def measured_traffic(phase: str, key: str):
    """HBM bytes per launch of the render kernel from the committed counter
    summary, if it was taken on the current kernel source over the same
    steps (bench arguments `key`), else None."""
    path = os.path.join(ROOT, TRAFFIC_FILES[phase])
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash() or vals.get("bench_args") != key:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


MI355X_BF16_DENSE_TFLOPS = 2500.0


def initnet_bench(args):
    """The learned initializer's training step in its per-view form: a batch
    of 32 views, 4096 back-projected depth samples each, 256 proposals per
    view (width 256, bfloat16 MFMA, float32 accumulation), ~30 target planes
    per view.  Forward (fused point layers on MFMA + head), set loss,
    backward and Adam timed with events over --steps repetitions.
    Algorithmic MFMA work of the forward: 2 x 256 x 256 x 2 flops per point
    (layers 2 and 3)."""
    import torch
    from paper_2412_03451_amd.initnet import InitNet
    B, N, P, T = 32, 4096, 256, 30
    rng = np.random.default_rng(0)
    # points of a view: a box room seen from inside (camera frame, z forward)
    X = np.stack([rng.uniform(-2, 2, (B, N)), rng.uniform(-1.5, 1.5, (B, N)), rng.uniform(0.5, 5.0, (B, N))], -1)
    X = torch.tensor(X.astype(np.float32), device="cuda")
    q = rng.normal(size=(B * T, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    tgt = np.concatenate([rng.uniform(-2, 2, (B * T, 3)), q, rng.uniform(0.05, 1.0, (B * T, 4))], 1)
    tgt = torch.tensor(tgt.astype(np.float32), device="cuda")
    off = torch.tensor(np.arange(B + 1, dtype=np.int32) * T, device="cuda")
    net = InitNet(P, seed=0)
    for _ in range(3):
        g, arg, out = net.forward(X)
        loss, d_out = net.set_loss(out, tgt, off)
        net.adam_step(net.backward(X, g, arg, d_out))
    st = torch.cuda.current_stream()
    names = ("fwd", "set_loss", "bwd", "adam")
    acc = {n: 0.0 for n in names}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(st)
        g, arg, out = net.forward(X)
        ev[1].record(st)
        loss, d_out = net.set_loss(out, tgt, off)
        ev[2].record(st)
        grad = net.backward(X, g, arg, d_out)
        ev[3].record(st)
        net.adam_step(grad)
        ev[4].record(st)
        torch.cuda.synchronize()
        for i, n in enumerate(names):
            acc[n] += ev[i].elapsed_time(ev[i + 1])
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    ms = {n: acc[n] / args.steps for n in names}
    fwd_flops = B * N * 2 * 256 * 256 * 2
    ach = fwd_flops / (ms["fwd"] * 1e-3) / 1e12
    step_ms = sum(ms.values())
    return {
        "metric": "learned-initializer training step", "value": round(B / (step_ms * 1e-3), 1),
        "unit": "views/s", "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
        "dtype": "bf16 (f32 accumulate)", "data": "synthetic",
        "config": {"workload": f"{B} views x {N} depth samples, width 256, {P} proposals per view, {T} targets per view"},
        "ms": {n: round(x, 4) for n, x in ms.items()}, "step_ms": round(step_ms, 4), "wall_ms_per_step": round(wall, 4),
        "roofline": {"kernel": "initnet fwd_kernel + head_kernel", "bound": "mfma", "achieved": round(ach, 2),
                     "peak": MI355X_BF16_DENSE_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / MI355X_BF16_DENSE_TFLOPS, 4)},
    }


def batched_bench(args):
    """Batched fitting step: --rooms synthetic rooms of uneven size (plane
    counts log-uniform in [200, 4000], 20-100 views, 320x240 or 640x480),
    every room advancing one iteration (one view) per step, all in one
    graph-replayed step of one launch per phase.  The tile shape from the
    autotuner (the batch's own steps timed with each shape; --no-autotune:
    16x16).  Value: sum over rooms of (pixels x planes) per second of step
    time."""
    import torch
    import synth
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd.autotune import Autotuner
    from paper_2412_03451_amd.fit import BatchFit, FitConfig, Scene

    specs = synth.room_batch_specs(args.rooms, seed=0)
    tuner = Autotuner(os.path.join(ROOT, "_build", "tune.json")) if args.autotune else None
    scenes, work = [], 0
    for sp in specs:
        gt, info = synth.room_planes(seed=sp["seed"], target_K=sp["K"])
        init = synth.room_init_planes(gt, seed=sp["seed"] + 1)
        cams = synth.room_trajectory(sp["seed"], sp["views"], info, width=sp["width"], height=sp["height"],
                                     f=sp["f"])
        tD, tN = li.render_targets((gt.center, gt.quat, gt.radii), cams)
        sc = Scene(init.center, init.quat, init.radii, cams, tD, tN)
        scenes.append(sc)
        work += sp["width"] * sp["height"] * gt.K
    log(f"{len(scenes)} rooms ready")
    from paper_2412_03451_amd.splat import SplatParams
    params = SplatParams(flags=256 if args.per_item_launch else 0)
    tile_times = None
    if tuner is not None:
        # one tile shape for the batch, from timing the batch's own steps with each shape
        tile, tile_times = tuner.tune_batch(scenes, cfg=FitConfig(one_launch=not args.separate_calls),
                                            params=params)
        for sc in scenes:
            sc.tile = tile
        log(f"tile shape {tile}: {tile_times}")
    fit = BatchFit(scenes, cfg=FitConfig(check_every=max(1, args.warmup), one_launch=not args.separate_calls),
                   params=params)
    fit.size_capacity()
    start_state = fit.state()
    fit.run(max(1, args.warmup), graph=True)
    fit.restore(start_state)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        fit.graph.replay()
    e1.record(st)
    torch.cuda.synchronize()
    if fit.overflowed():
        raise RuntimeError("pair capacity exceeded during the timed batched steps")
    ms = e0.elapsed_time(e1) / args.steps
    # the same steps again, phase by phase, with the render statistics
    fit.restore(start_state)
    phase_ms, _, cnt = sample_phases(fit, args.steps, min(args.phase_steps, args.steps), st)
    roof, hits, evals = render_roofline(phase_ms, cnt)
    tiles = {}
    for sc in scenes:
        k = f"{sc.tile[0]}x{sc.tile[1]}" if sc.tile else "16x16"
        tiles[k] = tiles.get(k, 0) + 1
    return {
        "metric": "fwd+bwd Mpixel*planes/s (batched fitting step)", "value": round(work / (ms * 1e-3) / 1e6, 1),
        "unit": "Mpixel*planes/s", "higher_is_better": True, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "dtype": "f32 (f64 ray-plane geometry)", "data": "synthetic",
        "config": {"workload": f"{len(scenes)} rooms, K log-uniform 200-4000, 20-100 views, 320x240 or 640x480, "
                               f"one view per room per step, lambda from ite 0", "rooms": len(scenes),
                   "launch": "one workgroup per 8x8 block" if args.per_item_launch else
                             "persistent (atomic work queue) where the blocks exceed 4x the resident workgroups",
                   "planes": int(fit.K), "pixels_per_step": int(fit.rend.n_pixels), "tiles": tiles,
                   "tile_ms_tried": tile_times,
                   "pair_capacity": int(fit.rend.L.pair_capacity)},
        "phase_ms": {k: round(x, 4) for k, x in phase_ms.items()},
        "render_stats": {"composited_hits": hits, "pairs_evaluated": evals,
                         "hits_per_evaluated_pair": round(hits / max(1, evals), 4)},
        "roofline": roof,
    }


def memory_bench(args):
    """Peak device memory of one forward + backward through the autograd
    front end on a large room (K ~ 20000 planes, one 1296 x 968 view,
    f = 1168.4): the recompute backward against the list-storing variant
    (M = 30 entries of list position, a* and transmittance per pixel)."""
    import torch
    import synth
    from paper_2412_03451_amd.autograd import PlaneSplatFn, PlaneSplatListsFn
    from paper_2412_03451_amd.splat import Job, Renderer

    gt, info = synth.room_planes(seed=0, target_K=20000)
    init = synth.room_init_planes(gt, seed=1)
    cams = synth.room_trajectory(seed=0, n_views=4, info=info, width=1296, height=968, f=577.0 * 1296 / 640)
    cam = cams[1]
    dev = torch.device("cuda")

    def T(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)

    lam = torch.tensor([7.3576], device=dev)
    out = {"metric": "peak device memory of forward+backward, recompute vs stored per-pixel lists",
           "unit": "MiB", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"room, K={gt.K} planes, one 1296x968 view, lambda(0)", "planes": gt.K}}
    res = {}
    # pair lists sized for this view (the binning grows the workspace to 1.5x the need)
    probe = Renderer([Job(0, gt.K, 0, cam.width, cam.height, (16, 16))], [cam])
    probe.project(T(init.center), T(init.quat), T(init.radii), lam)
    probe.bin()
    cap = int(probe.L.pair_capacity)
    del probe
    for name, fn in (("recompute", PlaneSplatFn), ("stored_lists", PlaneSplatListsFn)):
        for rep in range(2):   # the first pass loads the kernels; the second is measured
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            base = torch.cuda.memory_allocated()
            r = Renderer([Job(0, gt.K, 0, cam.width, cam.height, (16, 16))], [cam], pair_capacity=cap)
            c, q, rr = (T(x).requires_grad_(True) for x in (init.center, init.quat, init.radii))
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            D, N = fn.apply(c, q, rr, lam, r)
            ev[1].record()
            (D.sum() + N.sum()).backward()
            ev[2].record()
            torch.cuda.synchronize()
            peak = torch.cuda.max_memory_allocated() - base
            res[name] = {"peak_mib": round(peak / 2**20, 1), "workspace_mib": round(r.ws.numel() / 2**20, 1),
                         "pairs": int(r.last_pairs), "pair_capacity": cap,
                         "fwd_ms": round(ev[0].elapsed_time(ev[1]), 3), "bwd_ms": round(ev[1].elapsed_time(ev[2]), 3),
                         "grad_center_sum": float(c.grad.double().abs().sum())}
            del r, D, N, c, q, rr
    out.update(res)
    out["value"] = res["stored_lists"]["peak_mib"]
    out["ratio_stored_over_recompute"] = round(res["stored_lists"]["peak_mib"] / res["recompute"]["peak_mib"], 3)
    out["same_gradient"] = res["recompute"]["grad_center_sum"] == res["stored_lists"]["grad_center_sum"]
    return out


def scene_fit_bench(args):
    """The second half of the metric: iterations and wall-time to a depth L1
    of --target-l1 (1 cm), batched fits from the learned initialisation
    against plain fits one room at a time.

    Rooms of the single-room configuration (K ~ 2000 planes, 100 views of
    640x480, f = 577).  The initializer (4096 samples per view -> 256
    proposals) is trained first on --train-rooms rooms fitted by the plain
    method (time reported, not counted).  Then --rooms held-out rooms: each
    is fitted alone from its noisy initialisation until its depth L1 over
    its views (lambda = 300) is at most the target, checked every
    --check-every iterations, for at most --fit-iters iterations; then all of
    them together in one batched fit from the learned initialisation, each
    room checked the same way and leaving the batch once it is there.  Wall-times exclude the checks; the batched
    side includes the initialisation (network inference, proposal decoding,
    refinement, the fallback check).  value = plain seconds / batched
    seconds, every room to the target or the cap on both sides (the same
    ratio over only the rooms both sides bring to the target is reported
    beside it)."""
    import torch
    import synth
    from paper_2412_03451_amd import view_init as vi
    from paper_2412_03451_amd.fit import BatchFit, FitConfig, Scene
    from paper_2412_03451_amd.initnet import InitNet

    W, H, F, K, V = 640, 480, 577.0, 2000, 100
    target, every, cap = args.target_l1, args.check_every, args.fit_iters

    def room(seed):
        gt, info = synth.room_planes(seed=seed, target_K=K)
        cams = synth.room_trajectory(seed, V, info, width=W, height=H, f=F)
        rm = {"gt": gt, "init": synth.room_init_planes(gt, seed=seed + 7919), "cams": cams}
        rm["tD"], rm["tN"] = vi.render_targets((gt.center, gt.quat, gt.radii), cams)
        return rm

    # training data: rooms fitted by the plain method, one view per sample
    t0 = time.perf_counter()
    data = vi.ViewData()
    for s0 in range(0, args.train_rooms, 8):
        batch = [room(1000 + i) for i in range(s0, min(args.train_rooms, s0 + 8))]
        fitted = vi.fit_rooms(batch, args.train_fit_iters)
        for j, (rm, fp) in enumerate(zip(batch, fitted)):
            data.add_room(rm, fp, seed=1000 + s0 + j)
        del batch
        torch.cuda.empty_cache()
    data_s = time.perf_counter() - t0
    log(f"training data: {len(data.X)} views of {args.train_rooms} rooms in {data_s:.1f} s")
    t0 = time.perf_counter()
    net = InitNet(vi.N_PROPOSALS, seed=0)
    hist = vi.train(net, data, args.train_steps, batch=32, lr=1e-3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del data
    torch.cuda.empty_cache()

    rooms = [room(5000 + i) for i in range(args.rooms)]
    # plain: one fit per room, until the target or the iteration cap
    plain_s, plain_its = [], []
    for i, rm in enumerate(rooms):
        init = (rm["init"].center, rm["init"].quat, rm["init"].radii)
        fit = BatchFit([Scene(*init, rm["cams"], rm["tD"], rm["tN"])], cfg=FitConfig(check_every=every))
        fit.size_capacity()
        start = fit.state()
        fit.run(1, graph=True)       # capture outside the timed region
        fit.restore(start)
        secs, its = 0.0, 0
        while its < cap:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fit.run(every, graph=True)
            torch.cuda.synchronize()
            secs += time.perf_counter() - t1
            its += every
            if fit.depth_l1(0, lam=300.0) <= target:
                break
        reached = its < cap or fit.depth_l1(0, lam=300.0) <= target
        plain_s.append(secs)
        plain_its.append(its if reached else None)
        del fit
    log(f"plain: {sum(x is not None for x in plain_its)} of {len(rooms)} rooms reach {target} m, "
        f"{sum(plain_s):.2f} s")
    def batched(scenes):
        """One batched fit of the scenes until each reaches the target (or the
        cap): per room the iterations to the target, and the cumulative fit
        seconds at every check.  A room that reaches the target leaves the
        batch (BatchFit.subset: the others carry on with their own state and
        schedule); building the smaller batch and capturing its step count
        as fit time."""
        fit = BatchFit(scenes, cfg=FitConfig(check_every=every))
        fit.size_capacity()
        start = fit.state()
        fit.run(1, graph=True)
        fit.restore(start)
        done_at = [None] * len(scenes)
        idx = list(range(len(scenes)))      # batch position -> room
        secs, its, cum = 0.0, 0, {0: 0.0}
        while its < cap and idx:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fit.run(every, graph=True)
            torch.cuda.synchronize()
            secs += time.perf_counter() - t2
            its += every
            reached = [p for p in range(len(idx)) if fit.depth_l1(p, lam=300.0) <= target]
            for p in reached:
                done_at[idx[p]] = its
            rest = [p for p in range(len(idx)) if p not in reached]
            if reached and rest and its < cap:
                t3 = time.perf_counter()
                fit = fit.subset(rest)
                torch.cuda.synchronize()
                secs += time.perf_counter() - t3
            idx = [idx[p] for p in rest]
            cum[its] = secs
        del fit
        torch.cuda.empty_cache()
        return done_at, cum

    # batched + learned initialisation
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scenes, used, infos = [], 0, []
    for i, rm in enumerate(rooms):
        init = (rm["init"].center, rm["init"].quat, rm["init"].radii)
        planes, info = vi.learned_init(net, init, rm["cams"], rm["tD"], seed=5000 + i, conf_min=args.conf_min,
                                       d_max=args.d_max)
        used += info["used"] == "learned"
        infos.append(info)
        scenes.append(Scene(*planes, rm["cams"], rm["tD"], rm["tN"]))
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t1
    done_at, cum = batched(scenes)
    both = [i for i in range(len(rooms)) if plain_its[i] is not None and done_at[i] is not None]
    # the batched side's time for the rooms both reach: the batched run until the last of them
    # reaches the target (the others ride along); the plain side: those rooms' own fits
    last = max((done_at[i] for i in both), default=0)
    total = init_s + cum[last]
    plain_both = sum(plain_s[i] for i in both)
    # the same batched fit from the plain initialisation: what the batching alone gives
    done_p, cum_p = batched([Scene(rm["init"].center, rm["init"].quat, rm["init"].radii, rm["cams"], rm["tD"],
                                   rm["tN"]) for rm in rooms])
    both_p = [i for i in range(len(rooms)) if plain_its[i] is not None and done_p[i] is not None]
    last_p = max((done_p[i] for i in both_p), default=0)
    # every room to the target or the cap, on both sides: the plain fits' total
    # against the batched run's whole length (rooms that never reach the
    # target run to the cap on both sides)
    plain_all = sum(plain_s)
    batched_all = init_s + cum[max(cum)]
    batched_p_all = cum_p[max(cum_p)]
    return {
        "metric": "scene-fit wall-time to depth L1 <= 1 cm, batched+init vs plain",
        "value": round(plain_all / batched_all, 3) if batched_all > 0 else None,
        "unit": "x (plain seconds / batched+init seconds, every room to the target or the iteration cap)",
        "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f32 (f64 ray-plane geometry)",
        "config": {"workload": f"{len(rooms)} held-out rooms of the single-room configuration (K~{K}, {V} views of "
                               f"{W}x{H}); target depth L1 {target} m (lambda 300), checked every {every} "
                               f"iterations, at most {cap}; initializer: {vi.N_POINTS} samples per view -> "
                               f"{vi.N_PROPOSALS} proposals, trained on {args.train_rooms} rooms fitted by the "
                               f"plain method", "rooms": len(rooms)},
        "rooms_reaching_target": {"plain": sum(x is not None for x in plain_its),
                                  "batched": sum(d is not None for d in done_at), "both": len(both)},
        "plain_seconds": round(plain_all, 3), "batched_init_seconds": round(batched_all, 3),
        "learned_init_seconds": round(init_s, 3), "batched_fit_seconds": round(batched_all - init_s, 3),
        "rooms_both_reach": {"value": round(plain_both / total, 3) if total > 0 else None,
                             "plain_seconds": round(plain_both, 3), "batched_init_seconds": round(total, 3)},
        "iterations_to_target": {"plain": plain_its, "batched": done_at},
        "iterations_to_target_median": {
            "plain": float(np.median([plain_its[i] for i in both])) if both else None,
            "batched": float(np.median([done_at[i] for i in both])) if both else None},
        "batched_plain_init": {
            "rooms_reaching_target": sum(d is not None for d in done_p), "both": len(both_p),
            "value": round(plain_all / batched_p_all, 3) if batched_p_all > 0 else None,
            "batched_seconds": round(batched_p_all, 3),
            "rooms_both_reach_value": round(sum(plain_s[i] for i in both_p) / cum_p[last_p], 3) if last_p else None,
            "iterations_to_target": done_p},
        "refinement": {"conf_min": args.conf_min, "d_max": args.d_max},
        "learned_init_used": used,
        "depth_l1_init_plain_mean": round(float(np.mean([x["depth_l1_plain_init"] for x in infos])), 4),
        "depth_l1_init_learned_mean": round(float(np.mean([x["depth_l1_learned_init"] for x in infos])), 4),
        "planes_refined_mean": round(float(np.mean([x["planes_refined"] for x in infos])), 1),
        "initializer": {"training_data_seconds": round(data_s, 1), "training_seconds": round(train_s, 1),
                        "set_loss": hist},
    }


def init_ablation_bench(args):
    """Plane-initialisation ablation on the synthetic room (the analogue of
    the paper's Sec. 4.3 comparison).  The default room (~2000 ground-truth
    rectangles, 100 views of 640 x 480, targets at lambda = 300) is fitted for
    --fit-iters iterations (one view per step, plane splitting every 1000
    iterations) from three initialisations of 2000 planes: from the depth
    maps (Sec. 3.1: fused points at stride 4 and 2 cm voxels), on the scene's
    bounding sphere (Sec. 4.3, radii 0.05), and the noisy ground truth of the
    throughput workload; the depth initialisation is also fitted without
    splitting, with single-direction radii (the plane-radii ablation) and with
    the Gaussian splat function of Eq. 5 in place of the rectangle one.  Each fit ends with the plane merge (Sec. 3.3, 25 degrees and
    0.1 cm), timed, with its instance count beside the ground truth's.  Depth L1 over all views at lambda = 300 every 500
    iterations; fit wall-times exclude the evaluations; the initialisation
    kernels are timed on their own."""
    import torch
    from paper_2412_03451_amd import learned_init as li
    from paper_2412_03451_amd import scene_init as si
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    from paper_2412_03451_amd.splat import SplatParams

    gt, init, cams, info = build_workload(100)
    V, W, H = len(cams), cams[0].width, cams[0].height
    tD, tN = li.render_targets((gt.center, gt.quat, gt.radii), cams)
    D, N = tD.view(V, H, W), tN.view(V, 3, H, W)
    K = 2000

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / reps * 1e3

    (pts, nrm, n), pts_ms = timed(lambda: si.depth_points(D, N, cams, 4, 0.02))
    rng = np.random.default_rng(0)
    sel = rng.choice(n, K, replace=False).astype(np.int32)
    depth_init, planes_ms = timed(lambda: si.init_from_points(pts, nrm, sel))
    sphere_init, sphere_ms = timed(lambda: si.init_sphere(pts, K, seed=0))
    log(f"depth_points: {n} fused points from {V} views in {pts_ms:.2f} ms; plane_init_points {planes_ms:.3f} ms; "
        f"plane_init_sphere {sphere_ms:.3f} ms")
    runs = {"depth": (depth_init, 1000, False, 0), "depth, no splitting": (depth_init, 0, False, 0),
            "depth, single radii": (depth_init, 1000, True, 0), "depth, Gaussian splat": (depth_init, 1000, False, 2),
            "sphere": (sphere_init, 1000, False, 0),
            "noisy-gt": ((init.center, init.quat, init.radii), 1000, False, 0)}
    out = {}
    for name, (planes, split_every, single, mode) in runs.items():
        fit = SceneFit(*planes, cams, tD, tN, params=SplatParams(weight_mode=mode),
                       cfg=FitConfig(check_every=250, split_every=split_every, split_thresh=0.2, single_radii=single))
        curve = [[0, round(fit.depth_l1(lam=300.0), 5)]]
        fit_s = 0.0
        for ck in range(500, args.fit_iters + 1, 500):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fit.run(500, graph=True)
            torch.cuda.synchronize()
            fit_s += time.perf_counter() - t0
            curve.append([ck, round(fit.depth_l1(lam=300.0), 5)])
            log(f"{name}: iteration {ck} depth L1 {curve[-1][1]:.4f} m, K {fit.K}")
        c, q, _ = fit.planes()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, n_inst = si.merge_planes(c, q)
        merge_ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"depth_l1": curve, "K_final": int(fit.K), "fit_seconds": round(fit_s, 3),
                     "splits": [list(x) for x in fit.splits], "merged_instances": n_inst,
                     "merge_ms": round(merge_ms, 3)}
    _, gt_inst = si.merge_planes(*(torch.as_tensor(x, device="cuda") for x in (gt.center, gt.quat)))
    return {
        "metric": "depth L1 after the fit, by plane initialisation", "unit": "m",
        "ground_truth_instances": gt_inst,
        "value": out["depth"]["depth_l1"][-1][1], "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
        "dtype": "f32 (f64 ray-plane geometry)",
        "config": {"workload": f"room, {V} views of {W}x{H}, K_init = {K}, {args.fit_iters} iterations, "
                               "splitting every 1000", "fused_points": int(n)},
        "init_ms": {"depth_points": round(pts_ms, 3), "plane_init_points": round(planes_ms, 3),
                    "plane_init_sphere": round(sphere_ms, 3)},
        "runs": out,
    }


def sleep_cycles_for(ms: float, stream) -> int:
    """Cycles of torch's spin kernel that keep the stream busy for about `ms`."""
    import torch
    torch.cuda._sleep(1000)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    torch.cuda._sleep(1_000_000)
    e1.record(stream)
    torch.cuda.synchronize()
    return max(1000, int(1_000_000 * ms / max(e0.elapsed_time(e1), 1e-3)))


def sample_phases(fit, steps: int, n_samples: int, stream):
    """Per-phase durations and render statistics sampled over a trajectory:
    every `stride`-th of `steps` steps runs eagerly after a diagnostics pass
    on its state, the other steps are graph replays (same bits).  Before each
    phase of a sampled step the stream spins for ~0.5 ms while the host
    queues the phase's launches, so the events around the phase (on the
    stream the kernels are launched on) time its kernels back to back, not
    the host's launch latency.
    Returns (phase_ms, sum of the phases, counters averaged over the samples)."""
    import torch
    names = ("project", "bin", "fwd", "bwd", "adam")   # "fwd": forward with the render loss
    ev = {n: [] for n in names}
    n_samples = max(1, min(n_samples, steps))
    stride = max(1, steps // n_samples)
    cycles = sleep_cycles_for(0.5, stream)
    log(f"timing {n_samples} eager steps phase by phase, one every {stride} steps")
    stats = []
    for i in range(steps):
        if i % stride or len(stats) >= n_samples:
            fit.graph.replay()
            continue
        stats.append(fit.diagnose())
        ends, starts = [], []

        def mark():
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            ends.append(e)
            if len(ends) <= len(names):
                torch.cuda._sleep(cycles)
                b = torch.cuda.Event(enable_timing=True)
                b.record(stream)
                starts.append(b)
        fit._step(mark=mark)
        torch.cuda.synchronize()
        for j, n in enumerate(names):
            ev[n].append(starts[j].elapsed_time(ends[j + 1]))
    phase_ms = {n: float(np.mean(x)) for n, x in ev.items()}
    if one_launch_step(fit):
        # forward, loss, backward and Adam in one call: timed as one phase
        phase_ms = {"project": phase_ms["project"], "bin": phase_ms["bin"],
                    "step": phase_ms["fwd"] + phase_ms["bwd"] + phase_ms["adam"]}
    phase_sum = float(sum(phase_ms.values()))
    cnt = {k: float(np.mean([st[k] for st in stats])) for k in stats[0] if not isinstance(stats[0][k], list)}
    cnt["max_steps"] = max(st["max_steps"] for st in stats)
    cnt["max_wave_ticks"] = max(st["max_wave_ticks"] for st in stats)
    cnt["bwd_max_block_ticks"] = max(st["bwd_max_block_ticks"] for st in stats)
    return phase_ms, phase_sum, cnt


def one_launch_step(fit) -> bool:
    """The fitting step takes plane_render_step (forward, loss and backward
    in one render launch)."""
    c = fit.cfg
    return c.one_launch and not c.single_radii and not c.split_every


def dominant_phase(phase_ms) -> str:
    return "step" if "step" in phase_ms else max(("fwd", "bwd"), key=lambda n: phase_ms[n])


def render_roofline(phase_ms, cnt, traffic=None, peaks=None):
    """Roofline of the dominant render phase: algorithmic lane operations of
    the sampled launches (evaluated pairs and composited hits, the kernels'
    own counts) / the phase's mean launch time, against the vector ALU's
    non-packed issue rate.  The one-launch step does the forward's and the
    backward's algorithmic work."""
    hits = int(round(cnt["composited_hits"]))
    evals = int(round(cnt["evals"]))
    dom = dominant_phase(phase_ms)
    per_hit = {"fwd": OPS_PER_HIT_FWD, "bwd": OPS_PER_HIT_BWD, "step": OPS_PER_HIT_FWD + OPS_PER_HIT_BWD}[dom]
    per_eval = {"fwd": OPS_PER_EVAL, "bwd": OPS_PER_EVAL_BWD, "step": OPS_PER_EVAL + OPS_PER_EVAL_BWD}[dom]
    ops = evals * per_eval + hits * per_hit
    achieved = ops / (phase_ms[dom] * 1e-3) / 1e12
    roof = {
        "kernel": {"fwd": "render_fwd_kernel (plane_render_fwd_loss)",
                   "bwd": "render_bwd_kernel+bwd_reduce_kernel<Adam> (plane_render_bwd_adam)",
                   "step": "render_bwd_kernel<fused>+bwd_reduce_kernel<Adam> (plane_render_step: forward, "
                           "loss, backward, then the per-plane reduction with the Adam update)"}[dom],
        "bound": "alu",
        "achieved": round(achieved, 4),
        "peak": round(MI355X_VALU_TOPS, 2),
        "unit": "T lane-op/s",
        "frac": round(achieved / MI355X_VALU_TOPS, 5),
        "traffic": traffic,
        "launch_ms": round(phase_ms[dom], 4),
        "algorithmic_units": f"{evals} evaluated pairs x {per_eval} + {hits} composited hits x {per_hit} "
                             f"lane operations",
    }
    if peaks:
        roof["peak_measured"] = peaks
    return roof, hits, evals


def measured_peaks():
    """The chip's rates measured in the same process: the vector ALU issue
    rate for fp32 and fp64 fused multiply-adds (ps_valu_probe) and the HBM
    rate of a 1 GiB device copy (read + write bytes / time)."""
    import torch
    from paper_2412_03451_amd.splat import valu_probe
    f32, _ = valu_probe(0)
    f64, _ = valu_probe(1)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    st = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        dst.copy_(src)
        e1.record(st)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    hbm = 2 * src.numel() * 4 / best / 1e9
    del src, dst
    return {"valu_fp32_fma_T_lane_op_s": round(f32, 2), "valu_fp64_fma_T_lane_op_s": round(f64, 2),
            "hbm_copy_GB_s": round(hbm, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000, help="timed fitting iterations (the room fit is 5000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--views", type=int, default=1, help="views per fitting step")
    ap.add_argument("--tile", type=int, nargs=2, default=(16, 16))
    ap.add_argument("--start-ite", type=int, default=0)
    ap.add_argument("--pending", type=int, default=6, choices=(4, 6, 8, 12),
                    help="pending-hit buffer size of the render kernels")
    ap.add_argument("--separate-calls", action="store_true",
                    help="fitting step with plane_render_fwd_loss and plane_render_bwd_adam instead of "
                         "plane_render_step (forward, loss and backward in one render launch)")
    ap.add_argument("--force-rounds", action="store_true",
                    help="send every pixel through the exact round-based ordering path")
    ap.add_argument("--phase-steps", type=int, default=50,
                    help="eager steps timed phase by phase (per-kernel durations), spread over the timed steps")
    ap.add_argument("--sync-every", type=int, default=0,
                    help="synchronise after every N timed replays (for hardware-counter runs; off by default)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--workload", default="room", choices=("room", "scene-fit", "memory", "batched", "initnet",
                                                          "init-ablation"),
                    help="room: the fitting-step throughput (default); scene-fit: wall-time of plain fits "
                         "against batched fits from the learned initialisation at equal depth L1")
    ap.add_argument("--rooms", type=int, default=32, help="scene-fit: held-out rooms; batched: rooms")
    ap.add_argument("--autotune", dest="autotune", action="store_true", default=True,
                    help="batched: tile shape per room from the autotuner (default)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batched: 16x16 tiles for every room")
    ap.add_argument("--per-item-launch", action="store_true",
                    help="batched: one workgroup per 8x8 block instead of the persistent work-queue launch")
    ap.add_argument("--train-rooms", type=int, default=256, help="scene-fit: rooms fitted to train the initializer")
    ap.add_argument("--train-fit-iters", type=int, default=1000,
                    help="scene-fit: plain-fit iterations of the training rooms")
    ap.add_argument("--train-steps", type=int, default=6000, help="scene-fit: initializer training steps")
    ap.add_argument("--target-l1", type=float, default=0.01, help="scene-fit: depth L1 target (m)")
    ap.add_argument("--conf-min", type=float, default=0.8, help="scene-fit: proposal confidence for refinement")
    ap.add_argument("--d-max", type=float, default=0.03, help="scene-fit: largest set-loss distance of a match")
    ap.add_argument("--check-every", type=int, default=250, help="scene-fit: iterations between depth-L1 checks")
    ap.add_argument("--fit-iters", type=int, default=2000,
                    help="scene-fit: iterations of the plain fits; init-ablation: iterations of each fit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): scenes shard across GPUs "
              f"without communication, so the per-GPU number is the whole story", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_03451_amd.fit import FitConfig, SceneFit
    from paper_2412_03451_amd.splat import Job, Renderer, SplatParams

    if args.workload == "scene-fit":
        print(json.dumps(scene_fit_bench(args)), flush=True)
        return
    if args.workload == "memory":
        print(json.dumps(memory_bench(args)), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(batched_bench(args)), flush=True)
        return
    if args.workload == "initnet":
        print(json.dumps(initnet_bench(args)), flush=True)
        return
    if args.workload == "init-ablation":
        print(json.dumps(init_ablation_bench(args)), flush=True)
        return

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n_views = 100
    V = args.views
    log(f"building room workload ({n_views} views)")
    gt, init, cams, info = build_workload(n_views)
    K = init.K
    W, H = cams[0].width, cams[0].height
    dev = torch.device("cuda")

    def T(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)

    # targets: ground truth rendered at lambda = 300 by the parity-tested forward
    log("rendering targets")
    tr = Renderer([Job(0, K, i, W, H, tuple(args.tile)) for i in range(n_views)], cams, pair_capacity=1 << 22)
    tgt_d, tgt_n = tr.render(T(gt.center), T(gt.quat), T(gt.radii), torch.tensor([300.0], device=dev))
    del tr

    params = SplatParams(flags=({6: 0, 4: 1, 8: 2, 12: 3}[args.pending] << 4) | (1 if args.force_rounds else 0))
    cfg = FitConfig(tile=tuple(args.tile), views_per_step=V, check_every=max(1, args.warmup),
                    one_launch=not args.separate_calls)
    fit = SceneFit(init.center, init.quat, init.radii, cams, tgt_d.view(n_views, -1), tgt_n.view(n_views, -1),
                   cfg=cfg, params=params, device=dev)
    fit.ite.fill_(args.start_ite)
    need = fit.size_capacity()
    log(f"pairs needed (max over views) {need}, capacity {fit.rend.L.pair_capacity}")
    start_state = fit.state()

    # warm-up: the whole timed trajectory once through the fit loop (eager
    # step, graph capture, replays; the pair lists grow if any step of it
    # needs more), then back to the start
    log(f"warmup: the {args.steps}-step trajectory through the fit loop, then {args.warmup} replays")
    fit.run(args.steps, graph=True)
    fit.restore(start_state)
    for _ in range(max(1, args.warmup)):
        fit.graph.replay()
    fit.restore(start_state)

    # timed: K replays of the captured step from the start state (the fit's
    # first K iterations, lambda following Eq. 10), inputs resident in HBM
    log(f"timing {args.steps} graph-replayed steps")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    early = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    n_early = min(args.steps, 200)
    start.record(stream)
    for i in range(args.steps):
        fit.graph.replay()
        if i + 1 == n_early:
            early.record(stream)
        if args.sync_every and (i + 1) % args.sync_every == 0:
            torch.cuda.synchronize()
    end.record(stream)
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    ms_early = start.elapsed_time(early) / n_early
    if fit.overflowed():
        raise RuntimeError("pair capacity exceeded during the timed steps")
    final_loss = fit._graph_loss.sum(0).cpu().tolist()

    # per-phase durations and walk statistics, sampled over the same trajectory
    fit.restore(start_state)
    phase_ms, phase_sum, cnt = sample_phases(fit, args.steps, args.phase_steps, stream)
    pix = V * W * H
    value = pix * K / (ms_step * 1e-3) / 1e6
    dom = dominant_phase(phase_ms)
    roof, hits, evals = render_roofline(phase_ms, cnt, measured_traffic(dom, traffic_key(args)), measured_peaks())
    n_items = max(1, int(fit.rend.L.n_items))
    out = {
        "metric": "fwd+bwd Mpixel*planes/s",
        "value": round(value, 1),
        "unit": "Mpixel*planes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_first_200": round(ms_early, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 ray-plane geometry)",
        "data": "synthetic",
        "config": {"workload": f"single room, K={K} planes, {V} view(s)/step of {W}x{H}, f=577, "
                               f"tile {args.tile[0]}x{args.tile[1]}, fitting iterations {args.start_ite}-"
                               f"{args.start_ite + args.steps - 1} (lambda of Eq. 10), graph-replayed steps",
                   "planes": K, "views_per_step": V, "width": W, "height": H,
                   "pairs_per_step": int(cnt["pairs"]),
                   "step_form": ("one render launch (plane_render_step)" if one_launch_step(fit) else
                                 "plane_render_fwd_loss + plane_render_bwd_adam")},
        "phase_sum_ms": round(phase_sum, 4),
        "phase_ms": {k: round(x, 4) for k, x in phase_ms.items()},
        "final_loss": [round(x, 3) for x in final_loss[:3]],
        "render_stats": {"pending": args.pending, "composited_hits": hits, "pairs_evaluated": evals,
                         "hits_per_evaluated_pair": round(hits / max(1, evals), 4),
                         "round_path_pixels": int(cnt["slow_pixels"]),
                         "bwd_extra_passes": int(cnt["bwd_extra_passes"]),
                         "walk_steps": int(cnt["steps"]), "walk_steps_max_block": int(cnt["max_steps"]),
                         "block_us_mean": round(cnt["wave_ticks"] / 100.0 / n_items, 3),
                         "block_us_max": round(cnt["max_wave_ticks"] / 100.0, 3),
                         "blocks": n_items,
                         "bwd_block_us_mean": {k: round(cnt["bwd_ticks_" + k] / 100.0 / n_items, 3)
                                               for k in ("setup", "walk", "sort", "grad")},
                         "bwd_block_us_max": round(cnt["bwd_max_block_ticks"] / 100.0, 3),
                         "bwd_grad_candidates": int(cnt["bwd_grad_candidates"]),
                         "bwd_grad_groups": int(cnt["bwd_grad_groups"])},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (float64 oracle on a pixel sample)")
        import oracle
        out["cpu_baseline"] = cpu_baseline(init, cams, oracle.lambda_at(args.start_ite), args.cpu_seconds)
        if args.start_ite == 0:
            log("culling efficiency (float64 oracle on a pixel sample of view 0)")
            out["culling"] = culling_efficiency(init, cams, oracle.lambda_at(0), args.tile)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
