"""Autotuner of the render configuration: tile shape (8x8, 16x16, 32x8) and
pending-hit buffer size, chosen per (image size, plane-count bucket) by
timing graph-replayed fitting steps on the scene itself.

The results are cached in a JSON file (PLANESPLAT_TUNE_CACHE, else
~/.cache/planesplat/tune.json): key "WxH/K<bucket>" -> {"tile": [w, h],
"pending": p, "ms": step time, "tried": {...}}; tune_batch chooses one shape
for a whole batch by timing it.  Each configuration's time
is the median of three timed runs, and the first tile shape and buffer size
(16x16, 6) stay unless another is more than TILE_MARGIN faster, so timing
noise does not change the choice from run to run.  Tuning only reads the
scene; the fits it times are thrown away.
"""

from __future__ import annotations

import json
import math
import os
from dataclasses import replace

import torch

from .fit import BatchFit, FitConfig, Scene
from .splat import SplatParams

TILES = ((16, 16), (32, 8), (8, 8))
PENDING = (6, 8, 4)
TILE_MARGIN = 0.03   # a configuration other than the first replaces it only when this much faster
_PENDING_BITS = {6: 0, 4: 1, 8: 2, 12: 3}


def pending_flags(pending: int) -> int:
    """ps_params.flags bits 4-5 for a pending-buffer size."""
    return _PENDING_BITS[pending] << 4


def k_bucket(K: int) -> int:
    return 1 << max(0, int(round(math.log2(max(K, 1)))))


def cache_key(width: int, height: int, K: int, replicas: int = 1) -> str:
    return f"{width}x{height}/K{k_bucket(K)}" + (f"/x{replicas}" if replicas > 1 else "")


def default_cache_path() -> str:
    return os.environ.get("PLANESPLAT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "planesplat", "tune.json"))


class Autotuner:
    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.table = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.table = json.load(f)

    def save(self):
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, width: int, height: int, K: int, replicas: int = 1):
        """(tile, pending) cached for this shape, or None."""
        e = self.table.get(cache_key(width, height, K, replicas))
        return None if e is None else (tuple(e["tile"]), int(e["pending"]))

    @staticmethod
    def time_config(scene: Scene, tile, pending: int, cfg: FitConfig, steps: int, warmup: int,
                    replicas: int = 1) -> float:
        """ms per graph-replayed fitting step of `replicas` copies of the scene
        (one batch) with this configuration."""
        sc = replace(scene, tile=tuple(tile))
        return Autotuner.time_batch([sc] * replicas, SplatParams(flags=pending_flags(pending)), cfg, steps, warmup)

    def tune_batch(self, scenes, cfg: FitConfig | None = None, steps: int = 10, warmup: int = 3, tiles=TILES,
                   params: SplatParams | None = None):
        """One tile shape for a batch of scenes, chosen by timing the batch's
        own fitting steps with each shape: the step time of a batch is what it
        is run for, and shapes chosen per scene (alone, or on copies of it)
        need not minimise it (smaller tiles that win for one scene add
        binning work to the batch).  The first shape stays unless another is
        more than TILE_MARGIN faster.  Returns (tile, {shape: ms})."""
        cfg = cfg or FitConfig()
        tried = {}
        for t in tiles:
            scs = [replace(sc, tile=tuple(t)) for sc in scenes]
            tried[f"{t[0]}x{t[1]}"] = self.time_batch(scs, params or SplatParams(), cfg, steps, warmup)
        t0 = tried[f"{tiles[0][0]}x{tiles[0][1]}"]
        best = min(tiles, key=lambda t: tried[f"{t[0]}x{t[1]}"])
        if tried[f"{best[0]}x{best[1]}"] > t0 / (1.0 + TILE_MARGIN):
            best = tiles[0]
        return tuple(best), tried

    @staticmethod
    def time_batch(scenes, params: SplatParams, cfg: FitConfig, steps: int, warmup: int) -> float:
        """ms per graph-replayed fitting step of a batch of scenes."""
        fit = BatchFit(list(scenes), cfg=replace(cfg, check_every=max(1, warmup)), params=params)
        fit.size_capacity(rows=min(8, int(fit.table.shape[0])))
        fit.run(max(1, warmup), graph=True)
        st = torch.cuda.current_stream()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(3):   # the median of three runs: one slow run does not decide
            torch.cuda.synchronize()
            a.record(st)
            for _ in range(steps):
                fit.graph.replay()
            b.record(st)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) / steps)
        if fit.overflowed():
            return float("inf")
        return sorted(times)[1]

    def tune(self, scene: Scene, cfg: FitConfig | None = None, steps: int = 20, warmup: int = 5,
             tiles=TILES, pendings=PENDING, force: bool = False, replicas: int = 1):
        """Best (tile, pending) for the scene's shape; cached.  replicas > 1
        times that many copies of the scene in one batch: the configuration
        for a scene fitted in a large batch, where the GPU is full and
        throughput counts (alone, a small scene's step is latency: smaller
        tiles win there and lose in a batch)."""
        W, H = int(scene.cams[0].width), int(scene.cams[0].height)
        K = int(torch.as_tensor(scene.center).reshape(-1, 3).shape[0])
        key = cache_key(W, H, K, replicas)
        if not force and key in self.table:
            e = self.table[key]
            return tuple(e["tile"]), int(e["pending"])
        cfg = cfg or FitConfig()
        tried = {}
        # tiles first at the default buffer size, then buffer sizes at the best tile
        for t in tiles:
            tried[f"{t[0]}x{t[1]}/p{pendings[0]}"] = self.time_config(scene, t, pendings[0], cfg, steps, warmup,
                                                                      replicas)
        # another tile than the first (the default) only if it is clearly faster:
        # timing noise does not flip the choice from one run to the next
        t0 = tried[f"{tiles[0][0]}x{tiles[0][1]}/p{pendings[0]}"]
        best_t = min(tiles, key=lambda t: tried[f"{t[0]}x{t[1]}/p{pendings[0]}"])
        if tried[f"{best_t[0]}x{best_t[1]}/p{pendings[0]}"] > t0 / (1.0 + TILE_MARGIN):
            best_t = tiles[0]
        for p in pendings[1:]:
            tried[f"{best_t[0]}x{best_t[1]}/p{p}"] = self.time_config(scene, best_t, p, cfg, steps, warmup,
                                                                      replicas)
        best = f"{best_t[0]}x{best_t[1]}/p{pendings[0]}"
        for p in pendings[1:]:
            k = f"{best_t[0]}x{best_t[1]}/p{p}"
            if tried[k] < tried[best] / (1.0 + TILE_MARGIN):
                best = k
        tile_s, p_s = best.split("/p")
        tile = tuple(int(x) for x in tile_s.split("x"))
        self.table[key] = {"tile": list(tile), "pending": int(p_s), "ms": tried[best], "tried": tried}
        self.save()
        return tile, int(p_s)
