"""Autotuner for the launch shape of the batched fwd+bwd step.

Tries tile side (8, 16, 32) x Gaussians staged per LDS batch (64, 128, 256)
x launch mode (one workgroup per tile, or persistent workgroups pulling
(view, tile) items from a queue), times a few eager steps of the real
workload for each and keeps the fastest; then, for the winner, tries the
other batch sizes for the render backward alone.  Results are cached in a JSON file
keyed by device name and workload shape (Gaussian count, feature count,
view sizes, gradient mode), so later runs skip the sweep.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

from .raster import Config

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sgs_autotune.json")

CANDIDATES = [(t, b, p) for t in (8, 16, 32) for b in (64, 128, 256) for p in (0, 1)
              if not (t == 8 and b == 256)]


def _key(g, views, params, pose) -> str:
    dev = torch.cuda.get_device_name(0)
    sizes = ",".join(f"{v.width}x{v.height}" for v in views)
    return f"{dev}|n={g.n}|F={g.n_feat}|{sizes}|params={int(params)}|pose={int(pose)}"


def tune(g, views: Sequence, rgb_t, dep_t, lab, W, weights, params=True, pose=False,
         candidates: Optional[Iterable] = None, reps: int = 3, cache: Optional[str] = DEFAULT_CACHE,
         verbose: bool = False) -> Config:
    from .batched import MappingStep
    key = _key(g, views, params, pose)
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
            if key in table:
                return Config(**table[key]["config"])
        except (OSError, ValueError):
            pass
    best, best_ms, results = None, float("inf"), []

    def trial(cfg):
        st = MappingStep(g, views, cfg, rgb_t, dep_t, lab, W, weights, params=params, pose=pose)
        st.ensure_capacity()
        st.run()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            st.run()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        results.append({"tile": cfg.tile, "lds_batch": cfg.lds_batch, "persistent": cfg.persistent,
                        "lds_batch_bwd": cfg.lds_batch_bwd, "ms": ms})
        if verbose:
            print(f"[autotune] tile {cfg.tile} batch {cfg.lds_batch}/{cfg.lds_batch_bwd} "
                  f"persistent {cfg.persistent}: {ms:.3f} ms", flush=True)
        del st
        torch.cuda.empty_cache()
        return ms

    for tile, batch, persistent in (candidates or CANDIDATES):
        cfg = Config(tile=tile, lds_batch=batch, persistent=persistent)
        ms = trial(cfg)
        if ms < best_ms:
            best, best_ms = cfg, ms
    for bb in (64, 128, 256):
        if bb == best.lds_batch or (best.tile == 8 and bb == 256):
            continue
        cfg = dataclasses.replace(best, lds_batch_bwd=bb)
        ms = trial(cfg)
        if ms < best_ms:
            best, best_ms = cfg, ms
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            table = json.load(open(cache)) if os.path.exists(cache) else {}
            table[key] = {"config": dataclasses.asdict(best), "ms": best_ms, "sweep": results}
            json.dump(table, open(cache, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return best
