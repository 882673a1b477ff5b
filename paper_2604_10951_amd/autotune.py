"""Autotuner for the renderer's launch parameters.

Times whole frames (preprocess -> bin -> sort -> render) of the caller's own
scene and views for every candidate binning tile size (8, 16, 32), LDS batch
of list entries (16, 32) and render schedule (one workgroup per block, a
persistent longest-list-first work queue, or -- for Top-K -- the split
selection + gather passes, which take no batch size), and returns the fastest.  Results
are cached in a JSON file keyed by the workload's shape.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from .raster import Rasterizer

TILES = (8, 16, 32)
BATCHES = (16, 32)
SCHEDULES = ("grid", "persistent", "split")


def _cache_path() -> str:
    root = os.environ.get("FASTSEGSIM_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "fastsegsim"))
    return os.path.join(root, "autotune.json")


def workload_key(cams, n: int, C: int, topk: int, feat_dtype: str) -> str:
    res = ",".join(f"{c.width}x{c.height}" for c in cams)
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return f"{dev}|V{len(cams)}|{res}|N{n}|C{C}|K{topk}|{feat_dtype}"


def time_config(cams, tensors, *, tile: int, batch: int, schedule: str, topk: int, feat_dtype: str,
                steps: int = 5, device="cuda") -> float:
    rast = Rasterizer(cams, tile=tile, topk=topk, batch=batch, schedule=schedule, feat_dtype=feat_dtype,
                      device=device)
    rast.render(*tensors)
    out = rast.alloc_out(tensors[4].shape[1])
    rast.render_nosync(*tensors, out)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        rast.render_nosync(*tensors, out)
    b.record()
    torch.cuda.synchronize()
    if not rast.pairs_fit():
        raise RuntimeError("pair capacity exceeded while tuning")
    return a.elapsed_time(b) / steps


def tune(cams, tensors, *, topk: int, feat_dtype: str = "f32", steps: int = 5, use_cache: bool = True,
         candidates=None, device="cuda") -> dict:
    """Fastest {tile, batch, schedule, ms} for this workload (cached)."""
    cams = list(cams) if isinstance(cams, (list, tuple)) else [cams]
    n, C = tensors[4].shape
    key = workload_key(cams, n, C, topk, feat_dtype)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key], cached=True)
    cands = candidates or [(t, b, s) for t, b, s in itertools.product(TILES, BATCHES, SCHEDULES)
                           if s != "split" or (topk > 0 and b == BATCHES[-1])]
    trials = []
    for tile, batch, schedule in cands:
        ms = time_config(cams, tensors, tile=tile, batch=batch, schedule=schedule, topk=topk,
                         feat_dtype=feat_dtype, steps=steps, device=device)
        trials.append({"tile": tile, "batch": batch, "schedule": schedule, "ms": ms})
        torch.cuda.empty_cache()
    best = min(trials, key=lambda t: t["ms"])
    result = dict(best, trials=trials)
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = result
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return dict(result, cached=False)
