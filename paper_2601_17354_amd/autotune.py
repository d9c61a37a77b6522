"""Tuner for the batched multi-view step.

Candidates are the compositing kernels' compile-time shapes: tile
16x16, 8x8, 16x8, 32x8 or 8x32 pixels, and 32, 64, 128 or 256 splats staged
per LDS batch.  Each candidate builds its own buffers (its tile shape
changes the pair count and the trace), runs until nothing overflows, is
captured as a graph and timed over a few replays with HIP events; the
fastest wins.  Results are cached in a JSON file keyed by device name and
workload signature (Gaussian count, SH degree, view sizes), so a later run
on the same workload reuses the choice without timing.
"""

from __future__ import annotations

import json
import os
import time

import torch

from .batch import BatchedStep, time_steps

TILES = [(16, 16), (8, 8), (16, 8), (32, 8), (8, 32)]
BATCHES = [32, 64, 128, 256]


def candidates():
    return [(t, b) for t in TILES for b in BATCHES]


def signature(n: int, sh_degree: int, cams: list, cached: bool) -> str:
    views = "-".join(f"{c['width']}x{c['height']}" for c in cams)
    return f"n{n}-sh{sh_degree}-{'cached' if cached else 'recompute'}-{views}"


def cache_path() -> str:
    return os.environ.get("PGS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pocketgs", "tune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(params: torch.Tensor, sh_degree: int, cams: list, targets: list, cached: bool = True,
         steps: int = 5, warmup: int = 2, cands=None, use_cache: bool = True, log=None, **step_kw) -> dict:
    """Returns dict(tile, batch, ms, table) with the fastest candidate."""
    dev = torch.cuda.get_device_name(params.device)
    key = f"{dev}|{signature(params.shape[1], sh_degree, cams, cached)}"
    path = cache_path()
    store = _load(path) if use_cache else {}
    if use_cache and key in store:
        hit = dict(store[key])
        hit["cached"] = True
        return hit
    table = []
    t0 = time.perf_counter()
    for tile, batch in (cands or candidates()):
        st = BatchedStep(params.clone(), sh_degree, cams, targets, tile=tile, batch=batch, cached=cached,
                         **step_kw)
        st.prepare()
        st._alloc_pairs(int(st.capacity * 1.25), int(st.entry_capacity * 1.25))
        st.capture()
        ms = time_steps(st.replay, steps, warmup)
        ok = st.read_flags() == 0
        table.append(dict(tile=f"{tile[0]}x{tile[1]}", batch=batch, ms=round(ms, 4), ok=ok,
                          pairs=int(st.num_pairs.item())))
        if log:
            log(f"  tile {tile[0]}x{tile[1]} batch {batch}: {ms:.3f} ms/step{'' if ok else ' (overflowed)'}")
        del st
        torch.cuda.empty_cache()
    good = [r for r in table if r["ok"]] or table
    best = min(good, key=lambda r: r["ms"])
    tw, th = (int(x) for x in best["tile"].split("x"))
    res = dict(tile=[tw, th], batch=best["batch"], ms=best["ms"], table=table,
               seconds=round(time.perf_counter() - t0, 1), cached=False)
    if use_cache:
        store[key] = {k: v for k, v in res.items() if k != "cached"}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(store, f, indent=1)
    return res
