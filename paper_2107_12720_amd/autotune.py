"""Launch-parameter autotuner for libtrim calls.

A grid search over the sweep block size, the work-chunk size of the first
sweep (the paper's schedule(dynamic, s), Section 8; s = 4096 there) and the
number of persistent workers, each candidate timed with HIP events (median of
`reps` runs after one warm-up).  Results are cached as JSON, keyed by device
name, call kind and a shape bucket, in $TRIM_TUNE_CACHE (default
~/.cache/trim_tune.json).  Tuning only changes the schedule: the live set and
the traversed-edge total are the same for every candidate, which `tune`
checks for each of them.
"""
from __future__ import annotations

import json
import math
import os
import statistics

BLOCKS = (128, 256, 512, 1024)
CHUNKS = (256, 1024, 4096, 16384, 65536)


def cache_path() -> str:
    return os.environ.get("TRIM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "trim_tune.json"))


def shape_key(kind: str, n: int, m: int) -> str:
    import torch
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    return f"{dev}/{kind}/n2^{max(0, int(math.log2(max(n, 1))))}/m2^{max(0, int(math.log2(max(m, 1))))}"


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass


def time_call(fn, reps: int) -> float:
    """Median milliseconds of fn() over reps runs (after one warm-up)."""
    import torch
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(ctx, kind: str, n: int, m: int, run, workers=(0,), blocks=BLOCKS, chunks=CHUNKS,
         reps: int = 3, use_cache: bool = True):
    """Pick (block, chunk, workers) for `run(opts) -> TrimResult`.

    Returns (best_params, table) where table lists every candidate's median ms.
    Every candidate must give the same bitmap and traversed-edge total."""
    import paper_2107_12720_amd as T
    key = shape_key(kind, n, m)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return cache[key], None
    table = []
    ref = None
    for blk in blocks:
        for ch in chunks:
            for wk in workers:
                opts = T.make_opts(block=blk, chunk=ch, workers=wk)
                res = [None]

                def call():
                    res[0] = run(opts)
                ms = time_call(call, reps)
                sig = (res[0].live_bitmap.sum().item(), res[0].stats_dict()["edges_total"])
                if ref is None:
                    ref = sig
                elif sig != ref:
                    raise RuntimeError(f"schedule {blk}/{ch}/{wk} changed the result")
                table.append({"block": blk, "chunk": ch, "workers": wk, "ms": ms})
    best = min(table, key=lambda r: r["ms"])
    params = {"block": best["block"], "chunk": best["chunk"], "workers": best["workers"],
              "ms": best["ms"]}
    if use_cache:
        cache[key] = params
        save_cache(cache)
    return params, table
