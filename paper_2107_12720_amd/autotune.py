"""Launch-parameter autotuner for libtrim calls.

A grid search over the sweep block size, the work-chunk size of the first
sweep (the paper's schedule(dynamic, s), Section 8; s = 4096 there) and the
number of persistent workers.  Two stages: every candidate is timed with HIP
events (median of `reps` runs after one warm-up); then the `finalists` fastest
are timed again, round-robin over `4 * reps` rounds so that drift in the GPU's
clocks hits them alike, and the lowest median of that stage wins.  Results are
cached as JSON, keyed by device name, call kind and a shape bucket, in
$TRIM_TUNE_CACHE (default ~/.cache/trim_tune.json).  Tuning only changes the
schedule: the live bitmap, the traversed-edge total and (for batches, whose
per-graph totals do not depend on the schedule) the per-graph counts of every
candidate equal the first candidate's element by element, which `tune`
checks.
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
         reps: int = 3, use_cache: bool = True, finalists: int = 4,
         exact_counts: bool = False):
    """Pick (block, chunk, workers) for `run(opts) -> TrimResult`.

    Returns (best_params, table) where table lists every candidate's median ms
    of the first stage (and `final_ms` for the finalists).  Every candidate
    must give the first candidate's bitmap and traversed-edge total, and with
    `exact_counts` its worker_edges tensor too (per-graph totals of a batch)."""
    import torch

    import paper_2107_12720_amd as T
    key = shape_key(kind, n, m)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return cache[key], None
    table = []
    ref = None

    def check(res, what):
        nonlocal ref
        torch.cuda.synchronize()
        got = (res.live_bitmap.clone(), res.stats_dict()["edges_total"],
               res.worker_edges.clone() if exact_counts else None)
        if ref is None:
            ref = got
            return
        same = torch.equal(got[0], ref[0]) and got[1] == ref[1]
        if exact_counts:
            same = same and torch.equal(got[2], ref[2])
        if not same:
            raise RuntimeError(f"schedule {what} changed the result")

    for blk in blocks:
        for ch in chunks:
            for wk in workers:
                opts = T.make_opts(block=blk, chunk=ch, workers=wk)
                res = [None]

                def call():
                    res[0] = run(opts)
                ms = time_call(call, reps)
                check(res[0], f"{blk}/{ch}/{wk}")
                table.append({"block": blk, "chunk": ch, "workers": wk, "ms": ms})
    top = sorted(table, key=lambda r: r["ms"])[:max(1, finalists)]
    runs = {id(r): [] for r in top}
    calls = {id(r): (lambda o=T.make_opts(block=r["block"], chunk=r["chunk"],
                                          workers=r["workers"]): run(o)) for r in top}
    for _ in range(4 * reps):
        for r in top:
            runs[id(r)].append(time_call(calls[id(r)], 1))
    for r in top:
        r["final_ms"] = statistics.median(runs[id(r)])
    best = min(top, key=lambda r: r["final_ms"])
    params = {"block": best["block"], "chunk": best["chunk"], "workers": best["workers"],
              "ms": best["final_ms"]}
    if use_cache:
        cache[key] = params
        save_cache(cache)
    return params, table
