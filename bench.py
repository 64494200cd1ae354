#!/usr/bin/env python3
"""Benchmark of the trimming hot path on one MI355X.

One step = one complete AC-6 trim (init, first sweep, propagation, bitmap)
of the R-MAT scale-22 graph with a planted 100,000-vertex chain, with the
graph resident in HBM.  The value is input edges per second (m / step time).
The live bitmap and the traversed-edge total are checked against the CPU
oracle in the same run.

Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes / its average event-timed
                duration, against the 8 TB/s HBM peak (plus HBM traffic measured by
                rocprofv3 counters when a summary for the current kernel source is
                committed under profiles/);
  cpu_baseline  the oracle (sequential peel) timed on this host on the same graph;
  breakdown     every kernel's average duration;
  baselines     AC-4 and AC-3 on the same graph (one or a few runs each);
  depth         alpha times the measured per-step latency of a bare chain;
  two_sided     two-sided trimming (live successor and live predecessor) of the
                same graph with AC-6 and AC-4, kernel bytes and the oracle's time;
  sampling      edges or vertices sampled at 10 % .. 100 % (R-MAT scale 22), the
                scalability experiment of Section 9, all three algorithms;
  scc           strongly connected components by forward-backward search with
                two-sided trimming (Section 1.1), against scipy's in the CPU leg.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-baselines]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s + graphs/s: batched/learned-order AC-6 vs plain AC-6, bit-exact live set"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_FLOPS = 2.5e15   # dense BF16 matrix-core peak of MI355X
# 32-bit integer vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
INT32_VALU_PEAK_OPS = 256 * 64 * 2.4e9
# What the one-sided AC-6 kernels compile from: a committed counter summary of
# one of them stays valid while these are unchanged (other kernel files are
# separate translation units and cannot change them).
KERNEL_SOURCES = ("paper_2107_12720_amd/csrc/ac6.hip", "paper_2107_12720_amd/csrc/ac6_support.h",
                  "paper_2107_12720_amd/csrc/trim_device.h",
                  "paper_2107_12720_amd/csrc/trim_stats.h",
                  "paper_2107_12720_amd/csrc/trim_internal.h", "include/trim.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the kernel sources with comments and blank space removed, so a
    comment-only edit keeps a committed counter summary valid.  Of the public
    header only what the kernels use counts: the layouts of the graph, option
    and statistics structs and the schedule flags."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        if f.endswith("trim.h"):
            keep = re.findall(r"typedef struct \{[^}]*\} (?:trim_csr_t|trim_implicit_t|"
                              r"trim_opts_t|trim_stats_t);", code)
            keep += re.findall(r"#define TRIM_SCHED_\w+ \w+", code)
            code = "\n".join(keep)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, workers=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source and launch size; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash():
        return None
    if workers is not None and d.get("workers") not in (None, workers):
        return None
    return d.get("bytes_per_launch")


def prop_bytes(st, t6):
    """Algorithmic bytes of the propagation after the first sweep (its
    level-synchronous phases and its asynchronous tail together): 8 B per
    successor check (target id + target status), 16 B per close (two list-head
    exchanges), 16 B per join (record store + head CAS), 8 B per list member
    handed back (its record)."""
    return (8 * (t6 - st["edges_sweep"]) + 16 * st["closes"] + 16 * st["joins"]
            + 8 * st["visited"])


def jump_bytes(st):
    """Algorithmic bytes of the forest collapse: per list entry and round its
    entry, its link and its ancestor's link read, and one link or list entry
    written (16 B); per removed vertex an 8-byte head exchange and a 4-byte
    walk item."""
    return 16 * st["work_items"] + 12 * st["forest"]


def kernel_bytes(n, st, sw):
    """Algorithmic bytes of every AC-6 kernel of one trim (sw = the sweep's
    host counts: checks, joins, casualties, last-successor members).  The
    propagation's two kernels share one count: both get the combined bytes
    under the name 'propagation'."""
    checks, joins, cas, members = sw
    forest = st["forest"] > 0
    return {"ac6_init": 4 * (n + 1) + 8 * n + n // 8,
            "ac6_sweep": sweep_bytes(n, checks, joins, cas)
            + (4 * (joins + cas) + 4 * (members + cas) if forest else 0),
            "ac6_jump": jump_bytes(st),
            "propagation": prop_bytes(st, st["edges_total"]),
            "ac6_pack": 8 * n + n // 8}


def group_times(kavg):
    """Per-kernel average ms, with the propagation's two kernels summed."""
    out = {k: v for k, v in kavg.items() if k not in ("ac6_levels", "ac6_propagate")}
    out["propagation"] = kavg.get("ac6_levels", 0.0) + kavg.get("ac6_propagate", 0.0)
    return out


def sweep_counts(g, chunk=1 << 22):
    """(checks, joins, casualties, last-successor members) of the first sweep.
    Only out-degree-0 vertices are removed while it runs, so v joins the list
    of its first successor with out-degree > 0 (the S_last list if that is its
    last successor), or is left without a live successor if it has none.
    Counted over vertex ranges, so the largest graphs fit in host memory."""
    import numpy as np
    ro = g.row_off
    nz = np.diff(ro) > 0
    tot = [0, 0, 0, 0]
    for v0 in range(0, g.n, chunk):
        v1 = min(g.n, v0 + chunk)
        e0, e1 = int(ro[v0]), int(ro[v1])
        deg = np.diff(ro[v0:v1 + 1].astype(np.int64))
        if e1 == e0:
            continue
        ok = np.flatnonzero(nz[g.col[e0:e1]]) + e0
        start = ro[v0:v1].astype(np.int64)
        j = np.searchsorted(ok, start)
        first = np.where(j < ok.size, ok[np.minimum(j, max(ok.size - 1, 0))] if ok.size else -1,
                         -1)
        end = ro[v0 + 1:v1 + 1].astype(np.int64)
        has = (deg > 0) & (first >= start) & (first < end)
        tot[0] += int(np.where(has, first - start + 1, deg).sum())
        tot[1] += int(has.sum())
        tot[2] += int(((deg > 0) & ~has).sum())
        tot[3] += int((has & (first == end - 1)).sum())
    return tuple(tot)


def sweep_bytes(n, checks, joins, casualties):
    """Algorithmic bytes of one ac6_sweep launch: 4 B of offsets per vertex, 4 B
    per successor check (its target id; the target's status is a bit of the
    n/8-byte sinks bitmap, read once), 16 B per join (head exchange + record
    store), 4 B per queued casualty."""
    return 4 * (n + 1) + n // 8 + 4 * checks + 16 * joins + 4 * casualties


def first_ok(row_off, col, ok):
    """Per vertex: index in its list of the first neighbour with ok[] set, or -1."""
    import numpy as np
    start = row_off[:-1].astype(np.int64)
    end = row_off[1:].astype(np.int64)
    good = np.flatnonzero(ok[col]) if col.size else np.zeros(0, np.int64)
    j = np.searchsorted(good, start)
    first = np.where(j < good.size, good[np.minimum(j, max(good.size - 1, 0))], -1) \
        if good.size else np.full(start.shape, -1)
    has = (first >= start) & (first < end)
    return np.where(has, first - start, -1)


def two_sided_sweep_counts(g, rro, rcol):
    """(checks, joins, casualties, members, scanned) of the two-sided first
    sweep.  Vertices without a successor or a predecessor are the only ones
    removed while it runs; every other vertex (scanned) scans its successors
    for the first one not removed, and only if it finds one, its predecessors
    likewise.  Members: vertices that found both and whose out-support is
    their last successor (the forest collapse's tree members)."""
    import numpy as np
    deg = np.diff(g.row_off.astype(np.int64))
    indeg = np.diff(rro.astype(np.int64))
    alive0 = (deg > 0) & (indeg > 0)
    fo = first_ok(g.row_off, g.col, alive0)
    fi = first_ok(rro, rcol, alive0)
    out_ok = alive0 & (fo >= 0)
    in_ok = out_ok & (fi >= 0)
    checks = np.where(out_ok, fo + 1, deg)[alive0].sum() + np.where(fi >= 0, fi + 1, indeg)[out_ok].sum()
    joins = int(out_ok.sum() + in_ok.sum())
    members = int((in_ok & (fo == deg - 1)).sum())
    return int(checks), joins, int((alive0 & ~in_ok).sum()), members, int(alive0.sum())


def bench_two_sided(ctx, T, g, ro, col, rro_h, rcol_h, reps, with_ac3=True):
    """Two-sided trimming (a live successor and a live predecessor, Section 4.1)
    of the same graph: AC-6 and AC-4, with the kernels' algorithmic bytes, and
    the two-sided AC-3 rounds once (alpha + 1 of them)."""
    import numpy as np
    n, m = g.n, g.m
    rro, rcl = T.to_device(rro_h), T.to_device(rcol_h)
    ms6, kt6, res6 = time_gpu(ctx, lambda: ctx.trim_csr_two_sided(T.AC6, n, ro, col, rro, rcl),
                              reps, 1)
    st6 = res6.stats_dict()
    ms4, kt4, res4 = time_gpu(ctx, lambda: ctx.trim_csr_two_sided(T.AC4, n, ro, col, rro, rcl),
                              reps, 1)
    st4 = res4.stats_dict()
    # depth: a bare 100,000-vertex path whose first vertex has a self-loop
    # peels from its sink end only, one removal per step, like the planted chain
    L = 100000
    s_ = np.r_[np.arange(L - 1, dtype=np.int32), np.int32(0)]
    d_ = np.r_[np.arange(1, L, dtype=np.int32), np.int32(0)]
    import graphgen as gg
    gc = gg.from_edges(L, s_, d_)
    rc_t = gg.transpose(gc)
    dc = [T.to_device(x) for x in (gc.row_off, gc.col, rc_t[0], rc_t[1])]
    ms_chain, _, res_c = time_gpu(ctx, lambda: ctx.trim_csr_two_sided(T.AC6, L, *dc), 3, 1)
    chain_ok = res_c.stats_dict()["n_live"] == 1
    sc, sj, scas, smem, sscan = two_sided_sweep_counts(g, rro_h, rcol_h)
    forest = st6["forest"] > 0
    # bytes per unit: 4 B per read or write, 8 B per 4-byte atomic, 16 B per
    # 8-byte exchange (the paper's per-edge and per-vertex terms, both sides);
    # with the forest collapse the sweep also writes a link per scanned vertex
    # and a list entry per member and casualty, and the collapse reads and
    # writes 16 B per list entry and round, and exchanges both pairs (32 B)
    # and queues an item (4 B) per removal
    algo = {
        "ac6t_init": 8 * (n + 1) + 16 * n + n // 8,
        "ac6t_sweep": 8 * (n + 1) + n // 8 + 4 * sc + 16 * sj + 4 * scas
        + (4 * sscan + 4 * (smem + scas) if forest else 0),
        "ac6t_jump": 16 * st6["work_items"] + 36 * st6["forest"],
        "ac6t_propagate": (8 * (st6["edges_total"] - st6["edges_sweep"]) + 32 * st6["closes"]
                           + 16 * st6["joins"] + 8 * st6["visited"]),
        "ac6t_pack": 8 * n + n // 8,
    }
    k6 = {k: float(np.mean(v)) for k, v in kt6.items()}
    kernels = {k: {"avg_ms": v, "algorithmic_bytes": int(algo.get(k, 0)),
                   "achieved_GBs": algo.get(k, 0) / (v / 1e3) / 1e9,
                   "frac": algo.get(k, 0) / (v / 1e3) / 1e9 / HBM_PEAK_GBS} for k, v in k6.items()}
    dom = max(k6, key=k6.get)
    # AC-4: per removed vertex its two offsets pairs and queue slot (16 B), per
    # walked edge the neighbour id and the counter fetch-add (12 B)
    b4 = 12 * st4["edges_total"] + 8 * n + 16 * st4["n_dead"] + n // 8
    out = {"workload": "rmat22_ef16_chain100k", "n": n, "m": m,
           "ac6": {"ms": ms6, "edges_per_s": m / (ms6 / 1e3), "traversed": st6["edges_total"],
                   "n_live": st6["n_live"], "closes": st6["closes"], "joins": st6["joins"],
                   "forest": st6["forest"], "jump_rounds": st6["jump_rounds"],
                   "sweep_checks_match": sc == st6["edges_sweep"],
                   "kernels": kernels, "dominant": dom,
                   "roofline": {"bound": "hbm", "kernel": dom,
                                "achieved": kernels[dom]["achieved_GBs"], "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": kernels[dom]["frac"]},
                   "parity": None},
           "ac4": {"ms": ms4, "edges_per_s": m / (ms4 / 1e3), "traversed": st4["edges_total"],
                   "n_live": st4["n_live"],
                   "kernels_ms": {k: float(np.mean(v)) for k, v in kt4.items()},
                   "algorithmic_bytes": b4, "path_GBs": b4 / (ms4 / 1e3) / 1e9,
                   "parity": None},
           "ac6_speedup_vs_ac4": ms4 / ms6,
           "depth": {"chain_hop_us": ms_chain * 1e3 / (L - 1), "chain_live_ok": chain_ok}}
    checks = {"rro": rro_h, "rcol": rcol_h,
              "ac6": {"bitmap": res6.bitmap_numpy().copy(), "edges": st6["edges_total"],
                      "edges_live": st6["edges_live"]},
              "ac4": {"bitmap": res4.bitmap_numpy().copy(), "edges": st4["edges_total"]}}
    if with_ac3:
        # one call of about 5 s: no second call for a per-kernel split
        ms3, kt3, res3 = time_gpu(ctx, lambda: ctx.trim_csr_two_sided(T.AC3, n, ro, col, rro, rcl),
                                  1, 0, breakdown_steps=0)
        st3 = res3.stats_dict()
        out["ac3"] = {"ms": ms3, "edges_per_s": m / (ms3 / 1e3), "traversed": st3["edges_total"],
                      "rounds": st3["rounds"], "n_live": st3["n_live"],
                      "kernels_ms": {k: float(np.mean(v)) for k, v in kt3.items()},
                      "parity": None}
        out["ac6_speedup_vs_ac3"] = ms3 / ms6
        checks["ac3"] = {"bitmap": res3.bitmap_numpy().copy(), "edges": st3["edges_total"],
                         "rounds": st3["rounds"]}
    return checks, out


def bench_sampling(ctx, T, gg, ratios=tuple(k / 10 for k in range(1, 11))):
    """The scalability experiment of Section 9 on R-MAT scale 22, edge factor
    16 (the stand-in for the paper's largest graphs): edges or vertices are
    sampled at 10 % .. 100 %; unsampled edges are dropped, unsampled vertices
    are set to DEAD before trimming (trim_csr_preset).  Per ratio and
    algorithm: time, traversed edges, the largest per-worker count, and the
    share of vertices removed."""
    import numpy as np
    g = gg.rmat(22, 16, seed=0)
    n = g.n
    ro, col = T.to_device(g.row_off), T.to_device(g.col)
    rro_h, rcol_h = gg.transpose(g)
    rro, rcl = T.to_device(rro_h), T.to_device(rcol_h)
    names = {6: "ac6", 4: "ac4", 3: "ac3"}

    def measure(fn):
        ms, _, res = time_gpu(ctx, fn, 1, 1)
        st = res.stats_dict()
        return {"ms": ms, "traversed": st["edges_total"],
                "max_worker": int(res.worker_edges.max().item()), "n_live": st["n_live"]}, res

    out = {"workload": "rmat22_ef16", "n": n, "m": g.m, "edge": [], "vertex": []}
    checks = {}
    for ratio in ratios:
        preset, bm = gg.sample_vertices(n, ratio, seed=1)
        pd = T.to_device(bm.view(np.int32))
        row = {"ratio": ratio, "preset": int(preset.sum())}
        for a in (6, 4, 3):
            row[names[a]], res = measure(
                lambda: ctx.trim_csr_preset(a, n, ro, col, pd, rro, rcl))
            if ratio == 0.5:
                checks.setdefault("vertex", {"preset": preset})[a] = {
                    "bitmap": res.bitmap_numpy().copy(), "edges": row[names[a]]["traversed"]}
        row["removed_by_trimming_pct"] = 100.0 * (n - row["ac6"]["n_live"] - row["preset"]) / n
        row["dead_pct"] = 100.0 * (n - row["ac6"]["n_live"]) / n
        out["vertex"].append(row)

        h = g if ratio >= 1.0 else gg.sample_edges(g, ratio, seed=1)
        hro, hcol = T.to_device(h.row_off), T.to_device(h.col)
        a_h, b_h = (rro_h, rcol_h) if h is g else gg.transpose(h)
        hrro, hrcl = T.to_device(a_h), T.to_device(b_h)
        row = {"ratio": ratio, "m": h.m}
        for a in (6, 4, 3):
            row[names[a]], res = measure(
                lambda: ctx.trim_csr(a, n, hro, hcol, hrro if a == 4 else None,
                                     hrcl if a == 4 else None))
            if ratio == 0.5:
                checks.setdefault("edge", {"graph": h})[a] = {
                    "bitmap": res.bitmap_numpy().copy(), "edges": row[names[a]]["traversed"]}
        row["dead_pct"] = 100.0 * (n - row["ac6"]["n_live"]) / n
        out["edge"].append(row)
        log(f"sampling {ratio:.1f}: vertex AC-6 {out['vertex'][-1]['ac6']['ms']:.3f} ms, "
            f"edge AC-6 {row['ac6']['ms']:.3f} ms")
    checks["graph"] = g
    return checks, out


def bench_scc(ctx, T, graphs, reps):
    """SCC decomposition (forward-backward search with two-sided trimming,
    Section 1.1) of each (name, graph, G^T on the host) in `graphs`."""
    import numpy as np
    import torch
    out, checks = {}, {}
    for name, g, (rro_h, rcol_h) in graphs:
        ro, col = T.to_device(g.row_off), T.to_device(g.col)
        rro, rcl = T.to_device(rro_h), T.to_device(rcol_h)
        label = torch.empty(g.n, dtype=torch.int32, device="cuda")
        ctx.trim_scc(g.n, ro, col, rro, rcl, label=label)   # warm-up
        times, st = [], None
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            _, st = ctx.trim_scc(g.n, ro, col, rro, rcl, label=label)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        # search bytes: per examined list entry its neighbour id and the
        # neighbour's mark word (8 B); the live bits are a cache-resident bitmap
        sb = 8 * st["search_edges"]
        out[name] = {"n": g.n, "m": g.m, "ms": ms, "edges_per_s": g.m / (ms / 1e3), "stats": st,
                     "search_roofline": {"bound": "hbm", "algorithmic_bytes": sb,
                                         "achieved": sb / (st["search_ms"] / 1e3) / 1e9
                                         if st["search_ms"] > 0 else None,
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "note": "search_ms is host-timed and includes the "
                                                 "pivot choice and a synchronisation"},
                     "parity": None}
        checks[name] = {"graph": g, "label": label.cpu().numpy()[: g.n].copy()}
        log(f"scc {name}: {ms:.3f} ms, {st['n_scc']} components, giant {st['giant']}")
    return checks, out


def time_gpu(ctx, fn, steps, warmup, per_step=None, breakdown_steps=None):
    """Mean ms per call over `steps` timed calls with nothing recorded inside
    the timed region but one event pair around all of them; the per-kernel
    times of `breakdown_steps` further calls (default min(steps, 20); 0 = none)
    timed with the library's per-kernel events (those cost about 7 us per
    kernel of stream time, about 50 us per AC-6 trim, so they stay out of
    the calls the mean comes from; a kernel's own duration is the same); and
    the last result.  With a list `per_step`, a third loop of `steps` calls
    appends each call's own event-timed duration to it."""
    import torch
    for _ in range(warmup):
        fn()
    ctx.set_timing(0)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        res = fn()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    ktimes = {}
    nb = min(steps, 20) if breakdown_steps is None else breakdown_steps
    if nb > 0:
        ring = max(1, min(nb, 64))
        ctx.set_timing(ring)
        for i in range(nb):
            res = fn()
            if (i + 1) % ring == 0 or i + 1 == nb:
                for name, kms in ctx.kernel_times():
                    ktimes.setdefault(name, []).append(kms)
                ctx.set_timing(ring)
    ctx.set_timing(1)
    if per_step is not None:
        pairs = []
        for _ in range(steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            res = fn()
            b.record()
            pairs.append((a, b))
        torch.cuda.synchronize()
        per_step.extend(a.elapsed_time(b) for a, b in pairs)
    return ms, ktimes, res


def step_stats(times):
    """Median, mean and a 95 % confidence interval of the mean (normal
    approximation) of per-step times in ms."""
    import numpy as np
    t = np.asarray(times, dtype=np.float64)
    if t.size == 0:
        return None
    half = 1.96 * t.std(ddof=1) / np.sqrt(t.size) if t.size > 1 else 0.0
    return {"n": int(t.size), "median_ms": float(np.median(t)), "mean_ms": float(t.mean()),
            "ci95_ms": [float(t.mean() - half), float(t.mean() + half)]}


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth measured on this GPU (read + write bytes
    per second), the practical HBM ceiling beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "GBs": 2 * nbytes / (ms / 1e3) / 1e9}


def ev_time(fn, reps, warmup, stream):
    """Median ms of fn() measured with events recorded on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    stream.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(sorted(times)[len(times) // 2])


def bench_batch(ctx, T, gg, reps):
    """4,096 core+tail graphs: one autotuned, HIP-graph-captured launch sequence
    (graphs/s; one workgroup per graph), against the union path of trim_batch,
    the same AC-6 called once per graph, and the disjoint union trimmed as one
    graph."""
    import numpy as np
    import torch

    from paper_2107_12720_amd import autotune
    log("batch: generating 4096 graphs ...")
    b = gg.batch(4096, seed=0)
    bb = b.bitmap_base()
    G, N, M = b.G, int(b.vbase[-1]), int(b.ebase[-1])
    vb, ro, col, bbd = (T.to_device(b.vbase), T.to_device(b.row_off), T.to_device(b.col),
                        T.to_device(bb))
    lb = torch.empty(int(bb[-1]), dtype=torch.int32, device="cuda")
    ge = torch.empty(G, dtype=torch.int64, device="cuda")
    st = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    ctx.set_timing(False)

    def run(opts):
        return ctx.trim_batch(vb, ro, col, bbd, N, M, live_bitmaps=lb, graph_edges=ge, stats=st,
                              opts=opts, stream=s)
    with torch.cuda.stream(s):
        # one workgroup per graph: the block size is the tuning knob (the
        # chunk has no meaning there; workers 0 = one workgroup per slot the
        # occupancy allows)
        params, table = autotune.tune(ctx, "batch", N, M, run, workers=(0,),
                                      blocks=(256, 512, 1024), chunks=(0,), reps=3,
                                      use_cache=False, exact_counts=True)
        log(f"batch: tuned {params}")
        opts_g = T.make_opts(block=params["block"], chunk=params["chunk"],
                             workers=params["workers"], graph=True)
        ms_b = ev_time(lambda: run(opts_g), reps, 2, s)
        res = run(opts_g)
        s.synchronize()
    got = res.bitmap_numpy()
    bst = res.stats_dict()
    n_live_gpu = bst["n_live"]
    gedges = res.worker_edges.cpu().numpy().copy()
    # the same AC-6, one call per graph
    per = []
    for gi in range(G):
        v0, v1, e0, e1 = (int(b.vbase[gi]), int(b.vbase[gi + 1]), int(b.ebase[gi]),
                          int(b.ebase[gi + 1]))
        per.append((v1 - v0, ro[v0:v1 + 1] - e0, col[e0:e1], lb[int(bb[gi]):int(bb[gi + 1])]))
    P = ctx.num_workers(T.AC6)
    we = torch.empty(P, dtype=torch.int64, device="cuda")

    def each():
        for n_g, r_g, c_g, l_g in per:
            ctx.trim_csr(T.AC6, n_g, r_g, c_g, live_bitmap=l_g, worker_edges=we, stats=st,
                         stream=s)
    with torch.cuda.stream(s):
        ms_each = ev_time(each, 1, 1, s)
    # the same batch through the union path of trim_batch (device-wide kernels)
    opts_u = T.make_opts(flags=T.FLAG_BATCH_UNION, graph=True)
    with torch.cuda.stream(s):
        ms_bu = ev_time(lambda: run(opts_u), reps, 2, s)
        res_u = run(opts_u)
        s.synchronize()
    union_path_same = bool(np.array_equal(res_u.bitmap_numpy(), got)
                           and np.array_equal(res_u.worker_edges.cpu().numpy(), gedges))
    # the disjoint union as one graph (global target ids)
    col_u = T.to_device((b.col.astype(np.int64) + np.repeat(b.vbase[:-1], np.diff(b.ebase)))
                        .astype(np.int32))
    lbu = torch.empty((N + 31) // 32, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        ms_union = ev_time(lambda: ctx.trim_csr(T.AC6, N, ro, col_u, live_bitmap=lbu,
                                                worker_edges=we, stats=st, stream=s), reps, 1, s)
    ctx.set_timing(True)
    # the per-kernel split of one batch launch sequence, outside the graph
    # (event records are not captured)
    with torch.cuda.stream(s):
        opts_k = T.make_opts(block=params["block"], chunk=params["chunk"],
                             workers=params["workers"])
        _, kt, _ = time_gpu(ctx, lambda: run(opts_k), 5, 1)
    ksum = {k: float(np.mean(v)) for k, v in kt.items()}
    # B6 summed over the graphs: 8 B per check (target id and its status),
    # 20 B per vertex (offsets, list head, record), the bitmaps
    t6sum = int(gedges.sum())
    b6 = 8 * t6sum + 20 * N + N // 8
    roofline = {"bound": "hbm", "kernel": "whole batch (HIP graph)",
                "algorithmic_bytes": b6, "achieved": b6 / (ms_b / 1e3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": b6 / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS}
    check = {"batch": b, "bitmap_base": bb, "bitmap": got, "n_live": n_live_gpu,
             "graph_edges": gedges}
    return check, {"workload": "batch4096_coretail", "graphs": G, "sum_n": N, "sum_m": M,
            "ms": ms_b, "graphs_per_s": G / (ms_b / 1e3), "edges_per_s": M / (ms_b / 1e3),
            "parity": None, "tuned": params, "T6_sum": t6sum, "roofline": roofline,
            "kernels_ms": ksum, "stats": bst,
            "tuner": sorted(table, key=lambda r: r["ms"])[:8],
            "per_graph_calls": {"ms": ms_each, "graphs_per_s": G / (ms_each / 1e3)},
            "union_one_graph": {"ms": ms_union, "graphs_per_s": G / (ms_union / 1e3)},
            "batch_union_path": {"ms": ms_bu, "graphs_per_s": G / (ms_bu / 1e3),
                                 "same_result": union_path_same},
            "speedup_vs_per_graph_calls": ms_each / ms_b,
            "speedup_vs_union": ms_union / ms_b}


def bench_implicit(ctx, T, gg, reps, log2n=28, deferred=True):
    """AC-6 on the hash-generated graph G = (V, POST) with n = 2^28: successors
    are generated on the fly.  Checked at full size on sampled vertices: a live
    vertex has a live successor, a removed one has none."""
    import numpy as np
    import torch
    imp = gg.implicit(log2n=log2n, seed=0)
    table = T.to_device(imp.table)
    n = imp.n
    P = ctx.num_workers(T.AC6)
    lb = torch.empty((n + 31) // 32, dtype=torch.int32, device="cuda")
    we = torch.empty(P, dtype=torch.int64, device="cuda")
    st = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")
    log(f"implicit: n = 2^{log2n}")
    ms6, ktimes, res = time_gpu(ctx, lambda: ctx.trim_implicit(
        T.AC6, log2n, imp.seed, imp.zero_thr, table, live_bitmap=lb, worker_edges=we,
        stats=st), reps, 1)
    torch.cuda.synchronize()
    stat = res.stats_dict()
    bits = np.unpackbits(res.bitmap_numpy().view(np.uint8), bitorder="little")[:n]
    m = stat["graph_edges"]
    t6 = stat["edges_total"]
    # both bounds of the implicit path: status traffic (4 B per check, 16 B per
    # vertex, the bitmap) and hashing on the integer ALUs (at least one hash per
    # check and two per vertex, about 22 32-bit vector operations each)
    b6i = 4 * t6 + 16 * n + n // 8
    hashes = t6 + 2 * n
    int_ops = 22 * hashes
    hbm_frac = b6i / (ms6 / 1e3) / (HBM_PEAK_GBS * 1e9)
    alu_frac = int_ops / (ms6 / 1e3) / INT32_VALU_PEAK_OPS
    # the Jacobi AC-3 baseline on the same graph: 4 B per check (the target's
    # removal round; its id is hashed), 12 B per live-list entry and round
    P3 = ctx.num_workers(T.AC3)
    ms3, kt3, res3 = time_gpu(ctx, lambda: ctx.trim_implicit(
        T.AC3, log2n, imp.seed, imp.zero_thr, table, live_bitmap=lb, worker_edges=we[:P3],
        stats=st), 1, 0)
    st3 = res3.stats_dict()
    bits3 = np.unpackbits(res3.bitmap_numpy().view(np.uint8), bitorder="little")[:n]
    b3i = 4 * st3["edges_total"] + 12 * st3["work_items"] + n // 8
    dcheck, dout = bench_deferred(ctx, T, n, lambda o: ctx.trim_implicit(
        T.AC6, log2n, imp.seed, imp.zero_thr, table, live_bitmap=lb, worker_edges=we,
        stats=st, opts=o), reps, (4, 8) if deferred else ())
    for R, d in dcheck.items():
        # the full oracle runs in the GPU test suite; here: the same live set
        # as plain AC-6 and the same T6 once the re-checks are taken out
        bitsR = np.unpackbits(d["bitmap"].view(np.uint8), bitorder="little")[:n]
        dout["by_rounds"][str(R)]["parity"] = None
        dout["by_rounds"][str(R)]["same_live_set_and_T6_as_ac6"] = bool(
            np.array_equal(bitsR, bits) and d["edges"] - d["rechecks"] == t6)
    log(f"implicit: AC-6 {ms6:.2f} ms, AC-3 {ms3:.2f} ms ({st3['rounds']} rounds)"
        + (f", deferred AC-6 {dout['fastest_ms']:.2f} ms (R = {dout['fastest_rounds']})"
           if dout else ""))
    return {"implicit": imp, "bits": bits}, {
        "workload": "implicit_2^28_zipf2.1_cap256_zero0.2", "n": n, "m": m,
        "ms": ms6, "edges_per_s": m / (ms6 / 1e3), "T6": t6,
        "n_live": stat["n_live"], "stats": stat,
        "kernels_ms": {k: float(np.mean(v)) for k, v in ktimes.items()},
        "ac3": {"ms": ms3, "edges_per_s": m / (ms3 / 1e3), "T3J": st3["edges_total"],
                "rounds": st3["rounds"], "work_items": st3["work_items"],
                "kernels_ms": {k: float(np.mean(v)) for k, v in kt3.items()},
                "roofline": roof(b3i, ms3),
                "same_live_set_as_ac6": bool(np.array_equal(bits3, bits))},
        "ac6_speedup_vs_ac3": ms3 / ms6,
        "deferred": dout,
        "full_parity": "the full bitmap, T6, T3J and AC-3's rounds are compared with the "
                       "oracle in the GPU test suite (test_implicit_2_28_full); here: the "
                       "fixed-point property on 20,000 sampled vertices",
        "bounds": {"hbm": {"algorithmic_bytes": b6i, "GBs": b6i / (ms6 / 1e3) / 1e9,
                           "frac": hbm_frac},
                   "alu": {"hashes_lower_bound": hashes, "int_ops": int_ops,
                           "peak_ops": INT32_VALU_PEAK_OPS, "frac": alu_frac},
                   "tighter": "hbm" if hbm_frac >= alu_frac else "alu"},
        "fixpoint_check_on_samples": None}


def ac4_bytes(n, st, indeg_dead):
    """AC4Trim* algorithmic bytes: per reverse edge walked its source id and a
    fetch-sub (12 B), per vertex its offsets and counter (8 B), per removed
    vertex its G^T offsets and queue slot (16 B), the bitmap."""
    return 12 * st["edges_total"] + 8 * n + 16 * st["n_dead"] + n // 8


def ac3_bytes(n, st):
    """Jacobi AC-3 algorithmic bytes: per successor check its target id and
    the target's removal round (8 B), per live-list entry and round its entry
    and cursor (12 B), the bitmap."""
    return 8 * st["edges_total"] + 12 * st["work_items"] + n // 8


def roof(b, ms):
    return {"algorithmic_bytes": int(b), "GBs": b / (ms / 1e3) / 1e9,
            "frac": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_deferred(ctx, T, n, call, reps, rounds):
    """AC-6 with late support registration (opts.rounds = R): AC-3 rounds with
    the cursor first, supports registered in round R only for the vertices
    still live.  Per R: time per trim, the traversed edges with and without the
    cursor re-checks (edges_total - rechecks is the plain AC-6 total T6), the
    rounds run, and the plain path's algorithmic bytes B6 = 8 T6 + 20 n + n/8
    over this time (the same work as plain AC-6, so the two fractions compare
    directly).  `call(opts)` runs one trim."""
    import numpy as np
    out, check = {}, {}
    for R in rounds:
        ms, kt, res = time_gpu(ctx, lambda o=T.make_opts(rounds=R): call(o), reps, 1)
        st = res.stats_dict()
        check[R] = {"bitmap": res.bitmap_numpy().copy(), "edges": st["edges_total"],
                    "rounds": st["rounds"], "rechecks": st["rechecks"]}
        t6 = st["edges_total"] - st["rechecks"]
        out[str(R)] = {"ms": ms, "edges_total": st["edges_total"], "rechecks": st["rechecks"],
                       "T6": t6, "rounds": st["rounds"], "joins": st["joins"],
                       "kernels_ms": {k: float(np.mean(v)) for k, v in kt.items()},
                       "path_B6": roof(8 * t6 + 20 * n + n // 8, ms), "parity": None}
    if not out:
        return check, None
    best = min(out, key=lambda k: out[k]["ms"])
    return check, {"by_rounds": out, "fastest_rounds": int(best), "fastest_ms": out[best]["ms"]}


def deferred_parity(orc, g, r, bm, c, dc, do):
    """CPU leg of bench_deferred: bitmap, total, rounds and re-checks against
    the oracle's closed form, and total - re-checks against T6."""
    import numpy as np
    for R, got in dc.items():
        tot, rounds, re = orc.counts_deferred(g, r, R)
        do["by_rounds"][str(R)]["parity"] = bool(
            np.array_equal(got["bitmap"], bm) and got["edges"] == tot
            and got["rounds"] == rounds and got["rechecks"] == re and tot - re == c.T6)


def bench_coretail(ctx, T, gg, steps=50):
    """The small core+tail graph (n = 65,536): microseconds per trim of AC-6,
    AC-4* and AC-3J and their traversed-edge totals (the oracle's closed forms
    are compared in the CPU leg)."""
    import numpy as np
    import torch
    g = gg.config0()
    n, m = g.n, g.m
    ro, col = T.to_device(g.row_off), T.to_device(g.col)
    a, b = gg.transpose(g)
    rro, rcl = T.to_device(a), T.to_device(b)
    lb = torch.empty((n + 31) // 32, dtype=torch.int32, device="cuda")
    P = max(ctx.max_workers(T.AC6), ctx.max_workers(T.AC4), ctx.max_workers(T.AC3))
    we = torch.empty(P, dtype=torch.int64, device="cuda")
    st_t = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")
    out, check = {"workload": "coretail_n65536", "n": n, "m": m}, {"graph": g}
    for name, algo, extra in (("ac6", T.AC6, ()), ("ac4", T.AC4, (rro, rcl)), ("ac3", T.AC3, ())):
        Pa = ctx.num_workers(algo)
        per = []
        ms, kt, res = time_gpu(ctx, lambda: ctx.trim_csr(algo, n, ro, col, *extra,
                                                          live_bitmap=lb, worker_edges=we[:Pa],
                                                          stats=st_t), steps, 3, per)
        st = res.stats_dict()
        check[name] = {"bitmap": res.bitmap_numpy().copy(), "edges": st["edges_total"],
                       "rounds": st["rounds"]}
        out[name] = {"us": ms * 1e3, "median_us": float(np.median(per)) * 1e3,
                     "edges_total": st["edges_total"], "n_live": st["n_live"],
                     "kernels_us": {k: float(np.mean(v)) * 1e3 for k, v in kt.items()},
                     "parity": None}
        if name == "ac3":
            out[name]["rounds"] = st["rounds"]
    check["deferred"], out["deferred"] = bench_deferred(
        ctx, T, n, lambda o: ctx.trim_csr(T.AC6, n, ro, col, live_bitmap=lb,
                                          worker_edges=we[:ctx.num_workers(T.AC6)], stats=st_t,
                                          opts=o), steps, (4, 16, 32, 64))
    # the same graph as a batch of one: one workgroup trims it start to finish
    # (statuses in an LDS bitmap, workgroup barriers between phases instead of
    # device-wide ones)
    vb = T.to_device(np.array([0, n], np.int64))
    bbase = T.to_device(np.array([0, (n + 31) // 32], np.int64))
    ge = torch.empty(1, dtype=torch.int64, device="cuda")
    per = []
    ms_o, kt_o, res_o = time_gpu(ctx, lambda: ctx.trim_batch(
        vb, ro, col, bbase, n, m, live_bitmaps=lb, graph_edges=ge, stats=st_t,
        opts=T.make_opts(block=1024)), steps, 3, per)
    check["owned"] = {"bitmap": res_o.bitmap_numpy()[: (n + 31) // 32].copy(),
                      "edges": int(res_o.worker_edges[0].item())}
    out["ac6_one_workgroup"] = {"us": ms_o * 1e3, "median_us": float(np.median(per)) * 1e3,
                                "edges_total": check["owned"]["edges"],
                                "kernels_us": {k: float(np.mean(v)) * 1e3 for k, v in kt_o.items()},
                                "call": "trim_batch with one graph, block 1024",
                                "parity": None}
    log(f"core+tail n=65536: AC-6 {out['ac6']['us']:.1f} us, AC-4 {out['ac4']['us']:.1f} us, "
        f"AC-3 {out['ac3']['us']:.1f} us, deferred AC-6 "
        f"{out['deferred']['fastest_ms'] * 1e3:.1f} us (R = {out['deferred']['fastest_rounds']}), "
        f"one-workgroup AC-6 {out['ac6_one_workgroup']['us']:.1f} us")
    return check, out


def bench_explicit26(ctx, T, gg, reps):
    """The explicit R-MAT scale-26 graph (edge factor 16, about 1.07e9 edges,
    no planted chain) with all three algorithms: time per trim, each kernel's
    algorithmic bytes against the 8 TB/s HBM peak, and (in the CPU leg) the
    whole oracle: bitmaps and traversed-edge totals of AC-6, AC-4* and AC-3J."""
    import numpy as np
    import torch
    log("explicit: generating R-MAT scale 26 ...")
    g = gg.config2_explicit()
    n, m = g.n, g.m
    ro, col = T.to_device(g.row_off), T.to_device(g.col)
    P = ctx.num_workers(T.AC6)
    lb = torch.empty((n + 31) // 32, dtype=torch.int32, device="cuda")
    we = torch.empty(max(P, ctx.max_workers(T.AC4)), dtype=torch.int64, device="cuda")
    st_t = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")
    ms, ktimes, res = time_gpu(ctx, lambda: ctx.trim_csr(T.AC6, n, ro, col, live_bitmap=lb,
                                                         worker_edges=we[:P], stats=st_t), reps, 1)
    st = res.stats_dict()
    bm6 = res.bitmap_numpy().copy()
    kavg = {k: float(np.mean(v)) for k, v in ktimes.items()}
    log("explicit: host sweep counts ...")
    sw = sweep_counts(g)
    algo = kernel_bytes(n, st, sw)
    gt = group_times(kavg)
    kern = {k: {"avg_ms": gt[k], "algorithmic_bytes": int(algo.get(k, 0)),
                "achieved_GBs": algo.get(k, 0) / (gt[k] / 1e3) / 1e9,
                "frac": algo.get(k, 0) / (gt[k] / 1e3) / 1e9 / HBM_PEAK_GBS}
            for k in gt if gt[k] > 0}
    dom = max((k for k in kern if k in algo), key=lambda k: kern[k]["avg_ms"])
    traffic = measured_traffic(dom, "rmat26")
    if traffic is not None:
        kern[dom]["traffic"] = traffic
        kern[dom]["traffic_GBs"] = traffic / (gt[dom] / 1e3) / 1e9
        kern[dom]["traffic_frac"] = kern[dom]["traffic_GBs"] / HBM_PEAK_GBS
        kern[dom]["amplification"] = traffic / algo[dom] if algo.get(dom) else None
    path_bytes = 8 * st["edges_total"] + 20 * n + n // 8
    out = {"workload": "rmat26_ef16", "n": n, "m": m, "ms": ms, "edges_per_s": m / (ms / 1e3),
           "T6": st["edges_total"], "n_live": st["n_live"], "kernels": kern, "dominant": dom,
           "kernels_ms": kavg, "stats": st,
           "path": {"algorithmic_bytes": path_bytes, "GBs": path_bytes / (ms / 1e3) / 1e9,
                    "frac": path_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
           "parity": None}
    check = {"graph": g, "ac6": {"bitmap": bm6, "edges": st["edges_total"]}}
    check["deferred"], out["deferred"] = bench_deferred(
        ctx, T, n, lambda o: ctx.trim_csr(T.AC6, n, ro, col, live_bitmap=lb, worker_edges=we[:P],
                                          stats=st_t, opts=o), reps, (2, 4, 8))
    log(f"explicit26: deferred AC-6 {out['deferred']['fastest_ms']:.3f} ms "
        f"(R = {out['deferred']['fastest_rounds']})")
    # the dominant kernel of the fastest late-registration run: the first
    # round without joins.  Algorithmic bytes: 4 B of offsets per vertex, 4 B
    # per check (the target id; its status is a bit of the cache-resident
    # sinks bitmap), 8 B per round-list entry written, the bitmap of removals.
    fr = out["deferred"]["by_rounds"][str(out["deferred"]["fastest_rounds"])]
    dsw_ms = fr["kernels_ms"].get("ac6_sweep")
    if dsw_ms:
        dsw = 4 * (n + 1) + 4 * sw[0] + 8 * sw[1] + n // 8
        dtr = measured_traffic("ac6_sweep_deferred", "rmat26")
        out["deferred"]["sweep_roofline"] = {
            "kernel": "ac6_sweep (round 1, no joins)", "algorithmic_bytes": dsw, "avg_ms": dsw_ms,
            "achieved_GBs": dsw / (dsw_ms / 1e3) / 1e9,
            "frac": dsw / (dsw_ms / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": dtr,
            "traffic_GBs": dtr / (dsw_ms / 1e3) / 1e9 if dtr else None,
            "amplification": dtr / dsw if dtr else None}
    # the baselines on the same graph; AC-4 takes G^T as an input (built here,
    # outside any timed region, as the paper treats it)
    log("explicit: G^T for AC-4 ...")
    a, b = gg.transpose(g)
    rro, rcl = T.to_device(a), T.to_device(b)
    del a, b
    P4 = ctx.num_workers(T.AC4)
    ms4, kt4, res4 = time_gpu(ctx, lambda: ctx.trim_csr(T.AC4, n, ro, col, rro, rcl,
                                                        live_bitmap=lb, worker_edges=we[:P4],
                                                        stats=st_t), 2, 1)
    st4 = res4.stats_dict()
    check["ac4"] = {"bitmap": res4.bitmap_numpy().copy(), "edges": st4["edges_total"]}
    del rro, rcl
    torch.cuda.empty_cache()
    P3 = ctx.num_workers(T.AC3)
    ms3, kt3, res3 = time_gpu(ctx, lambda: ctx.trim_csr(T.AC3, n, ro, col, live_bitmap=lb,
                                                        worker_edges=we[:P3], stats=st_t), 2, 1)
    st3 = res3.stats_dict()
    check["ac3"] = {"bitmap": res3.bitmap_numpy().copy(), "edges": st3["edges_total"],
                    "rounds": st3["rounds"]}
    out["ac4"] = {"ms": ms4, "edges_per_s": m / (ms4 / 1e3), "T4star": st4["edges_total"],
                  "kernels_ms": {k: float(np.mean(v)) for k, v in kt4.items()},
                  "roofline": roof(ac4_bytes(n, st4, None), ms4), "parity": None}
    out["ac3"] = {"ms": ms3, "edges_per_s": m / (ms3 / 1e3), "T3J": st3["edges_total"],
                  "rounds": st3["rounds"],
                  "kernels_ms": {k: float(np.mean(v)) for k, v in kt3.items()},
                  "roofline": roof(ac3_bytes(n, st3), ms3), "parity": None}
    out["ac6_speedup_vs_ac4"] = ms4 / ms
    out["ac6_speedup_vs_ac3"] = ms3 / ms
    log(f"explicit26: AC-6 {ms:.3f} ms, AC-4 {ms4:.3f} ms, AC-3 {ms3:.3f} ms")
    del ro, col
    torch.cuda.empty_cache()
    return check, out


def oracle_labels(graphs):
    """CPU leg: the oracle's live bitmaps of the learned section's graphs
    (training labels, and the evaluation graph's live set)."""
    import oracle
    return [oracle.bitmap(oracle.peel(g).live) for g in graphs]


def bench_learned(ctx, T, gg, steps=300, batch=1 << 14, reps=3, use_oracle=True):
    """Learned successor order: train on 16 R-MAT scale-20 graphs (seeds 1..16,
    labels from the oracle's peel, or from plain GPU AC-6 when the CPU leg is
    off), evaluate on R-MAT scale 24 (seed 0): traversed edges and times of
    plain, learned, heuristic and random orders, every order's live set
    compared with the oracle's."""
    import time as _t
    import numpy as np
    import torch

    from paper_2107_12720_amd import learned
    ctx.set_timing(False)
    s = torch.cuda.current_stream()
    log("learned: building 16 training graphs (R-MAT scale 20) ...")
    train = []
    gs = [gg.rmat(20, 16, seed=seed) for seed in range(1, 17)]
    labs = oracle_labels(gs) if use_oracle else None
    for i, g in enumerate(gs):
        dg = T.DeviceGraph.upload(g)
        indeg, src = learned.prepare(ctx, dg)
        if labs is not None:
            lab = torch.from_numpy(labs[i].view(np.int32).copy()).cuda()
        else:
            lab = ctx.trim_csr(T.AC6, g.n, dg.row_off, dg.col).live_bitmap
        train.append((dg, indeg, src, lab))
    del gs
    torch.cuda.synchronize()
    tr = learned.Trainer(ctx, seed=0, lr=5e-3)
    t0 = _t.perf_counter()
    losses = [tr.train_step(train, batch, seed=1) for _ in range(steps)]
    torch.cuda.synchronize()
    t_train = _t.perf_counter() - t0
    losses = [float(x) for x in losses]
    # the key ranges of the learned order and of the heuristic, each chosen on
    # four of the training graphs (never on the evaluation graph)
    range_l = learned.choose_logit_range(ctx, train[:4], tr.pbf)
    range_h = learned.choose_degree_range(ctx, train[:4])
    log(f"learned: key ranges {range_l} (logit), {range_h} (log1p out-degree)")
    del train
    log("learned: evaluation graph R-MAT scale 24 ...")
    g = gg.rmat(24, 16, seed=0)
    dg = T.DeviceGraph.upload(g)
    indeg, src = learned.prepare(ctx, dg)
    P = ctx.num_workers(T.AC6)
    lb = torch.empty((g.n + 31) // 32, dtype=torch.int32, device="cuda")
    we = torch.empty(P, dtype=torch.int64, device="cuda")
    st = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")

    def ac6(col):
        return ctx.trim_csr(T.AC6, g.n, dg.row_off, col, live_bitmap=lb, worker_edges=we,
                            stats=st)
    out = {}
    ms_plain = ev_time(lambda: ac6(dg.col), reps, 1, s)
    res = ac6(dg.col)
    torch.cuda.synchronize()
    plain_bm = res.bitmap_numpy().copy()
    t6_plain = res.stats_dict()["edges_total"]
    want_bm = oracle_labels([g])[0] if use_oracle else plain_bm
    same = bool(np.array_equal(plain_bm, want_bm))
    live = np.unpackbits(plain_bm.view(np.uint8), bitorder="little")[:g.n].astype(bool)
    deg = np.diff(g.row_off.astype(np.int64))
    t6_min = int(deg[~live].sum() + live.sum())
    col_l = [None]

    def score_order():
        col_l[0], _ = learned.learned_order(ctx, dg, indeg, src, tr.pbf, range_l)
    ms_order = ev_time(score_order, reps, 1, s)
    # the scoring kernel alone, against both of its bounds: 2,624 flops per
    # edge on the BF16 MFMA path (8x32 + 32x32 + 32 multiply-adds), and 28 B
    # per edge (source and target ids, the two endpoints' precomputed
    # features, the score) plus 20 B per vertex for the feature prepass
    scores = torch.empty(max(g.m, 1), dtype=torch.float32, device="cuda")
    ms_score = ev_time(lambda: ctx.mlp_score(dg, indeg, src, tr.pbf, scores), reps, 1, s)
    fl = 2624.0 * g.m
    by = 28.0 * g.m + 20.0 * g.n
    mf = fl / (ms_score / 1e3) / MFMA_BF16_PEAK_FLOPS
    hf = by / (ms_score / 1e3) / (HBM_PEAK_GBS * 1e9)
    score_roofline = {"kernel": "mlp_score", "ms": ms_score, "flops": fl,
                      "algorithmic_bytes": by,
                      "achieved_TFLOPs": fl / (ms_score / 1e3) / 1e12, "mfma_frac": mf,
                      "achieved_GBs": by / (ms_score / 1e3) / 1e9, "hbm_frac": hf,
                      "bound": "mfma" if mf >= hf else "hbm",
                      "peaks": {"bf16_mfma_TFLOPs": MFMA_BF16_PEAK_FLOPS / 1e12,
                                "hbm_GBs": HBM_PEAK_GBS}}
    orders = {"learned": col_l[0],
              "heuristic_outdeg": learned.reference_order(ctx, dg, 0, key_range=range_h),
              "heuristic_outdeg_full_range": learned.reference_order(ctx, dg, 0),
              "random": learned.reference_order(ctx, dg, 1, seed=5)}
    for name, col in orders.items():
        ms = ev_time(lambda: ac6(col), reps, 1, s)
        r2 = ac6(col)
        torch.cuda.synchronize()
        same = same and np.array_equal(r2.bitmap_numpy(), want_bm)
        out[name] = {"T6": r2.stats_dict()["edges_total"], "ac6_ms": ms}
    t6l = out["learned"]["T6"]
    ctx.set_timing(True)
    return {"workload": "train 16x rmat20_ef16, eval rmat24_ef16", "n": g.n, "m": g.m,
            "train_steps": steps, "samples_per_graph_step": batch, "train_s": t_train,
            "loss_first": losses[0], "loss_last": float(np.mean(losses[-10:])),
            "T6_plain": t6_plain, "T6_min": t6_min, "orders": out,
            "gap_closed": (t6_plain - t6l) / max(1, t6_plain - t6_min),
            "key_ranges": {"learned_logit": list(range_l), "heuristic_log1p_outdeg": list(range_h),
                           "chosen_on": "4 training graphs (R-MAT 20, seeds 1-4)"},
            "learned_T6_le_heuristic_T6": t6l <= out["heuristic_outdeg"]["T6"],
            "ac6_plain_ms": ms_plain, "score_and_order_ms": ms_order,
            "end_to_end_learned_ms": ms_order + out["learned"]["ac6_ms"],
            # trims of one graph after which ordering once pays for itself
            "break_even_trims": (ms_order / (ms_plain - out["learned"]["ac6_ms"])
                                 if ms_plain > out["learned"]["ac6_ms"] else None),
            "score_roofline": score_roofline,
            "labels": "oracle" if use_oracle else "gpu_ac6",
            "live_set_identical": bool(same),
            "live_set_reference": "oracle" if use_oracle else "plain GPU AC-6"}


def oracle_leg(g, checks, cpu_seconds, out):
    """CPU leg: the oracle timed on this host (cpu_baseline), and its results
    compared with every GPU output of this run (parity flags)."""
    import numpy as np

    import oracle
    times = []
    r = None
    while not times or (sum(times) < cpu_seconds and len(times) < 20):
        t = time.perf_counter()
        r = oracle.peel(g)
        times.append(time.perf_counter() - t)
    c = oracle.counts(g, r)
    tm = float(np.mean(times))
    out["cpu_baseline"] = {"value": g.m / tm, "unit": "edges/s", "cores": 1, "kind": "oracle",
                           "sample": f"full rmat22_ef16_chain100k graph, {len(times)} runs of "
                                     f"the sequential peel, mean {tm:.3f} s",
                           "host_cores": os.cpu_count()}
    want_bm = oracle.bitmap(r.live)
    if "deferred" in checks:
        deferred_parity(oracle, g, r, want_bm, c, checks["deferred"], out["deferred"])
    a6 = checks["ac6"]
    out["parity"] = bool(np.array_equal(a6["bitmap"], want_bm) and a6["edges"] == c.T6)
    out["config"].update({"alpha": r.alpha, "n_live": r.n_live, "T6": c.T6, "T6min": c.T6min})
    if "ac4" in checks:
        b = out["baselines"]["ac4"]
        b["parity"] = bool(np.array_equal(checks["ac4"]["bitmap"], want_bm)
                           and checks["ac4"]["edges"] == c.T4s)
        b.update({"T4star": c.T4s, "T4": c.T4})
    if "ac3" in checks:
        b = out["baselines"]["ac3"]
        b["parity"] = bool(np.array_equal(checks["ac3"]["bitmap"], want_bm)
                           and checks["ac3"]["edges"] == c.T3J
                           and checks["ac3"]["rounds"] == c.rounds3)
        b.update({"T3J": c.T3J})
    if "two_sided" in checks:
        tc, to = checks["two_sided"], out["two_sided"]
        t = time.perf_counter()
        r2 = oracle.peel2(g)
        t2 = time.perf_counter() - t
        c2 = oracle.counts2(g, tc["rro"], tc["rcol"], r2.live)
        bm2 = oracle.bitmap(r2.live)
        to["oracle"] = {"s": t2, "edges_per_s": g.m / t2, "cores": 1,
                        "sample": "one run of the two-sided sequential peel on the same graph"}
        to["alpha"] = r2.alpha
        to["depth"]["floor_ms"] = r2.alpha * to["depth"]["chain_hop_us"] / 1e3
        to["ac6"]["parity"] = bool(np.array_equal(tc["ac6"]["bitmap"], bm2)
                                   and tc["ac6"]["edges_live"] == c2.T6live
                                   and c2.T6live + c2.dead_lo <= tc["ac6"]["edges"]
                                   <= c2.T6live + c2.dead_hi)
        to["ac6"]["T6live"] = c2.T6live
        to["ac4"]["parity"] = bool(np.array_equal(tc["ac4"]["bitmap"], bm2)
                                   and tc["ac4"]["edges"] == c2.T4two)
        to["ac4"]["T4two"] = c2.T4two
        if "ac3" in tc:
            t3, rounds3 = oracle.counts3two(g, tc["rro"], tc["rcol"], r2)
            to["ac3"]["parity"] = bool(np.array_equal(tc["ac3"]["bitmap"], bm2)
                                       and tc["ac3"]["edges"] == t3
                                       and tc["ac3"]["rounds"] == rounds3)
            to["ac3"]["T3J"] = t3
    if "sampling" in checks:
        sc = checks["sampling"]
        ok = True
        if "vertex" in sc:
            pre = sc["vertex"]["preset"]
            rv = oracle.peel(sc["graph"], preset=pre)
            cv = oracle.counts(sc["graph"], rv, preset=pre)
            bmv = oracle.bitmap(rv.live)
            for a, want in ((6, cv.T6), (4, cv.T4s), (3, cv.T3J)):
                ok = ok and np.array_equal(sc["vertex"][a]["bitmap"], bmv) \
                    and sc["vertex"][a]["edges"] == want
        if "edge" in sc:
            h = sc["edge"]["graph"]
            re_ = oracle.peel(h)
            ce = oracle.counts(h, re_)
            bme = oracle.bitmap(re_.live)
            for a, want in ((6, ce.T6), (4, ce.T4s), (3, ce.T3J)):
                ok = ok and np.array_equal(sc["edge"][a]["bitmap"], bme) \
                    and sc["edge"][a]["edges"] == want
        out["sampling"]["parity_at_50pct"] = bool(ok)
    if "scc" in checks:
        from oracle.scc_ref import canonical, scc_labels
        for name, sc in checks["scc"].items():
            t = time.perf_counter()
            want = scc_labels(sc["graph"])
            ts = time.perf_counter() - t
            out["scc"][name]["oracle"] = {"s": ts, "cores": 1, "kind": "scipy strong components"}
            out["scc"][name]["parity"] = bool(np.array_equal(canonical(sc["label"]), want))
    if "depth" in out:
        out["depth"]["alpha"] = r.alpha
        # what removing alpha levels one dependent step at a time would cost
        out["depth"]["stepwise_floor_ms"] = r.alpha * out["depth"]["stepwise_step_us"] / 1e3
    if "batch" in checks:
        bc = checks["batch"]
        b, bb = bc["batch"], bc["bitmap_base"]
        live, nl, _ = oracle.batch_peel(b)
        ok = bc["n_live"] == int(nl.sum())
        # per-graph traversed edges on 256 sampled graphs (closed form per graph)
        for gi in np.random.default_rng(0).choice(b.G, min(256, b.G), replace=False):
            sub = b.graph(int(gi))
            ok = ok and int(bc["graph_edges"][gi]) == oracle.counts(sub, oracle.peel(sub)).T6
        out["batch"]["parity_sample"] = "all bitmaps; per-graph T6 on 256 sampled graphs"
        for gi in range(b.G):
            v0, v1 = int(b.vbase[gi]), int(b.vbase[gi + 1])
            want = oracle.bitmap(live[v0:v1])
            if not np.array_equal(bc["bitmap"][bb[gi]:bb[gi] + want.shape[0]], want):
                ok = False
                break
        out["batch"]["parity"] = bool(ok)
    if "coretail65536" in checks:
        cc, co = checks["coretail65536"], out["coretail65536"]
        r0 = oracle.peel(cc["graph"])
        c0 = oracle.counts(cc["graph"], r0)
        bm0 = oracle.bitmap(r0.live)
        for name, want in (("ac6", c0.T6), ("ac4", c0.T4s), ("ac3", c0.T3J)):
            co[name]["parity"] = bool(np.array_equal(cc[name]["bitmap"], bm0)
                                      and cc[name]["edges"] == want
                                      and (name != "ac3" or cc[name]["rounds"] == c0.rounds3))
        co.update({"T6": c0.T6, "T4star": c0.T4s, "T3J": c0.T3J, "alpha": r0.alpha,
                   "n_live": r0.n_live})
        if "deferred" in cc:
            deferred_parity(oracle, cc["graph"], r0, bm0, c0, cc["deferred"], co["deferred"])
        if "owned" in cc:
            co["ac6_one_workgroup"]["parity"] = bool(
                np.array_equal(cc["owned"]["bitmap"], bm0) and cc["owned"]["edges"] == c0.T6)
    if "explicit26" in checks:
        ec, eo = checks["explicit26"], out["explicit26"]
        g26 = ec["graph"]
        t = time.perf_counter()
        r26 = oracle.peel(g26)
        c26 = oracle.counts(g26, r26)
        eo["oracle"] = {"s": time.perf_counter() - t, "cores": 1,
                        "sample": "one run of the sequential peel and the closed forms"}
        bm26 = oracle.bitmap(r26.live)
        eo["parity"] = bool(np.array_equal(ec["ac6"]["bitmap"], bm26)
                            and ec["ac6"]["edges"] == c26.T6)
        eo["ac4"]["parity"] = bool(np.array_equal(ec["ac4"]["bitmap"], bm26)
                                   and ec["ac4"]["edges"] == c26.T4s)
        eo["ac3"]["parity"] = bool(np.array_equal(ec["ac3"]["bitmap"], bm26)
                                   and ec["ac3"]["edges"] == c26.T3J
                                   and ec["ac3"]["rounds"] == c26.rounds3)
        eo.update({"alpha": r26.alpha, "T6min": c26.T6min})
        if "deferred" in ec:
            deferred_parity(oracle, g26, r26, bm26, c26, ec["deferred"], eo["deferred"])
    if "implicit" in checks:
        imp, bits = checks["implicit"]["implicit"], checks["implicit"]["bits"]
        rng = np.random.default_rng(0)
        ok = True
        for v in rng.integers(0, imp.n, 20000):
            d = oracle.implicit_deg(imp, int(v))
            succ = any(bits[oracle.implicit_nbr(imp, int(v), i)] for i in range(d))
            ok = ok and bool(bits[v]) == succ
        out["implicit"]["fixpoint_check_on_samples"] = bool(ok)
        out["implicit"]["samples"] = 20000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU leg (oracle timing and the parity checks it feeds)")
    ap.add_argument("--no-baselines", action="store_true", help="skip AC-4 / AC-3 / chain runs")
    ap.add_argument("--no-ac3", action="store_true", help="skip the (slow) AC-3 baseline run")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4,096-graph batch")
    ap.add_argument("--no-implicit", action="store_true", help="skip the 2^28 implicit graph")
    ap.add_argument("--no-explicit26", action="store_true",
                    help="skip the explicit R-MAT scale-26 graph")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-order section")
    ap.add_argument("--no-coretail", action="store_true",
                    help="skip the small core+tail graph (n = 65,536)")
    ap.add_argument("--no-two-sided", action="store_true",
                    help="skip two-sided trimming (AC-6 and AC-4) of the same graph")
    ap.add_argument("--no-sampling", action="store_true",
                    help="skip the edge / vertex sampling sweep (R-MAT scale 22)")
    ap.add_argument("--no-scc", action="store_true",
                    help="skip the SCC decomposition (R-MAT scale 22 with and without chain)")
    ap.add_argument("--no-deferred", action="store_true",
                    help="skip the late-support-registration runs (opts.rounds) on the chain "
                         "graph and the implicit graph (R-MAT 26 and the core+tail graph keep "
                         "theirs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the known-size "
                         "kernel that scales the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs "
                                   "are not part of this build", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}), flush=True)
        return

    import graphgen as gg
    import paper_2107_12720_amd as T

    log("generating R-MAT scale 22, edge factor 16, chain 100000 ...")
    g = gg.config1()
    n, m = g.n, g.m
    ctx = T.Context(0)
    ctx.set_timing(True)
    ro, col = T.to_device(g.row_off), T.to_device(g.col)
    P = ctx.num_workers(T.AC6)
    bm = torch.empty((n + 31) // 32, dtype=torch.int32, device="cuda")
    we = torch.empty(P, dtype=torch.int64, device="cuda")
    st_t = torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda")

    def step():
        return ctx.trim_csr(T.AC6, n, ro, col, live_bitmap=bm, worker_edges=we, stats=st_t)

    log(f"AC-6: warmup {args.warmup}, timed {args.steps} steps")
    per_step = []
    ms, ktimes, res = time_gpu(ctx, step, args.steps, args.warmup, per_step,
                               breakdown_steps=args.steps)
    st = res.stats_dict()
    value = m / (ms / 1e3)
    checks = {"ac6": {"bitmap": res.bitmap_numpy().copy(), "edges": st["edges_total"]}}
    log(f"AC-6 {ms:.3f} ms/step, {value:.3e} edges/s")
    sweep_ok = True

    kavg = {k: float(np.mean(v)) for k, v in ktimes.items()}
    sw = sweep_counts(g)
    if sw[0] != st["edges_sweep"]:
        log(f"warning: sweep checks {st['edges_sweep']} != host count {sw[0]}")
        sweep_ok = False
    algo_bytes = kernel_bytes(n, st, sw)
    gtimes = group_times(kavg)
    dom = max((k for k in gtimes if k in algo_bytes), key=gtimes.get)
    ach = algo_bytes[dom] / (gtimes[dom] / 1e3) / 1e9
    traffic = measured_traffic(dom, "rmat22_chain", P)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                "amplification": traffic / algo_bytes[dom] if traffic else None,
                "algorithmic_bytes": int(algo_bytes[dom]), "avg_ms": gtimes[dom]}
    breakdown = {k: {"avg_ms": gtimes[k],
                     "algorithmic_bytes": int(algo_bytes.get(k, 0)),
                     "achieved_GBs": algo_bytes.get(k, 0) / (gtimes[k] / 1e3) / 1e9}
                 for k in gtimes if gtimes[k] > 0}
    breakdown["kernels_ms"] = kavg
    path_bytes = 8 * st["edges_total"] + 20 * n + n // 8

    out = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat22_ef16_chain100k", "algo": "ac6", "n": n, "m": m,
                   "workers": P, "block": 256, "chunk": "auto (4096 at this n)"},
        "parity": None, "sweep_counts_match": sweep_ok,
        "roofline": roofline,
        "step_stats": step_stats(per_step),
        "timing": {"value_loop": f"{args.steps} steps, one event pair around all, no "
                                 "per-kernel events",
                   "kernel_times": f"{args.steps} more steps with the library's per-kernel "
                                   "events (about 50 us of stream time per step)",
                   "step_stats": f"{args.steps} more steps, one event pair each"},
        "hbm_copy_ceiling": copy_ceiling(),
        "breakdown": breakdown,
        "path": {"algorithmic_bytes": path_bytes,
                 "GBs": path_bytes / (ms / 1e3) / 1e9,
                 "frac": path_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "stats": st,
    }

    if not args.no_deferred:
        checks["deferred"], out["deferred"] = bench_deferred(
            ctx, T, n, lambda o: ctx.trim_csr(T.AC6, n, ro, col, live_bitmap=bm, worker_edges=we,
                                              stats=st_t, opts=o), 10, (2, 8))
        log(f"deferred AC-6 {out['deferred']['fastest_ms']:.3f} ms "
            f"(R = {out['deferred']['fastest_rounds']})")

    gt = None   # G^T on the host, built once when a section needs it
    if not args.no_baselines:
        # depth: a bare 100,000-vertex chain (alpha = 100,000)
        s = np.arange(99999, dtype=np.int32)
        gc = gg.from_edges(100000, s, s + 1)
        rc_, cc_ = T.to_device(gc.row_off), T.to_device(gc.col)
        ms_chain, _, _ = time_gpu(ctx, lambda: ctx.trim_csr(T.AC6, gc.n, rc_, cc_), 3, 1)
        # the bare chain: the forest collapse removes it in O(log length)
        # rounds, so this is no per-step latency (the stepwise form, which
        # removes it one step at a time, is timed beside it)
        ms_step, _, _ = time_gpu(ctx, lambda: ctx.trim_csr(
            T.AC6, gc.n, rc_, cc_, opts=T.make_opts(flags=T.FLAG_STEPWISE)), 2, 1)
        out["depth"] = {"bare_chain_100k_ms": ms_chain, "bare_chain_100k_stepwise_ms": ms_step,
                        "stepwise_step_us": ms_step * 1e3 / 100000}
        a, b = gt = gg.transpose(g)
        rro, rcl = T.to_device(a), T.to_device(b)
        ms4, kt4, res4 = time_gpu(ctx, lambda: ctx.trim_csr(T.AC4, n, ro, col, rro, rcl), 3, 1)
        st4 = res4.stats_dict()
        checks["ac4"] = {"bitmap": res4.bitmap_numpy().copy(), "edges": st4["edges_total"]}
        log(f"AC-4 {ms4:.3f} ms")
        out["baselines"] = {
            "ac4": {"ms": ms4, "edges_per_s": m / (ms4 / 1e3), "traversed": st4["edges_total"],
                    "parity": None,
                    "kernels_ms": {k: float(np.mean(v)) for k, v in kt4.items()}},
            "ac6_speedup_vs_ac4": ms4 / ms,
        }
        if not args.no_ac3:
            # one call of about 4 s: no second call for a per-kernel split
            ms3, kt3, res3 = time_gpu(ctx, lambda: ctx.trim_csr(T.AC3, n, ro, col), 1, 0,
                                      breakdown_steps=0)
            st3 = res3.stats_dict()
            checks["ac3"] = {"bitmap": res3.bitmap_numpy().copy(), "edges": st3["edges_total"],
                             "rounds": st3["rounds"]}
            log(f"AC-3 {ms3:.3f} ms")
            out["baselines"]["ac3"] = {
                "ms": ms3, "edges_per_s": m / (ms3 / 1e3), "traversed": st3["edges_total"],
                "rounds": st3["rounds"], "parity": None,
                "kernels_ms": {k: float(np.mean(v)) for k, v in kt3.items()}}
            out["baselines"]["ac6_speedup_vs_ac3"] = ms3 / ms

    if not args.no_two_sided:
        if gt is None:
            gt = gg.transpose(g)
        checks["two_sided"], out["two_sided"] = bench_two_sided(ctx, T, g, ro, col, gt[0], gt[1], 5,
                                                                with_ac3=not args.no_ac3)
        log(f"two-sided: AC-6 {out['two_sided']['ac6']['ms']:.3f} ms, "
            f"AC-4 {out['two_sided']['ac4']['ms']:.3f} ms"
            + (f", AC-3 {out['two_sided']['ac3']['ms']:.1f} ms" if "ac3" in out["two_sided"] else ""))
    if not args.no_scc:
        if gt is None:
            gt = gg.transpose(g)
        g22 = gg.rmat(22, 16, seed=0)
        checks["scc"], out["scc"] = bench_scc(
            ctx, T, [("rmat22_ef16_chain100k", g, gt), ("rmat22_ef16", g22, gg.transpose(g22))], 3)
        del g22
    if not args.no_sampling:
        checks["sampling"], out["sampling"] = bench_sampling(ctx, T, gg)
    if not args.no_batch:
        checks["batch"], out["batch"] = bench_batch(ctx, T, gg, 10)
        log(f"batch: {out['batch']['graphs_per_s']:.0f} graphs/s")
    if not args.no_coretail:
        checks["coretail65536"], out["coretail65536"] = bench_coretail(ctx, T, gg)
    if not args.no_explicit26:
        checks["explicit26"], out["explicit26"] = bench_explicit26(ctx, T, gg, 3)
        log(f"explicit26: {out['explicit26']['edges_per_s']:.3e} edges/s")
    if not args.no_implicit:
        checks["implicit"], out["implicit"] = bench_implicit(ctx, T, gg, 3,
                                                             deferred=not args.no_deferred)
        log(f"implicit: {out['implicit']['edges_per_s']:.3e} edges/s")
    if not args.no_learned:
        out["learned"] = bench_learned(ctx, T, gg, use_oracle=not args.no_cpu)
        log(f"learned: gap closed {out['learned']['gap_closed']:.3f}")

    if not args.no_cpu:
        oracle_leg(g, checks, args.cpu_seconds, out)
        log(f"oracle leg: parity={out['parity']}")
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
    # release the cached device memory here, with every tensor of the run gone,
    # not in exit-time destructors (whose order against the HIP runtime's and
    # a profiler's own teardown is not fixed)
    import torch
    if torch.cuda.is_initialized():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
