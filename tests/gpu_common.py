"""Helpers shared by the GPU parity tests (imported by test modules only)."""
import sys

import numpy as np

import graphgen
import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def upload(g, with_reverse=False):
    import torch
    import paper_2107_12720_amd as T
    ro = T.to_device(g.row_off)
    col = T.to_device(g.col) if g.m else torch.zeros(1, dtype=torch.int32, device="cuda")
    rro = rc = None
    if with_reverse:
        a, b = graphgen.transpose(g)
        rro = T.to_device(a)
        rc = T.to_device(b) if g.m else torch.zeros(1, dtype=torch.int32, device="cuda")
    return ro, col, rro, rc


def run_csr(ctx, g, algo, opts=None, dev=None):
    """Run one algorithm through the C ABI; returns (bitmap uint32[], edges, stats)."""
    import torch
    dev = dev or upload(g, with_reverse=(algo == 4))
    ro, col, rro, rc = dev
    res = ctx.trim_csr(algo, g.n, ro, col if g.m else None, rro, rc if g.m else None, opts=opts)
    torch.cuda.synchronize()
    st = res.stats_dict()
    bm = res.bitmap_numpy()[: (g.n + 31) // 32]
    return bm, int(res.worker_edges.sum().item()), st


def sweep_counts(g):
    """(checks, joins, casualties) of the AC-6 first sweep.  During it only
    out-degree-0 vertices are removed, so v joins the list of its first
    successor with out-degree > 0 (checking every successor up to it) or, with
    none, checks all its successors and is queued for removal."""
    deg = np.diff(g.row_off.astype(np.int64))
    checks = joins = cas = 0
    if g.m:
        ok = np.flatnonzero(deg[g.col] > 0)
        start = g.row_off[:-1].astype(np.int64)
        j = np.searchsorted(ok, start)
        first = np.where(j < ok.size, ok[np.minimum(j, max(ok.size - 1, 0))] if ok.size else -1, -1)
        has = (deg > 0) & (first >= start) & (first < g.row_off[1:])
        checks = int(np.where(has, first - start + 1, deg).sum())
        joins = int(has.sum())
        cas = int(((deg > 0) & ~has).sum())
    return checks, joins, cas


def expected(g):
    r = oracle.peel(g)
    c = oracle.counts(g, r)
    return r, c, oracle.bitmap(r.live)


def check_all(ctx, g, algos=(6, 4, 3), opts=None, name=""):
    r, c, bm = expected(g)
    want = {6: c.T6, 4: c.T4s, 3: c.T3J}
    for a in algos:
        say(f"  [{name}] AC-{a} n={g.n} m={g.m}")
        got, edges, st = run_csr(ctx, g, a, opts=opts)
        assert np.array_equal(got, bm), f"AC-{a} bitmap differs on {name}"
        assert edges == want[a] == st["edges_total"], (a, edges, want[a], st)
        assert st["n_live"] == r.n_live and st["n_dead"] == g.n - r.n_live, st
        if a == 3:
            assert st["rounds"] == r.alpha + 1, st
            assert st["q_highwater"] == 0, st
        else:
            # private LDS queues never hold more than their 1,024 entries
            assert 0 <= st["q_highwater"] <= 1024, st
        if a == 6:
            checks, joins, _ = sweep_counts(g)
            deg0 = int((np.diff(g.row_off) == 0).sum())
            # every vertex removed after the sweep is closed exactly once, and
            # every join except the last one of a live vertex is handed back once
            assert st["edges_sweep"] == checks, (st, checks)
            assert st["closes"] == (g.n - r.n_live) - deg0, st
            assert st["visited"] == joins + st["joins"] - r.n_live, (st, joins)
    return r, c
