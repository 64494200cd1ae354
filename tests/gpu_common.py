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


def forest_count(g):
    """Vertices the AC-6 forest collapse removes: the vertices the first sweep
    leaves without a live successor, plus every vertex whose support is its
    last successor and whose chain of such supports ends at one of them.
    Chains are followed by repeated doubling of the parent array; a chain that
    runs into a cycle never reaches such a vertex."""
    n = g.n
    if n == 0 or g.m == 0:
        return 0
    deg = np.diff(g.row_off.astype(np.int64))
    start = g.row_off[:-1].astype(np.int64)
    ok = np.flatnonzero(deg[g.col] > 0)
    j = np.searchsorted(ok, start)
    first = np.full(n, -1, np.int64)
    inb = j < ok.size
    first[inb] = ok[j[inb]]
    has = (deg > 0) & (first >= start) & (first < g.row_off[1:])
    cas = (deg > 0) & ~has
    last = has & (first == g.row_off[1:] - 1)
    par = np.arange(n, dtype=np.int64)
    par[last] = g.col[first[last]]
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 2):
        par = par[par]
    at_root = par[par] == par
    return int(cas.sum() + (last & at_root & cas[par]).sum())


def expected(g):
    r = oracle.peel(g)
    c = oracle.counts(g, r)
    return r, c, oracle.bitmap(r.live)


def check_all(ctx, g, algos=(6, 4, 3), opts=None, name="", stepwise=True):
    """Bit-exact bitmap and exact totals for each algorithm; AC-6 also in
    its stepwise form (TRIM_FLAG_STEPWISE) unless ``stepwise`` is False."""
    import paper_2107_12720_amd as T
    r, c = _check_all(ctx, g, algos, opts, name)
    if stepwise and 6 in algos:
        o = opts or T.make_opts()
        o2 = T.make_opts(block=o.block, workers=o.workers, chunk=o.chunk, schedule=o.schedule,
                         budget=o.budget, flags=o.flags | T.FLAG_STEPWISE, rounds=o.rounds)
        _check_all(ctx, g, (6,), o2, name + " stepwise")
    return r, c


def _check_all(ctx, g, algos, opts, name):
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
            check_ac6_counters(g, r, st, stepwise=bool(opts and opts.flags & 1))
    return r, c


def check_ac6_counters(g, r, st, stepwise=False):
    """Counter invariants of one AC-6 run.  Every vertex removed after the
    sweep is removed exactly once, by the forest collapse or by a close of the
    propagation; every join except the last one of a live vertex is handed
    back once, except the joins of the tree members the collapse removed
    (their lists are not walked: all their members fall in the same rounds).
    The collapse removes at least the sweep's casualties, and nothing with
    TRIM_FLAG_STEPWISE."""
    checks, joins, cas = sweep_counts(g)
    deg0 = int((np.diff(g.row_off) == 0).sum())
    assert st["edges_sweep"] == checks, (st, checks)
    assert st["closes"] + st["forest"] == (g.n - r.n_live) - deg0, st
    if stepwise:
        assert st["forest"] == 0 and st["jump_rounds"] == 0, st
    else:
        want = forest_count(g)
        assert st["forest"] == want, (st, want)
        assert want == 0 or st["jump_rounds"] >= 1, st
    members = st["forest"] - cas if st["forest"] else 0
    assert members >= 0, (st, cas)
    assert st["visited"] == joins + st["joins"] - r.n_live - members, (st, joins, cas)
