"""GPU parity for the implicit (hash-generated) graph and for packed batches.

Implicit: the oracle materialises POST with its own SplitMix64 code and peels
the result; the GPU generates successors on the fly.  Batch: every graph of the
packed batch is compared with the oracle run on that graph alone.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import check_ac6_counters, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def implicit_case(ctx, log2n, seed, algos=(6, 3)):
    import torch
    import paper_2107_12720_amd as T
    imp = gg.implicit(log2n=log2n, seed=seed)
    ro, col = oracle.implicit_csr(imp)
    g = gg.CSR(imp.n, ro, col)
    r = oracle.peel(g)
    c = oracle.counts(g, r)
    bm = oracle.bitmap(r.live)
    table = T.to_device(imp.table)
    for a in algos:
        say(f"  implicit log2n={log2n} seed={seed} AC-{a} m={g.m}")
        res = ctx.trim_implicit(a, log2n, imp.seed, imp.zero_thr, table)
        torch.cuda.synchronize()
        st = res.stats_dict()
        got = res.bitmap_numpy()[: bm.shape[0]]
        assert np.array_equal(got, bm), f"AC-{a} implicit bitmap differs"
        want = c.T6 if a == 6 else c.T3J
        assert st["edges_total"] == want == int(res.worker_edges.sum().item())
        assert st["n_live"] == r.n_live
        if a == 3:
            assert st["rounds"] == r.alpha + 1
        if a == 6:
            check_ac6_counters(g, r, st)
    return g, r


@pytest.mark.parametrize("log2n,seed", [(1, 0), (4, 1), (10, 2), (16, 3), (20, 0)])
def test_implicit_small(ctx, log2n, seed):
    implicit_case(ctx, log2n, seed)


def test_implicit_2_24(ctx):
    g, r = implicit_case(ctx, 24, 0, algos=(6, 3))
    say(f"  2^24: m={g.m} live={r.n_live} alpha={r.alpha}")


def test_implicit_zero_degree_all():
    """zero_frac = 1 makes every vertex a sink: nothing survives (no GPU state
    involved beyond one call)."""
    import torch
    import paper_2107_12720_amd as T
    c = T.Context(0)
    imp = gg.implicit(log2n=12, seed=9, zero_frac=1.0)
    res = c.trim_implicit(6, 12, imp.seed, (1 << 64) - 1, T.to_device(imp.table))
    torch.cuda.synchronize()
    assert not res.bitmap_numpy().any() and res.stats_dict()["edges_total"] == 0
    c.close()


def batch_expect(b):
    bb = b.bitmap_base()
    want_bm = np.zeros(int(bb[-1]), np.uint32)
    want_e = np.zeros(b.G, np.int64)
    n_live = 0
    for gi in range(b.G):
        g = b.graph(gi)
        r = oracle.peel(g)
        c = oracle.counts(g, r)
        want_bm[bb[gi]:bb[gi] + (g.n + 31) // 32] = oracle.bitmap(r.live)
        want_e[gi] = c.T6
        n_live += r.n_live
    return bb, want_bm, want_e, n_live


def run_batch(ctx, b, bb, opts=None, stream=None, dev=None, outs=None):
    import torch
    import paper_2107_12720_amd as T
    if dev is None:
        dev = (T.to_device(b.vbase), T.to_device(b.row_off), T.to_device(b.col), T.to_device(bb))
    vb, ro, col, bbd = dev
    if outs is None:
        lb = torch.full((int(bb[-1]),), -1, dtype=torch.int32, device="cuda")
        ge = st = None
    else:
        lb, ge, st = outs
        lb.fill_(-1)
        ge.fill_(-1)
    res = ctx.trim_batch(vb, ro, col, bbd, int(b.vbase[-1]), int(b.ebase[-1]), live_bitmaps=lb,
                         graph_edges=ge, stats=st, opts=opts, stream=stream)
    return res, dev


@pytest.mark.parametrize("G,seed,nmax", [(1, 0, 100), (7, 1, 300), (64, 2, 5000), (300, 3, 20000)])
def test_batch_small(ctx, G, seed, nmax):
    import torch
    b = gg.batch(G, seed=seed, n_range=(100, nmax))
    bb, want_bm, want_e, n_live = batch_expect(b)
    say(f"  batch G={G} sum_n={b.vbase[-1]} sum_m={b.ebase[-1]}")
    res, _ = run_batch(ctx, b, bb)
    torch.cuda.synchronize()
    assert np.array_equal(res.bitmap_numpy(), want_bm)
    assert np.array_equal(res.worker_edges.cpu().numpy(), want_e)
    st = res.stats_dict()
    assert st["n_live"] == n_live and st["edges_total"] == want_e.sum()


def test_batch_graph_capture_replays(ctx):
    """The captured launch sequence is replayed several times, with eager calls
    and host synchronisation in between; every replay must match."""
    import torch
    import paper_2107_12720_amd as T
    b = gg.batch(200, seed=11, n_range=(100, 10000))
    bb, want_bm, want_e, _ = batch_expect(b)
    s = torch.cuda.Stream()
    opts = T.make_opts(graph=True)
    dev = None
    outs = (torch.empty(int(bb[-1]), dtype=torch.int32, device="cuda"),
            torch.empty(b.G, dtype=torch.int64, device="cuda"),
            torch.empty(T.STATS_WORDS, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    g_small = gg.uniform(5000, 6000, seed=4)
    from gpu_common import check_all
    for rep in range(4):
        say(f"  graph replay {rep}")
        with torch.cuda.stream(s):
            res, dev = run_batch(ctx, b, bb, opts=opts, stream=s, dev=dev, outs=outs)
        s.synchronize()
        assert np.array_equal(res.bitmap_numpy(), want_bm), rep
        assert np.array_equal(res.worker_edges.cpu().numpy(), want_e), rep
        check_all(ctx, g_small, algos=(6,), name="eager between replays")


def test_batch_config3_full(ctx):
    """4,096 graphs, n log-uniform in [100, 1e5]: per-graph live sets from the
    oracle (one graph per thread) and per-graph traversed edges."""
    import torch
    b = gg.batch(4096, seed=0)
    bb = b.bitmap_base()
    say(f"  config3 sum_n={b.vbase[-1]} sum_m={b.ebase[-1]}")
    live, nl, al = oracle.batch_peel(b)
    res, _ = run_batch(ctx, b, bb)
    torch.cuda.synchronize()
    got = res.bitmap_numpy()
    ge = res.worker_edges.cpu().numpy()
    rng = np.random.default_rng(0)
    for gi in range(b.G):
        v0, v1 = int(b.vbase[gi]), int(b.vbase[gi + 1])
        want = oracle.bitmap(live[v0:v1])
        assert np.array_equal(got[bb[gi]:bb[gi] + want.shape[0]], want), gi
    # exact per-graph T6 on a sample of graphs (closed form per graph)
    for gi in rng.choice(b.G, 64, replace=False):
        g = b.graph(int(gi))
        r = oracle.peel(g)
        assert ge[gi] == oracle.counts(g, r).T6, gi
    assert res.stats_dict()["n_live"] == int(nl.sum())
