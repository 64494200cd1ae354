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
    # AC-6 twice: stepwise (the implicit default) and with the forest collapse
    runs = [(a, 0) for a in algos] + ([(6, T.FLAG_FOREST)] if 6 in algos else [])
    for a, flags in runs:
        say(f"  implicit log2n={log2n} seed={seed} AC-{a} flags={flags} m={g.m}")
        res = ctx.trim_implicit(a, log2n, imp.seed, imp.zero_thr, table,
                                opts=T.make_opts(flags=flags))
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
            check_ac6_counters(g, r, st, stepwise=not flags)
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


def path_opts(union, **kw):
    import paper_2107_12720_amd as T
    return T.make_opts(flags=T.FLAG_BATCH_UNION if union else 0, **kw)


def batch_counters(b, st):
    """Counters of the run against the oracle: closes + forest removals = the
    removed vertices that had successors; list members handed back = joins of
    the whole run minus the live vertices' final joins (the forest collapse's
    own removals excepted: their lists are not walked)."""
    live, _, _ = oracle.batch_peel(b)
    deg = np.diff(b.row_off.astype(np.int64))
    dead_with_succ = int(((live == 0) & (deg > 0)).sum())
    assert st["closes"] + st["forest"] == dead_with_succ, st
    assert st["graph_edges"] == int(b.ebase[-1]), st


@pytest.mark.parametrize("union", [False, True], ids=["owned", "union"])
@pytest.mark.parametrize("G,seed,nmax", [(1, 0, 100), (7, 1, 300), (64, 2, 5000), (300, 3, 20000)])
def test_batch_small(ctx, G, seed, nmax, union):
    import torch
    b = gg.batch(G, seed=seed, n_range=(100, nmax))
    bb, want_bm, want_e, n_live = batch_expect(b)
    say(f"  batch G={G} sum_n={b.vbase[-1]} sum_m={b.ebase[-1]} union={union}")
    res, _ = run_batch(ctx, b, bb, opts=path_opts(union))
    torch.cuda.synchronize()
    assert np.array_equal(res.bitmap_numpy(), want_bm)
    assert np.array_equal(res.worker_edges.cpu().numpy(), want_e)
    st = res.stats_dict()
    assert st["n_live"] == n_live and st["edges_total"] == want_e.sum()
    batch_counters(b, st)


def pack_graphs(graphs):
    """A Batch holding the given CSR graphs in order (some may be empty)."""
    vbase = np.zeros(len(graphs) + 1, np.int64)
    ebase = np.zeros(len(graphs) + 1, np.int64)
    vbase[1:] = np.cumsum([g.n for g in graphs])
    ebase[1:] = np.cumsum([g.m for g in graphs])
    row_off = np.concatenate([g.row_off[:-1].astype(np.int64) + e0
                              for g, e0 in zip(graphs, ebase[:-1])] + [ebase[-1:]])
    col = np.concatenate([g.col for g in graphs] + [np.zeros(0, np.int32)]).astype(np.int32)
    return gg.Batch(vbase, ebase, row_off.astype(np.int32), col, [])


@pytest.mark.parametrize("union", [False, True], ids=["owned", "union"])
def test_batch_special_graphs(ctx, union):
    """Empty graphs, a lone sink, self-loops, cycles, a chain, a live hub and a
    dying hub (3,000 members in its S_last list) inside one batch, with odd
    word alignments."""
    import torch
    graphs = [gg.from_adjacency([]), gg.from_adjacency([[0]]), gg.from_adjacency([]),
              gg.from_adjacency([[]]), gg.from_adjacency([[1], [0]]),
              gg.from_adjacency([[1], [2], [1, 3], []]), gg.from_adjacency([]),
              gg.from_edges(70, np.arange(69, dtype=np.int32), np.arange(1, 70, dtype=np.int32)),
              gg.from_edges(3001, np.r_[np.zeros(3000, np.int32), np.arange(1, 3001, dtype=np.int32)],
                            np.r_[np.arange(1, 3001, dtype=np.int32), np.zeros(3000, np.int32)]),
              gg.from_edges(3002, np.r_[np.int32(0), np.arange(1, 3001, dtype=np.int32)],
                            np.r_[np.int32(3001), np.zeros(3000, np.int32)]),
              gg.uniform(1000, 1100, seed=3)] + [gg.from_adjacency([])] * 40
    b = pack_graphs(graphs)
    bb, want_bm, want_e, n_live = batch_expect(b)
    res, _ = run_batch(ctx, b, bb, opts=path_opts(union))
    torch.cuda.synchronize()
    assert np.array_equal(res.bitmap_numpy(), want_bm)
    assert np.array_equal(res.worker_edges.cpu().numpy(), want_e)
    assert res.stats_dict()["n_live"] == n_live


@pytest.mark.parametrize("union", [False, True], ids=["owned", "union"])
def test_batch_more_graphs_than_vertices(ctx, union):
    """300 empty graphs around a 2-cycle: G exceeds the vertex count."""
    import torch
    graphs = [gg.from_adjacency([])] * 150 + [gg.from_adjacency([[1], [0]])] + \
        [gg.from_adjacency([])] * 150
    b = pack_graphs(graphs)
    bb, want_bm, want_e, n_live = batch_expect(b)
    res, _ = run_batch(ctx, b, bb, opts=path_opts(union))
    torch.cuda.synchronize()
    assert np.array_equal(res.bitmap_numpy(), want_bm) and n_live == 2
    assert np.array_equal(res.worker_edges.cpu().numpy(), want_e)


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_batch_schedule_invariance(ctx, schedule):
    """Jitter inside the race windows, several block sizes and worker counts:
    bitmaps and per-graph totals never change."""
    import torch
    b = gg.batch(120, seed=21, n_range=(100, 30000))
    bb, want_bm, want_e, _ = batch_expect(b)
    for block, workers in ((64, 1), (256, 0), (1024, 7), (128, 300)):
        res, _ = run_batch(ctx, b, bb, opts=path_opts(False, block=block, workers=workers,
                                                      schedule=schedule))
        torch.cuda.synchronize()
        assert np.array_equal(res.bitmap_numpy(), want_bm), (block, workers)
        assert np.array_equal(res.worker_edges.cpu().numpy(), want_e), (block, workers)


@pytest.mark.parametrize("union", [False, True], ids=["owned", "union"])
def test_batch_graph_capture_replays(ctx, union):
    """The captured launch sequence is replayed several times, with eager calls
    and host synchronisation in between; every replay must match."""
    import torch
    import paper_2107_12720_amd as T
    b = gg.batch(200, seed=11, n_range=(100, 10000))
    bb, want_bm, want_e, _ = batch_expect(b)
    s = torch.cuda.Stream()
    opts = path_opts(union, graph=True)
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


@pytest.fixture(scope="module")
def config3():
    b = gg.batch(4096, seed=0)
    live, nl, al = oracle.batch_peel(b)
    return b, live, nl


@pytest.mark.parametrize("union", [False, True], ids=["owned", "union"])
def test_batch_config3_full(ctx, config3, union):
    """4,096 graphs, n log-uniform in [100, 1e5]: per-graph live sets from the
    oracle (one graph per thread) and per-graph traversed edges."""
    import torch
    b, live, nl = config3
    bb = b.bitmap_base()
    say(f"  config3 sum_n={b.vbase[-1]} sum_m={b.ebase[-1]} union={union}")
    res, _ = run_batch(ctx, b, bb, opts=path_opts(union))
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
