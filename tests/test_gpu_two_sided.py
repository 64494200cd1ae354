"""GPU parity of two-sided trimming against the oracle.

Two-sided trimming also needs a live predecessor (the in-degree check over G^T
of Section 4.1).  The live bitmap must equal oracle.peel2's bit for bit.
AC-4: the edge total equals the closed form sum over removed v of
(out-degree + in-degree).  AC-6: the live vertices' checks do not depend on
the schedule and must equal oracle.counts2 T6live exactly (stats.edges_live,
read off the final cursors), the removed vertices' checks lie between the
oracle's bounds, stats.closes + stats.forest counts the vertices removed
after the start (those that had a successor and a predecessor), and
stats.forest the vertices of the out-side last-successor trees whose root
the first sweep removed (both forms run: the forest collapse and
TRIM_FLAG_STEPWISE).  AC-3: the total equals
the oracle's closed form of the two-sided rounds (oracle.counts3two) and the
rounds number alpha + 1 of two-sided peeling.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def run_two(ctx, g, algo, opts=None, dev=None):
    import torch
    ro, col, rro, rc = dev or upload(g, with_reverse=True)
    res = ctx.trim_csr_two_sided(algo, g.n, ro, col if g.m else None, rro,
                                 rc if g.m else None, opts=opts)
    torch.cuda.synchronize()
    return (res.bitmap_numpy()[: (g.n + 31) // 32], int(res.worker_edges.sum().item()),
            res.stats_dict())


def expected_two(g):
    r = oracle.peel2(g)
    rro, rcol = gg.transpose(g)
    c = oracle.counts2(g, rro, rcol, r.live)
    deg = np.diff(g.row_off.astype(np.int64))
    indeg = np.diff(rro.astype(np.int64))
    n_dead0 = int(((deg == 0) | (indeg == 0)).sum())
    t3 = oracle.counts3two(g, rro, rcol, r)
    return r, c, oracle.bitmap(r.live), n_dead0, t3


def _first_live(row_off, adj, dead0):
    """Per vertex, the position of its first neighbour outside dead0 in its
    list [row_off[v], row_off[v+1]), or -1."""
    n = row_off.size - 1
    start = row_off[:-1].astype(np.int64)
    ok = np.flatnonzero(~dead0[adj])
    j = np.searchsorted(ok, start)
    first = np.full(n, -1, np.int64)
    inb = j < ok.size
    first[inb] = ok[j[inb]]
    first[(first < start) | (first >= row_off[1:])] = -1
    return first


def forest_count2(g):
    """Vertices the two-sided forest collapse removes: the vertices the first
    sweep leaves without a live successor or a live predecessor (live: outside
    the start-removed set of vertices without either), plus every vertex whose
    out-support is its last successor and whose chain of such supports ends at
    one of them (a chain into a cycle never does)."""
    n = g.n
    if n == 0 or g.m == 0:
        return 0
    rro, rcol = gg.transpose(g)
    deg = np.diff(g.row_off.astype(np.int64))
    indeg = np.diff(rro.astype(np.int64))
    dead0 = (deg == 0) | (indeg == 0)
    fo = _first_live(g.row_off, g.col, dead0)
    fi = _first_live(rro, rcol, dead0)
    cas = ~dead0 & ((fo < 0) | (fi < 0))
    last = ~dead0 & ~cas & (fo == g.row_off[1:] - 1)
    par = np.arange(n, dtype=np.int64)
    par[last] = g.col[fo[last]]
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 2):
        par = par[par]
    at_root = par[par] == par
    return int(cas.sum() + (last & at_root & cas[par]).sum())


def check_two(ctx, g, algos=(6, 4, 3), opts=None, name="", dev=None, exp=None, stepwise=True):
    """Every algorithm in `algos` against the oracle; AC-6 also in its stepwise
    form (TRIM_FLAG_STEPWISE) unless ``stepwise`` is False."""
    import paper_2107_12720_amd as T
    r, c, bm, n_dead0, (t3, rounds3) = exp or expected_two(g)
    dev = dev or upload(g, with_reverse=True)
    runs = [(a, opts) for a in algos]
    if stepwise and 6 in algos:
        o = opts or T.make_opts()
        runs.append((6, T.make_opts(block=o.block, workers=o.workers, chunk=o.chunk,
                                    schedule=o.schedule, budget=o.budget,
                                    flags=o.flags | T.FLAG_STEPWISE)))
    want_forest = None
    for a, op in runs:
        step = bool(op and op.flags & T.FLAG_STEPWISE)
        say(f"  [{name}] two-sided AC-{a}{' stepwise' if step else ''} n={g.n} m={g.m}")
        got, edges, st = run_two(ctx, g, a, opts=op, dev=dev)
        assert np.array_equal(got, bm), f"two-sided AC-{a} bitmap differs on {name}"
        assert st["n_live"] == r.n_live and st["n_dead"] == g.n - r.n_live, st
        assert edges == st["edges_total"], st
        assert 0 <= st["q_highwater"] <= 1024, st
        if a == 4:
            assert edges == c.T4two, (edges, c)
        elif a == 3:
            assert edges == t3 and st["rounds"] == rounds3 == r.alpha + 1, (edges, t3, st)
        else:
            # the live vertices' checks, read off their final cursors, exactly
            assert st["edges_live"] == c.T6live, (st, c)
            assert c.T6live + c.dead_lo <= edges <= c.T6live + c.dead_hi, (edges, c)
            # every vertex removed after the start is removed once: by the
            # forest collapse or by a close of the propagation
            assert st["closes"] + st["forest"] == g.n - r.n_live - n_dead0, (st, n_dead0)
            if step:
                assert st["forest"] == 0 and st["jump_rounds"] == 0, st
            else:
                if want_forest is None:
                    want_forest = forest_count2(g)
                assert st["forest"] == want_forest, (st, want_forest)
                assert want_forest == 0 or st["jump_rounds"] >= 1, st
            assert st["graph_edges"] == g.m, st
    return r, c


@pytest.mark.parametrize("adj,name", [
    ([], "empty"),
    ([[], [], []], "edgeless"),
    ([[0]], "self-loop"),
    ([[1], [0]], "2-cycle"),
    ([[1], [2], [1, 3], []], "source-cycle-sink"),
    ([[1], [2], [2]], "path into a self-loop"),
    ([[1], [2], [3], []], "path"),
    ([[1, 1, 1], [0, 0]], "duplicates"),
    ([[1], [0], [0], [4], []], "cycle-in-out"),
    ([[1], [2], [0], [0], [3]], "cycle fed by a 2-cycle chain"),
])
def test_special_cases(ctx, adj, name):
    check_two(ctx, gg.from_adjacency(adj), name=name)


def test_hand_example_values(ctx):
    g = gg.from_adjacency([[1], [2], [1, 3], []])
    r, c = check_two(ctx, g, name="hand example")
    assert list(r.live) == [0, 1, 1, 0] and c.T4two == 2 and c.T6live == 5
    # two-sided AC-3: 10 checks in 2 rounds (worked out in the oracle's pins)
    assert oracle.counts3two(g, *gg.transpose(g), r) == (10, 2)


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs(ctx, seed):
    rng = np.random.default_rng(2000 + seed)
    for n, dens in ((97, 0.9), (1000, 1.3), (5000, 1.1), (20000, 2.0), (70001, 1.2)):
        g = gg.uniform(n, int(dens * n), seed=seed * 37 + n, drop_self=bool(rng.integers(2)))
        check_two(ctx, g, name=f"uniform n={n} seed={seed}")


def test_config0(ctx):
    check_two(ctx, gg.config0(), name="core+tail n=65536")


def test_two_ended_chain(ctx):
    """A path of 200,001 vertices: one-sided trimming peels it from the sink
    only, two-sided from both ends at once (100,001 steps)."""
    L = 200001
    g = gg.from_edges(L, np.arange(L - 1, dtype=np.int32), np.arange(1, L, dtype=np.int32))
    r, c = check_two(ctx, g, name="path")
    assert r.n_live == 0 and r.alpha == (L + 1) // 2


def test_dying_predecessor_hub(ctx):
    """A source feeds a hub that feeds 300,000 leaves.  The source dies at the
    start, then the hub; every leaf had the hub as its in-support.  Leaves with
    a self-loop (a second predecessor later in their list) resume and stay;
    the others lose their last predecessor and die at once."""
    N = 300000
    hub, src = 0, 1
    leaves = np.arange(2, N + 2, dtype=np.int32)
    looped = leaves[::2]
    s = np.r_[np.int32(src), np.zeros(N, np.int32), looped]
    d = np.r_[np.int32(hub), leaves, looped]
    g = gg.from_edges(N + 2, s, d)
    rro, rcol = gg.transpose(g)
    # the hub comes first in every looped leaf's predecessor list
    assert all(rcol[rro[v]] == hub for v in looped[:50])
    r, c = check_two(ctx, g, name="predecessor hub")
    assert r.n_live == looped.size


def test_rmat_with_chain(ctx):
    check_two(ctx, gg.rmat(16, 16, seed=7, chain=3000), name="rmat16+chain")


def test_rmat_scale18(ctx):
    check_two(ctx, gg.rmat(18, 16, seed=2), name="rmat18")


def test_schedule_invariance(ctx):
    import paper_2107_12720_amd as T
    g = gg.rmat(17, 8, seed=11, chain=2000)
    exp = expected_two(g)
    dev = upload(g, with_reverse=True)
    for block, chunk, workers in ((64, 64, 1), (256, 4096, 7), (1024, 65536, 0), (128, 1, 3),
                                  (512, 300, 512)):
        opts = T.make_opts(block=block, chunk=chunk, workers=workers)
        check_two(ctx, g, opts=opts, dev=dev, exp=exp,
                  name=f"block={block} chunk={chunk} workers={workers}")


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_schedule_perturbation(ctx, schedule):
    """Reversed sweep chunks (1), pauses inside the race windows (2), and both:
    twenty repeats each; output never changes."""
    import paper_2107_12720_amd as T
    N = 20000
    hub_src = np.r_[np.int32(1), np.zeros(N, np.int32), np.arange(2, N + 2, 2, dtype=np.int32)]
    hub_dst = np.r_[np.int32(0), np.arange(2, N + 2, dtype=np.int32),
                    np.arange(2, N + 2, 2, dtype=np.int32)]
    graphs = [("predecessor hub", gg.from_edges(N + 2, hub_src, hub_dst)),
              ("uniform", gg.uniform(30000, 36000, seed=4)),
              ("rmat14+chain", gg.rmat(14, 16, seed=9, chain=800))]
    for name, g in graphs:
        exp = expected_two(g)
        dev = upload(g, with_reverse=True)
        say(f"  schedule={schedule} {name}: 20 repeats of two-sided AC-6 and AC-4")
        for k in range(20):
            opts = T.make_opts(schedule=schedule, chunk=(64, 4096)[k % 2], workers=(0, 37)[k % 2])
            r, c, bm, _, _ = exp
            for a in (6, 4):
                got, edges, st = run_two(ctx, g, a, opts=opts, dev=dev)
                assert np.array_equal(got, bm), (name, a, k)
                if a == 4:
                    assert edges == c.T4two, (name, k)
                else:
                    assert c.T6live + c.dead_lo <= edges <= c.T6live + c.dead_hi, (name, k)


def test_one_sided_unchanged_after_two_sided(ctx):
    """The two calls share the context's working memory: a one-sided call after
    a two-sided one still matches the one-sided oracle."""
    from gpu_common import check_all
    g = gg.rmat(15, 16, seed=3, chain=400)
    check_two(ctx, g, name="rmat15 two-sided")
    check_all(ctx, g, algos=(6, 4), name="rmat15 one-sided")


def test_config1_full(ctx):
    """R-MAT scale 22, edge factor 16, planted 100,000-vertex chain."""
    g = gg.config1()
    say(f"  config1 n={g.n} m={g.m}")
    check_two(ctx, g, name="rmat22+chain")


def test_errors(ctx):
    import torch
    import paper_2107_12720_amd as T
    g = gg.from_adjacency([[1], [0]])
    ro, col, rro, rc = upload(g, with_reverse=True)
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr_two_sided(5, g.n, ro, col, rro, rc)
    assert e.value.code == -1
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr_two_sided(6, g.n, ro, col, None, rc)
    assert e.value.code == -1
    bad = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr_two_sided(6, g.n, ro, col, bad, rc, opts=T.make_opts(validate=True))
    assert e.value.code == -5
