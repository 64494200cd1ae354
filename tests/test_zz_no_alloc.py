"""trim_csr_noalloc (AC-6 with the library's fixed per-GPU working array)
against trim_csr with TRIM_AC6 on a context, through the C ABI: the live
bitmap bit for bit, the traversed-edge total (equal to the oracle's T6), and
the schedule-independent statistics, on consecutive calls whose sizes shrink
(the array keeps the previous call's contents), at the maximum size, and after
a call abandoned by the watchdog.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say, upload

pytestmark = pytest.mark.gpu

FIXED = ("edges_total", "n_live", "n_dead", "edges_sweep", "closes", "graph_edges", "forest")


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def both(ctx, g, opts=None):
    import torch
    import paper_2107_12720_amd as T
    ro, col, _, _ = upload(g)
    a = T.trim_csr_noalloc(g.n, ro, col if g.m else None, opts=opts)
    torch.cuda.synchronize()
    b = ctx.trim_csr(6, g.n, ro, col if g.m else None, opts=opts)
    torch.cuda.synchronize()
    w = (g.n + 31) // 32
    return (a.bitmap_numpy()[:w], int(a.worker_edges.sum().item()), a.stats_dict(),
            b.bitmap_numpy()[:w], int(b.worker_edges.sum().item()), b.stats_dict())


def check(ctx, g, name, opts=None):
    r = oracle.peel(g)
    c = oracle.counts(g, r)
    bm = oracle.bitmap(r.live)
    say(f"  [{name}] n={g.n} m={g.m}")
    bm_a, ea, sa, bm_b, eb, sb = both(ctx, g, opts)
    assert np.array_equal(bm_a, bm_b) and np.array_equal(bm_a, bm), name
    assert ea == eb == c.T6 == sa["edges_total"], (name, ea, eb, c.T6)
    for k in FIXED:
        assert sa[k] == sb[k], (name, k, sa[k], sb[k])
    assert sa["stalled"] == 0 and sa["n_live"] == r.n_live


def test_two_calls_second_smaller(ctx):
    check(ctx, gg.rmat(18, 16, seed=9, chain=5000), "rmat18+chain")
    check(ctx, gg.rmat(12, 8, seed=3, chain=700), "rmat12+chain")


def test_ragged_and_degenerate(ctx):
    check(ctx, gg.core_tail(65536 - 37, seed=4), "core+tail ragged")
    check(ctx, gg.from_adjacency([[1], [0], [0], []]), "tiny")
    check(ctx, gg.from_adjacency([]), "empty")


def test_maximum_size(ctx):
    import paper_2107_12720_amd as T
    g = gg.core_tail(T.NOALLOC_MAX_N, seed=1)
    check(ctx, g, "core+tail at the maximum n")


def test_after_a_stalled_call(ctx):
    import torch
    import paper_2107_12720_amd as T
    g = gg.rmat(14, 8, seed=5, chain=3000)
    ro, col, _, _ = upload(g)
    res = T.trim_csr_noalloc(g.n, ro, col, opts=T.make_opts(budget=1))
    torch.cuda.synchronize()
    assert res.stats_dict()["stalled"] == 1
    check(ctx, g, "after a stall")


def test_argument_errors():
    import paper_2107_12720_amd as T
    g = gg.from_adjacency([[1], [0]])
    ro, col, _, _ = upload(g)
    for opts in (T.make_opts(workers=T.NOALLOC_WORKERS + 1), T.make_opts(graph=True)):
        with pytest.raises(T.TrimError) as e:
            T.trim_csr_noalloc(g.n, ro, col, opts=opts)
        assert e.value.code == -1
    with pytest.raises(T.TrimError) as e:
        T.trim_csr_noalloc(T.NOALLOC_MAX_N + 1, ro, col)
    assert e.value.code == -1 and "fixed array" in T.last_error()
