"""Failure handling through the C ABI, every condition forced from the host.

* Watchdog: opts.budget shrinks the persistent kernels' own bounded loops
  (AC-6 / AC-4 / two-sided AC-6 propagation, the AC-3 round barrier) so that
  they give up; every wavefront exits normally, trim_ctx_status reports
  TRIM_E_STALLED and stats.stalled is set.  The next call on the same
  context, with the default budget, is bit-exact against the oracle again
  (the shared queue was restored).
* Memory cap: a context whose mem_budget cannot hold a call's working memory
  returns TRIM_E_NOMEM before enqueuing anything and keeps working for calls
  that fit.
* Worker cap: opts.workers above trim_max_workers is TRIM_E_INVAL.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say, upload

pytestmark = pytest.mark.gpu

STALLED, NOMEM, INVAL = -6, -2, -1


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def chain_graph():
    g = gg.rmat(14, 8, seed=5, chain=3000)
    r = oracle.peel(g)
    return g, r, oracle.counts(g, r), oracle.bitmap(r.live)


def run(ctx, g, algo, dev, opts=None, two=False):
    import torch
    ro, col, rro, rc = dev
    if two:
        res = ctx.trim_csr_two_sided(algo, g.n, ro, col, rro, rc, opts=opts)
    else:
        res = ctx.trim_csr(algo, g.n, ro, col, rro, rc, opts=opts)
    status = ctx.status()
    torch.cuda.synchronize()
    return status, res.bitmap_numpy()[: (g.n + 31) // 32], res.stats_dict()


@pytest.mark.parametrize("algo,two", [(6, False), (4, False), (3, False), (6, True)],
                         ids=["AC-6", "AC-4", "AC-3", "two-sided AC-6"])
def test_watchdog_stalls_then_context_recovers(ctx, chain_graph, algo, two):
    import paper_2107_12720_amd as T
    g, r, c, bm = chain_graph
    dev = upload(g, with_reverse=True)
    say(f"  budget 1: AC-{algo}{' two-sided' if two else ''} on a 3000-vertex chain")
    status, _, st = run(ctx, g, algo, dev, opts=T.make_opts(budget=1), two=two)
    assert status == STALLED and st["stalled"] == 1, (status, st)
    with pytest.raises(T.TrimError) as e:
        ctx.check()
    assert e.value.code == STALLED
    say("  default budget on the same context")
    status, got, st = run(ctx, g, algo, dev, two=two)
    assert status == 0 and st["stalled"] == 0
    if two:
        r2 = oracle.peel2(g)
        assert np.array_equal(got, oracle.bitmap(r2.live))
    else:
        assert np.array_equal(got, bm)
        assert st["edges_total"] == {6: c.T6, 4: c.T4s, 3: c.T3J}[algo]


def test_generous_budget_is_not_a_stall(ctx, chain_graph):
    """A budget large enough for the work changes nothing."""
    import paper_2107_12720_amd as T
    g, r, c, bm = chain_graph
    dev = upload(g, with_reverse=True)
    for algo in (6, 4, 3):
        status, got, st = run(ctx, g, algo, dev, opts=T.make_opts(budget=1 << 20))
        assert status == 0 and np.array_equal(got, bm), algo


def test_memory_cap(chain_graph):
    import paper_2107_12720_amd as T
    g, r, c, bm = chain_graph
    with pytest.raises(T.TrimError) as e:
        T.Context(0, mem_budget=4096)           # below the control block
    assert e.value.code == NOMEM
    small = T.Context(0, mem_budget=2 << 20)   # the control block fits, no working memory
    try:
        used = small.mem_used()
        assert 0 < used <= 2 << 20
        dev = upload(g)
        with pytest.raises(T.TrimError) as e:
            small.trim_csr(6, g.n, dev[0], dev[1])
        assert e.value.code == NOMEM and small.mem_used() == used
    finally:
        small.close()
    big = T.Context(0, mem_budget=256 << 20)
    try:
        status, got, st = run(big, g, 6, upload(g))
        assert status == 0 and np.array_equal(got, bm) and st["edges_total"] == c.T6
        assert big.mem_used() <= 256 << 20
    finally:
        big.close()


def test_worker_cap(ctx, chain_graph):
    import paper_2107_12720_amd as T
    g, r, c, bm = chain_graph
    dev = upload(g, with_reverse=True)
    for algo in (6, 4, 3):
        cap = ctx.max_workers(algo)
        assert cap >= 1
        status, got, _ = run(ctx, g, algo, dev, opts=T.make_opts(workers=cap))
        assert status == 0 and np.array_equal(got, bm)
        with pytest.raises(T.TrimError) as e:
            ctx.num_workers(algo, T.make_opts(workers=cap + 1))
        assert e.value.code == INVAL
        with pytest.raises(T.TrimError) as e:
            ctx.trim_csr(algo, g.n, *dev, opts=T.make_opts(workers=cap + 1))
        assert e.value.code == INVAL
    assert ctx.max_workers(3) <= ctx.max_workers(6)
