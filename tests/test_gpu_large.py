"""Full-size parity on the largest workloads: R-MAT scale 26, edge factor 16
(about 1.07e9 edges) against the whole oracle, and the implicit graph with
2^28 vertices on sampled vertices.  Generation and the sequential oracle take
about a minute each, so these tests have their own time limits."""
import pytest

import graphgen as gg
from gpu_common import check_all, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


@pytest.mark.timeout(900)
def test_config2_explicit_full(ctx):
    say("  generating R-MAT scale 26 ...")
    g = gg.config2_explicit()
    say(f"  rmat26 n={g.n} m={g.m}; oracle and AC-6 ...")
    check_all(ctx, g, algos=(6,), name="rmat26")


@pytest.mark.timeout(600)
def test_implicit_2_28_samples(ctx):
    """The implicit graph at its full size, 2^28 vertices, in the launch
    configuration the benchmark times (default options).  The oracle's own
    hash gives the degree and successors of 20,000 sampled vertices; each must
    be live iff one of its successors is live (the fixed point, on both sides:
    no removed vertex keeps a live successor, no live one lacks one)."""
    import numpy as np
    import torch
    import oracle
    import paper_2107_12720_amd as T
    imp = gg.implicit(log2n=28, seed=0)
    say("  implicit 2^28: AC-6 ...")
    res = ctx.trim_implicit(T.AC6, 28, imp.seed, imp.zero_thr, T.to_device(imp.table))
    torch.cuda.synchronize()
    st = res.stats_dict()
    bits = np.unpackbits(res.bitmap_numpy().view(np.uint8), bitorder="little")[: imp.n]
    assert st["n_live"] == int(bits.sum()) and st["n_live"] + st["n_dead"] == imp.n
    assert st["edges_total"] >= st["n_live"]
    rng = np.random.default_rng(28)
    live_seen = dead_seen = 0
    for v in rng.integers(0, imp.n, 20000):
        d = oracle.implicit_deg(imp, int(v))
        succ_live = any(bits[oracle.implicit_nbr(imp, int(v), i)] for i in range(d))
        assert bool(bits[v]) == succ_live, int(v)
        live_seen += int(bits[v])
        dead_seen += 1 - int(bits[v])
    say(f"  samples: {live_seen} live, {dead_seen} removed; n_live {st['n_live']}")
    assert live_seen > 1000 and dead_seen > 1000
