"""GPU parity of the SCC decomposition (forward-backward search with
trimming, Section 1.1) against the oracle's strongly connected components.

The partition must be identical: the GPU labels, relabelled with the smallest
vertex id of each class, must equal the oracle's canonical labels vertex for
vertex, and every label must be the id of a vertex of its own component.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.scc_ref import canonical, scc_labels, summary
from gpu_common import say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def check_scc(ctx, g, opts=None, name="", want=None):
    import torch
    say(f"  [{name}] SCC n={g.n} m={g.m}")
    ro, col, rro, rc = upload(g, with_reverse=True)
    label, st = ctx.trim_scc(g.n, ro, col if g.m else None, rro, rc if g.m else None, opts=opts)
    torch.cuda.synchronize()
    lab = label.cpu().numpy()[: g.n].astype(np.int64)
    want = scc_labels(g) if want is None else want
    assert (lab >= 0).all() and (lab < max(g.n, 1)).all(), name
    assert (lab[lab] == lab).all(), f"a label is not a member of its component ({name})"
    assert np.array_equal(canonical(lab), want), f"SCC partition differs on {name}"
    s = summary(want)
    assert st["n_scc"] == s["n_scc"], (st, s)
    assert 0 <= st["giant"] <= s["largest"] and st["trimmed"] <= s["n_single"], (st, s)
    return st, want


@pytest.mark.parametrize("adj,name", [
    ([], "empty"),
    ([[]], "one vertex"),
    ([[0]], "self-loop"),
    ([[1], [0]], "2-cycle"),
    ([[1], [2], [0, 3], [4], [5], [3]], "two joined 3-cycles"),
    ([[1], [2], [3], []], "path"),
    ([[1], [2], [2]], "path into a self-loop"),
    ([[1, 2], [3], [3], []], "diamond DAG"),
    ([[1, 1], [0, 0]], "duplicate edges"),
])
def test_special_cases(ctx, adj, name):
    check_scc(ctx, gg.from_adjacency(adj), name=name)


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs(ctx, seed):
    rng = np.random.default_rng(3000 + seed)
    for n, dens in ((60, 1.2), (1000, 1.0), (5000, 1.5), (30001, 2.2), (70001, 1.1)):
        g = gg.uniform(n, int(dens * n), seed=seed * 41 + n, drop_self=bool(rng.integers(2)))
        st, _ = check_scc(ctx, g, name=f"uniform n={n} seed={seed}")


def test_chain_of_two_cycles(ctx):
    """80 two-cycles in a chain whose ids decrease downstream: every colour
    round resolves only the component that holds the largest id left, so this
    needs many rounds (the method's worst case); the result must not change."""
    K = 80
    src, dst = [], []
    for i in range(K):
        a, b = 2 * i, 2 * i + 1
        src += [a, b]
        dst += [b, a]
        if i > 0:
            src.append(a)
            dst.append(a - 1)
    g = gg.from_edges(2 * K, np.array(src, np.int32), np.array(dst, np.int32))
    st, want = check_scc(ctx, g, name="chain of 2-cycles")
    assert summary(want)["n_scc"] == K


def test_config0(ctx):
    check_scc(ctx, gg.config0(), name="core+tail n=65536")


def test_rmat_with_chain(ctx):
    check_scc(ctx, gg.rmat(16, 16, seed=7, chain=3000), name="rmat16+chain")


def test_rmat_scale18(ctx):
    st, want = check_scc(ctx, gg.rmat(18, 16, seed=2), name="rmat18")
    assert st["giant"] == summary(want)["largest"], st


def test_schedules(ctx):
    import paper_2107_12720_amd as T
    g = gg.rmat(15, 8, seed=4, chain=300)
    want = scc_labels(g)
    for block, chunk, workers, sched in ((64, 64, 1, 0), (1024, 65536, 0, 1), (256, 300, 37, 3)):
        check_scc(ctx, g, opts=T.make_opts(block=block, chunk=chunk, workers=workers,
                                           schedule=sched),
                  name=f"block={block} chunk={chunk} workers={workers} schedule={sched}",
                  want=want)


def test_trimming_calls_after_scc(ctx):
    """trim_csr and trim_csr_two_sided on the same context after an SCC call."""
    from gpu_common import check_all
    from test_gpu_two_sided import check_two
    g = gg.rmat(14, 16, seed=2, chain=200)
    check_scc(ctx, g, name="rmat14")
    check_all(ctx, g, algos=(6, 4), name="rmat14 one-sided")
    check_two(ctx, g, name="rmat14 two-sided")


def test_config1_full(ctx):
    """R-MAT scale 22, edge factor 16, planted 100,000-vertex chain."""
    g = gg.config1()
    st, want = check_scc(ctx, g, name="rmat22+chain")
    say(f"  stats {st}")


def test_errors(ctx):
    import paper_2107_12720_amd as T
    g = gg.from_adjacency([[1], [0]])
    ro, col, rro, rc = upload(g, with_reverse=True)
    with pytest.raises(T.TrimError) as e:
        ctx.trim_scc(g.n, ro, col, None, rc)
    assert e.value.code == -1


def planted_pairs(g, k, seed):
    """g plus k planted 2-cycles {a, b} on new vertices, fed by (or feeding) a
    random vertex of g: after the large component is assigned they are
    components of two that the size-2 check finds."""
    rng = np.random.default_rng(seed)
    src = list(np.repeat(np.arange(g.n), np.diff(g.row_off)))
    dst = list(g.col)
    n = g.n
    for i in range(k):
        a, b = n + 2 * i, n + 2 * i + 1
        src += [a, b]
        dst += [b, a]
        hook = int(rng.integers(g.n))
        if i % 2:
            src.append(hook); dst.append(a)     # fed from the graph
        else:
            src.append(b); dst.append(hook)     # feeding the graph
    return gg.from_edges(n + 2 * k, np.array(src, np.int32), np.array(dst, np.int32))


@pytest.mark.parametrize("seed", range(4))
def test_size2_against_oracle(ctx, seed):
    import torch
    import paper_2107_12720_amd as T
    from oracle.scc_ref import size2_pairs
    rng = np.random.default_rng(seed)
    for n, dens in ((50, 1.0), (3000, 1.2), (40001, 1.5)):
        g = gg.uniform(n, int(dens * n), seed=seed * 7 + n)
        g = planted_pairs(g, max(2, n // 50), seed)
        for ratio in (1.0, 0.7):
            preset, bm = gg.sample_vertices(g.n, ratio, seed=seed + 1)
            say(f"  size-2 n={g.n} m={g.m} ratio={ratio}")
            ro, col, rro, rc = upload(g, with_reverse=True)
            pd = T.to_device(bm.view(np.int32)) if ratio < 1.0 else None
            partner, npair = ctx.trim_size2(g.n, ro, col, rro, rc, pd)
            torch.cuda.synchronize()
            got = partner.cpu().numpy()[: g.n]
            want = size2_pairs(g, preset if ratio < 1.0 else None)
            assert np.array_equal(got, want), (n, ratio)
            assert npair == int((want >= 0).sum())


def test_scc_uses_size2(ctx):
    g = planted_pairs(gg.rmat(14, 8, seed=3), 300, 5)
    st, want = check_scc(ctx, g, name="rmat14 + 300 planted pairs")
    assert st["paired"] >= 2 * 250, st
