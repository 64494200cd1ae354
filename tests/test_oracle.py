"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against an
independent definition (greatest fixed point by subset search, the peeling of
Def. alpha done by whole steps, the reach-a-cycle characterisation through a
library SCC routine), a worked example printed in the paper, closed forms of
a graph family, or a published test vector.
"""
import os
import itertools

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def parse_golden(path):
    adj, fields, in_graph = [], {}, False
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line == "graph":
            in_graph = True
            continue
        if line == "end":
            in_graph = False
            continue
        if in_graph:
            _, rest = line.split(":", 1)
            adj.append([int(x) for x in rest.split()])
        else:
            k, *vals = line.split()
            fields[k] = [int(x) for x in vals]
    return adj, fields


# ------------------------------------------------------------ independent refs
def jacobi_peel(adj):
    """Def. alpha written out: each step removes, all at once, every remaining
    vertex without a remaining successor.  Returns (live, level)."""
    n = len(adj)
    alive = [True] * n
    level = [0] * n
    step = 0
    while True:
        step += 1
        rm = [v for v in range(n) if alive[v] and not any(alive[w] for w in adj[v])]
        if not rm:
            break
        for v in rm:
            alive[v] = False
            level[v] = step
    return alive, level


def greatest_by_subsets(n, adj_masks):
    """Union of every vertex subset S with: each v in S has a successor in S
    (Def. Trimmed Graph); the union of such sets is such a set, so this is the
    greatest one."""
    best = 0
    for S in range(1 << n):
        ok = True
        for v in range(n):
            if (S >> v) & 1 and not (adj_masks[v] & S):
                ok = False
                break
        if ok:
            best |= S
    return best


def reaches_cycle(g):
    """v is live iff v reaches a directed cycle (a self-loop counts): nontrivial
    strongly connected components from scipy, then reverse reachability."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components, breadth_first_order
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.row_off))
    A = sp.csr_matrix((np.ones(g.m), (src, g.col)), shape=(n, n))
    ncomp, lab = connected_components(A, directed=True, connection="strong")
    size = np.bincount(lab, minlength=ncomp)
    cyclic = size[lab] > 1
    cyclic[src[src == g.col]] = True
    # reverse reachability from every cyclic vertex via an extra super-source
    R = sp.csr_matrix((np.ones(g.m), (g.col, src)), shape=(n + 1, n + 1)).tolil()
    for v in np.nonzero(cyclic)[0]:
        R[n, v] = 1
    order = breadth_first_order(R.tocsr(), n, directed=True, return_predecessors=False)
    out = np.zeros(n, bool)
    out[order[order < n]] = True
    return out


def check_certificate(g, live, level):
    """Soundness (each LIVE vertex has a LIVE successor) plus a removal
    certificate (each DEAD vertex has only DEAD successors, all removed at a
    strictly earlier step, and its step is one more than their latest step).
    The certificate proves the live set greatest: no removed vertex can be in
    any self-supporting set, by induction on the step."""
    ro, col = g.row_off, g.col
    for v in range(g.n):
        succ = col[ro[v]:ro[v + 1]]
        if live[v]:
            assert level[v] == 0
            assert live[succ].any(), f"live {v} without live successor"
        else:
            assert not live[succ].any(), f"dead {v} with live successor"
            mx = level[succ].max() if succ.size else 0
            assert level[v] == mx + 1, f"level of {v}"


# ------------------------------------------------------------------ tests
def test_worked_example(orc, gen):
    adj, f = parse_golden(os.path.join(GOLDEN, "worked_example.txt"))
    g = gen.from_adjacency(adj)
    r = orc.peel(g)
    assert list(r.live) == f["live"]
    assert list(r.level) == f["levels"]
    assert r.alpha == f["alpha"][0]
    # removal order by steps: {v2, v5}, v4, v3, v1
    assert sorted(r.order[:2]) == [1, 4] and list(r.order[2:]) == [3, 2, 0]
    c = orc.counts(g, r)
    assert (c.T6, c.T4s, c.T4, c.T3J, c.rounds3) == (
        f["T6"][0], f["T4s"][0], f["T4"][0], f["T3J"][0], f["rounds3"][0])
    live6, t6, _ = orc.ac6_seq(g)
    assert t6 == f["T6"][0] and not live6.any()
    live3, t3, rounds = orc.ac3(g)
    assert (t3, rounds) == (f["T3J"][0], f["rounds3"][0]) and not live3.any()
    assert r.rev_edges == f["T4s"][0]


def test_splitmix64_reference_vector(orc, gen):
    # SplitMix64 from state 0 (Steele, Lea, Flood 2014; reference C by Vigna):
    # outputs are fin(k * golden) for k = 1, 2, 3, 4.
    golden = 0x9E3779B97F4A7C15
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    for k, e in enumerate(expect, 1):
        z = (golden * k) & ((1 << 64) - 1)
        assert orc.fin64(z) == e
        assert gen.fin64(z) == e


@pytest.mark.parametrize("seed", range(12))
def test_random_small_vs_stepwise_peel(orc, gen, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    m = int(rng.integers(0, 4 * n))
    g = gen.uniform(n, m, seed=seed, drop_self=bool(seed % 2))
    adj = [list(g.col[g.row_off[v]:g.row_off[v + 1]]) for v in range(n)]
    alive, level = jacobi_peel(adj)
    r = orc.peel(g)
    assert list(r.live.astype(bool)) == alive
    assert list(r.level) == level
    assert r.alpha == max(level + [0])
    check_certificate(g, r.live.astype(bool), r.level)


@pytest.mark.parametrize("seed", range(6))
def test_simulations_equal_closed_forms(orc, gen, seed):
    """The sequential AC-6 and AC-3 runs, counting every successor check, agree
    with the closed forms, and T6 <= T3(in place) <= T3J (Section 8: each edge
    at most once for AC-6; AC-3 re-checks its cursor edge every repetition)."""
    for n, m in ((50, 60), (400, 800), (2000, 2500), (3000, 9000)):
        g = gen.uniform(n, m, seed=100 + seed, drop_self=False)
        r = orc.peel(g)
        c = orc.counts(g, r)
        live6, t6, _ = orc.ac6_seq(g)
        live3, t3, rounds = orc.ac3(g, jacobi=True)
        live3i, t3i, rounds_i = orc.ac3(g, jacobi=False)
        assert (live6 == r.live).all() and (live3 == r.live).all() and (live3i == r.live).all()
        assert t6 == c.T6
        assert t3 == c.T3J and rounds == c.rounds3 == r.alpha + 1
        assert c.T6 <= t3i <= c.T3J and rounds_i <= rounds
        assert r.rev_edges == c.T4s and c.T4 == c.T4s + g.m
        assert c.T6min <= c.T6 <= g.m


def test_exhaustive_four_vertices(orc, gen):
    """All 2^16 digraphs on 4 vertices (self-loops included) against the
    greatest self-supporting subset found by enumeration."""
    n = 4
    for code in range(1 << (n * n)):
        masks = [(code >> (n * v)) & 0xF for v in range(n)]
        adj = [[w for w in range(n) if (masks[v] >> w) & 1] for v in range(n)]
        g = gen.from_adjacency(adj)
        r = orc.peel(g)
        got = sum(1 << v for v in range(n) if r.live[v])
        assert got == greatest_by_subsets(n, masks), (code, adj)


def test_exhaustive_three_vertices_all_algorithms(orc, gen):
    n = 3
    for code in range(1 << (n * n)):
        masks = [(code >> (n * v)) & 0x7 for v in range(n)]
        adj = [[w for w in range(n) if (masks[v] >> w) & 1] for v in range(n)]
        g = gen.from_adjacency(adj)
        want = greatest_by_subsets(n, masks)
        for live in (orc.peel(g).live, orc.ac6_seq(g)[0], orc.ac3(g)[0], orc.ac3(g, False)[0]):
            assert sum(1 << v for v in range(n) if live[v]) == want


def test_duplicates_and_self_loops_special_cases(orc, gen):
    # a self-loop keeps its vertex and everything that reaches it
    g = gen.from_adjacency([[1], [2], [2], [0], []])
    r = orc.peel(g)
    assert list(r.live) == [1, 1, 1, 1, 0]
    # duplicate edges to a dying vertex: removed once, counted per edge
    g = gen.from_adjacency([[1, 1, 1], []])
    r = orc.peel(g)
    c = orc.counts(g, r)
    assert list(r.live) == [0, 0] and c.T6 == 3 and c.T4s == 3 and r.alpha == 2
    # a 2-cycle survives; a chain into it survives; a chain out of it dies
    g = gen.from_adjacency([[1], [0], [0], [4], []])
    assert list(orc.peel(g).live) == [1, 1, 1, 0, 0]
    # empty graph and edgeless graph
    g = gen.from_adjacency([])
    r = orc.peel(g)
    assert r.n_live == 0 and r.alpha == 0
    g = gen.from_adjacency([[], [], []])
    r = orc.peel(g)
    assert r.alpha == 1 and r.n_live == 0


@pytest.mark.parametrize("seed", range(4))
def test_reach_cycle_characterisation(orc, gen, seed):
    for n, m in ((1000, 900), (5000, 6000), (20000, 30000)):
        g = gen.uniform(n, m, seed=seed * 7 + 1, drop_self=bool(seed % 2))
        r = orc.peel(g)
        assert (r.live.astype(bool) == reaches_cycle(g)).all()


def test_chain_long():
    import graphgen as gen
    import oracle as orc
    n = 100000
    adj_src = np.arange(n - 1, dtype=np.int32)
    g = gen.from_edges(n, adj_src, adj_src + 1)
    r = orc.peel(g)
    assert r.alpha == n and r.n_live == 0
    assert r.level[0] == n and r.level[n - 1] == 1
    c = orc.counts(g, r)
    assert c.T6 == n - 1 and c.T3J == sum(1 + (n - v) - 1 for v in range(n - 1))


def test_config0_closed_form(orc, gen):
    """Core + tail: every core vertex keeps a core successor (8 uniform draws,
    self-loops dropped) and every tail vertex only points to higher tail ids,
    which end in sinks.  So the live set is the core exactly, T6 = n_core +
    E_tail, T4* = E_tail, T4 = m + E_tail."""
    g = gen.config0()
    n_core = g.meta["n_core"]
    assert (g.n, n_core, g.meta["n_sink"]) == (65536, 45875, 655)
    r = orc.peel(g)
    assert r.live[:n_core].all() and not r.live[n_core:].any()
    e_tail = int(g.row_off[-1] - g.row_off[n_core])
    c = orc.counts(g, r)
    assert c.T6 == n_core + e_tail
    assert c.T4s == e_tail and c.T4 == g.m + e_tail
    deg = g.degrees()
    assert c.T3J == int((deg[n_core:] + r.level[n_core:] - 1).sum()) + n_core * (r.alpha + 1)
    check_certificate(g, r.live.astype(bool), r.level)
    live6, t6, _ = orc.ac6_seq(g)
    assert t6 == c.T6


def test_rmat_chain_depth(orc, gen):
    """A planted chain of L vertices ending in a sink forces alpha >= L and
    c_i removed at step >= L - i."""
    g = gen.rmat(14, 8, seed=3, chain=3000)
    r = orc.peel(g)
    ch = g.meta["chain_ids"]
    assert r.alpha >= 3000
    assert (r.level[ch] >= 3000 - np.arange(3000)).all()
    check_certificate(g, r.live.astype(bool), r.level)
    live6, t6, _ = orc.ac6_seq(g)
    assert (live6 == r.live).all() and t6 == orc.counts(g, r).T6


def test_implicit_generator_two_implementations(orc, gen):
    """The oracle's POST against the workload definition recomputed here from
    the graphgen finalizer (two separate SplitMix64 implementations), plus the
    zero-degree fraction and Zipf mean as statistical sanity checks."""
    imp = gen.implicit(log2n=16, seed=5)
    M = (1 << 64) - 1
    for v in (0, 1, 2, 77, 4095, 65535):
        z = gen.fin64(imp.seed ^ gen.IMPLICIT_TAG_ZERO ^ (v << 8))
        if z < imp.zero_thr:
            d = 0
        else:
            u = gen.fin64(imp.seed ^ gen.IMPLICIT_TAG_DEG ^ (v << 8))
            d = 1 + int(np.sum(np.uint64(u) >= imp.table[:255]))
        assert orc.implicit_deg(imp, v) == d
        for i in range(min(d, 5)):
            w = gen.fin64((imp.seed ^ gen.IMPLICIT_TAG_NBR ^ ((v << 8) | i)) & M) & (imp.n - 1)
            assert orc.implicit_nbr(imp, v, i) == w
    ro, col = orc.implicit_csr(imp)
    deg = np.diff(ro)
    assert abs((deg == 0).mean() - 0.2) < 0.01
    # E[min(Zipf(2.1), 256)] = sum_{k<256} k p_k + 256 P(K >= 256) ~= 3.44
    assert abs(deg[deg > 0].mean() - 3.44) < 0.15
    assert deg.max() <= 256 and col.max() < imp.n


def test_batch_oracle_per_graph(orc, gen):
    b = gen.batch(12, seed=1, n_range=(100, 3000))
    live, nl, al = orc.batch_peel(b)
    for g in range(b.G):
        r = orc.peel(b.graph(g))
        v0, v1 = b.vbase[g], b.vbase[g + 1]
        assert (live[v0:v1] == r.live).all() and nl[g] == r.n_live and al[g] == r.alpha


def test_bitmap_layout(orc):
    live = np.zeros(70, np.uint8)
    live[[0, 5, 31, 32, 69]] = 1
    bm = orc.bitmap(live)
    assert bm.dtype == np.uint32 and bm.shape == (3,)
    assert bm[0] == (1 | (1 << 5) | (1 << 31)) and bm[1] == 1 and bm[2] == (1 << 5)


def test_mlp_reference_finite_differences():
    from oracle import mlp_ref
    pin_finite_differences(mlp_ref)


def pin_finite_differences(mlp_ref):
    """The FP64 reference's backward pass against central differences of its
    own forward pass (no BF16 rounding), on random features and weights."""
    rng = np.random.default_rng(7)
    p = rng.normal(0, 0.4, mlp_ref.NPARAM)
    X = rng.normal(0, 1, (24, 8))
    y = (rng.random(24) < 0.5).astype(float)
    w = (rng.random(24) < 0.8).astype(float) / 24
    loss, g = mlp_ref.loss_and_grad(p, X, y, w, bf16=False)
    eps = 1e-6
    for i in list(range(0, mlp_ref.NPARAM, 37)) + [255, 287, 1311, 1343, 1375, 1376]:
        q = p.copy()
        q[i] += eps
        lp, _ = mlp_ref.loss_and_grad(q, X, y, w, bf16=False)
        q[i] -= 2 * eps
        lm, _ = mlp_ref.loss_and_grad(q, X, y, w, bf16=False)
        assert abs((lp - lm) / (2 * eps) - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), i


def test_mlp_reference_bf16_rounding():
    from oracle import mlp_ref
    pin_bf16_rounding(mlp_ref)


def pin_bf16_rounding(mlp_ref):
    x = np.array([1.0, 1.00390625, 1.005, 3.14159265, -2.71828, 1e-3, 0.0])
    r = mlp_ref.bf16_round(x)
    # BF16 keeps 8 significant bits: 1 + 2^-8 is exactly halfway and rounds to even
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125 and r[3] == 3.140625
    assert r[4] == -2.71875 and r[6] == 0.0


def test_mlp_logits_hand_computed():
    from oracle import mlp_ref
    pin_logits_hand_computed(mlp_ref)


def pin_logits_hand_computed(mlp_ref):
    """A network with one path 8 -> 1 -> 1 -> 1 computes 6 relu(x0) - 1 by
    hand: W1[0][0] = 1, W2[0][0] = 2, w3[0] = 3, b3 = -1, all else 0."""
    p = np.zeros(mlp_ref.NPARAM)
    p[0] = 1.0            # W1[0][0]
    p[288] = 2.0          # W2[0][0]
    p[1344] = 3.0         # w3[0]
    p[1376] = -1.0        # b3
    X = np.zeros((3, 8))
    X[:, 0] = [0.5, -1.0, 2.0]
    X[:, 3] = [9.0, 9.0, 9.0]     # other inputs have zero weight
    np.testing.assert_allclose(mlp_ref.logits(p, X, bf16=False), [2.0, -1.0, 11.0])
    # the loss of loss_and_grad is the BCE of these logits
    y = np.array([1.0, 0.0, 1.0])
    w = np.ones(3)
    s = np.array([2.0, -1.0, 11.0])
    want = np.sum(np.log1p(np.exp(-s)) * y + np.log1p(np.exp(s)) * (1 - y))
    loss, _ = mlp_ref.loss_and_grad(p, X, y, w, bf16=False)
    assert abs(loss - want) < 1e-12


def pin_features_hand_computed(mlp_ref, fin64):
    """Feature rows of a 3-vertex graph worked out by hand: 0 -> [1, 2],
    1 -> [2], 2 -> [0], so out-degrees (2, 1, 1) and in-degrees (1, 1, 2).
    Edge u -> w at list position i has log1p(outdeg u), log1p(indeg u),
    log1p(outdeg w), log1p(indeg w), log1p(outdeg u) - log1p(outdeg w) and
    +-1 for bits 0, 1, 2 of SplitMix64(i).  The finalizer maps 0 to 0, so
    position 0 gives -1, -1, -1; position 1 takes its bits from ``fin64``
    (pinned on the published vector)."""
    row_off = np.array([0, 2, 3, 4])
    col = np.array([1, 2, 2, 0])
    indeg = np.array([1, 1, 2])
    X, src, dst = mlp_ref.features(row_off, col, indeg, [0, 1, 2, 3])
    assert list(src) == [0, 0, 1, 2] and list(dst) == [1, 2, 2, 0]
    l2, l3 = np.log(2.0), np.log(3.0)
    h = fin64(1)
    b = [1.0 if (h >> k) & 1 else -1.0 for k in range(3)]
    want = np.array([
        [l3, l2, l2, l2, l3 - l2, -1, -1, -1],     # 0 -> 1, position 0
        [l3, l2, l2, l3, l3 - l2] + b,             # 0 -> 2, position 1
        [l2, l2, l2, l3, 0.0, -1, -1, -1],         # 1 -> 2, position 0
        [l2, l3, l3, l2, l2 - l3, -1, -1, -1],     # 2 -> 0, position 0
    ])
    # the features are computed in FP32, as on the GPU
    np.testing.assert_allclose(X, want, rtol=2e-7, atol=2e-7)


def pin_adam_first_step(mlp_ref):
    """At step 1 from zero moments, m_hat = g and v_hat = g^2, so every
    parameter moves by exactly lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 0.0, 1e-9, 3e4])
    p0 = np.array([1.0, -1.0, 0.25, 0.0, 2.0])
    lr, eps = 0.1, 1e-8
    p, m, v = mlp_ref.adam_step(p0, np.zeros(5), np.zeros(5), g, lr, 0.9, 0.999, eps, 1)
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def pin_adam_two_steps_by_hand(mlp_ref):
    """Gradients +1 then -1 with beta1 = 0.9, beta2 = 0.999: after step 1,
    m = 0.1, v = 0.001 and the parameter moves down by lr / (1 + eps).  Step 2
    gives m = 0.09 - 0.1 = -0.01, v = 0.000999 + 0.001 = 0.001999, so
    m_hat = -0.01 / 0.19, v_hat = 0.001999 / 0.001999 = 1, and the parameter
    moves up by lr * (0.01 / 0.19) / (1 + eps)."""
    lr, eps = 0.05, 1e-8
    p, m, v = mlp_ref.adam_step([0.0], [0.0], [0.0], [1.0], lr, 0.9, 0.999, eps, 1)
    assert abs(p[0] + lr / (1 + eps)) < 1e-15 and abs(m[0] - 0.1) < 1e-15
    p, m, v = mlp_ref.adam_step(p, m, v, [-1.0], lr, 0.9, 0.999, eps, 2)
    assert abs(m[0] + 0.01) < 1e-15 and abs(v[0] - 0.001999) < 1e-15
    want = -lr / (1 + eps) + lr * (0.01 / 0.19) / (1 + eps)
    assert abs(p[0] - want) < 1e-14


def test_mlp_features_hand_computed(orc):
    from oracle import mlp_ref
    pin_features_hand_computed(mlp_ref, orc.fin64)


def test_mlp_adam_first_step():
    from oracle import mlp_ref
    pin_adam_first_step(mlp_ref)


def test_mlp_adam_two_steps_by_hand():
    from oracle import mlp_ref
    pin_adam_two_steps_by_hand(mlp_ref)


# --------------------------------------------------------- two-sided trimming
def greatest_two_sided_by_subsets(n, adj_masks):
    """Union of every subset S in which each vertex has a successor and a
    predecessor in S (the in-degree improvement of Section 4.1); such sets are
    closed under union, so this is the greatest one."""
    pred = [0] * n
    for u in range(n):
        for v in range(n):
            if (adj_masks[u] >> v) & 1:
                pred[v] |= 1 << u
    best = 0
    for S in range(1 << n):
        if all(not (S >> v) & 1 or ((adj_masks[v] & S) and (pred[v] & S)) for v in range(n)):
            best |= S
    return best


def stepwise_peel2(adj):
    """Peeling by whole steps: each step removes, all at once, every remaining
    vertex without a remaining successor or without a remaining predecessor."""
    n = len(adj)
    pred = [[] for _ in range(n)]
    for u in range(n):
        for w in adj[u]:
            pred[w].append(u)
    alive = [True] * n
    level = [0] * n
    step = 0
    while True:
        step += 1
        rm = [v for v in range(n) if alive[v] and
              (not any(alive[w] for w in adj[v]) or not any(alive[u] for u in pred[v]))]
        if not rm:
            break
        for v in rm:
            alive[v] = False
            level[v] = step
    return alive, level


def test_two_sided_hand_examples(orc, gen):
    # 0 -> 1 <-> 2 -> 3: 0 has no predecessor, 3 no successor; the 2-cycle stays
    g = gen.from_adjacency([[1], [2], [1, 3], []])
    r = orc.peel2(g)
    assert list(r.live) == [0, 1, 1, 0] and list(r.level) == [1, 0, 0, 1] and r.alpha == 1
    rro, rcol = gen.transpose(g)
    assert list(rcol[rro[1]:rro[2]]) == [0, 2]
    c = orc.counts2(g, rro, rcol, r.live)
    # live 1: successor 2 first (1 check); predecessors 0 (dead), 2 (2 checks)
    # live 2: successor 1 first, predecessor 1 first: 2 checks
    assert (c.T6live, c.dead_lo, c.dead_hi, c.T4two, c.n_live) == (5, 0, 0, 2, 2)
    assert r.rev_edges == 2
    # one-sided trimming keeps vertex 0 (it reaches the cycle)
    assert list(orc.peel(g).live) == [1, 1, 1, 0]
    # 0 -> 1 -> 2 with a self-loop on 2: removal runs forward along the path
    g = gen.from_adjacency([[1], [2], [2]])
    r = orc.peel2(g)
    assert list(r.live) == [0, 0, 1] and list(r.level) == [1, 2, 0] and r.alpha == 2
    rro, rcol = gen.transpose(g)
    c = orc.counts2(g, rro, rcol, r.live)
    # live 2: own self-loop found first as successor; predecessors 1 (dead), 2
    assert (c.T6live, c.dead_lo, c.dead_hi, c.T4two) == (3, 1, 2, 3)
    assert r.rev_edges == 3
    # a directed cycle keeps everything, a path loses everything
    assert orc.peel2(gen.from_adjacency([[1], [2], [0]])).n_live == 3
    r = orc.peel2(gen.from_adjacency([[1], [2], [3], []]))
    assert r.n_live == 0 and list(r.level) == [1, 2, 2, 1] and r.alpha == 2
    # empty graph
    r = orc.peel2(gen.from_adjacency([]))
    assert r.n_live == 0 and r.alpha == 0


def test_two_sided_exhaustive_three_and_four(orc, gen):
    for n in (3, 4):
        full = (1 << n) - 1
        for code in range(1 << (n * n)):
            masks = [(code >> (n * v)) & full for v in range(n)]
            adj = [[w for w in range(n) if (masks[v] >> w) & 1] for v in range(n)]
            g = gen.from_adjacency(adj)
            r = orc.peel2(g)
            got = sum(1 << v for v in range(n) if r.live[v])
            assert got == greatest_two_sided_by_subsets(n, masks), (code, adj)


@pytest.mark.parametrize("seed", range(3))
def test_two_sided_levels_by_whole_steps(orc, gen, seed):
    rng = np.random.default_rng(seed)
    for n, m in ((12, 14), (40, 50), (200, 260)):
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        adj = [[] for _ in range(n)]
        for s, d in zip(src, dst):
            adj[int(s)].append(int(d))
        g = gen.from_adjacency(adj)
        r = orc.peel2(g)
        alive, level = stepwise_peel2(adj)
        assert list(r.live.astype(bool)) == alive
        assert list(r.level) == level
        assert r.alpha == max(level + [0])


@pytest.mark.parametrize("seed", range(3))
def test_two_sided_reach_and_reached_from_cycle(orc, gen, seed):
    """v survives two-sided trimming iff it reaches a cycle and a cycle reaches
    it: the path from one cycle through v to the other, with both cycles, is a
    set in which every vertex has both neighbours; conversely, following
    predecessors (successors) inside a finite such set must close a cycle."""
    for n, m in ((1000, 1100), (5000, 6500), (20000, 26000)):
        g = gen.uniform(n, m, seed=seed * 5 + 3, drop_self=bool(seed % 2))
        rro, rcol = gen.transpose(g)
        gt = gen.CSR(g.n, rro, rcol)
        r = orc.peel2(g)
        fwd = reaches_cycle(g)
        bwd = reaches_cycle(gt)
        assert (r.live.astype(bool) == (fwd & bwd)).all()
        # and equals one-sided trimming of G intersected with that of G^T
        assert (r.live == (orc.peel(g).live & orc.peel(gt).live)).all()
        c = orc.counts2(g, rro, rcol, r.live)
        deg = np.diff(g.row_off)
        indeg = np.diff(rro)
        dead = r.live == 0
        assert c.T4two == r.rev_edges == int((deg + indeg)[dead].sum())
        both = dead & (deg > 0) & (indeg > 0)
        assert c.dead_lo == int(np.minimum(deg, indeg)[both].sum())
        assert c.n_live == r.n_live


def test_two_sided_ac3_hand_example(orc, gen):
    """Source -> cycle -> sink (0->1, 1->2, 2->1, 2->3).  Round 1: vertex 0
    checks 1 successor and has no predecessor (1 check, removed); 1 and 2
    check one successor and one predecessor each (4); 3 has no successor (0,
    removed).  Round 2: 1 rechecks its successor, finds its predecessor 0
    removed and moves on to 2 (3 checks); 2 rechecks both (2).  Nothing is
    removed in round 2: 10 checks in 2 rounds."""
    g = gen.from_adjacency([[1], [2], [1, 3], []])
    rro, rcol = gen.transpose(g)
    a = orc.ac3_jacobi2(g, rro, rcol)
    assert (a.edges, a.rounds, a.n_live) == (10, 2, 2)
    assert list(a.live) == [0, 1, 1, 0] and list(a.level) == [1, 0, 0, 1]
    assert orc.counts3two(g, rro, rcol, orc.peel2(g)) == (10, 2)
    # a path peels from both ends: alpha = 51 for 101 vertices
    L = 101
    g = gen.from_edges(L, np.arange(L - 1, dtype=np.int32), np.arange(1, L, dtype=np.int32))
    rro, rcol = gen.transpose(g)
    a = orc.ac3_jacobi2(g, rro, rcol)
    assert a.n_live == 0 and a.rounds == 52
    assert (a.edges, a.rounds) == orc.counts3two(g, rro, rcol, orc.peel2(g))


@pytest.mark.parametrize("seed", range(3))
def test_two_sided_ac3_rounds_match_peeling(orc, gen, seed):
    """The literal two-sided AC-3 rounds (statuses of each round's start)
    remove exactly the vertices of two-sided peeling, each in the round equal
    to its peeling step (or_peel2, an independent counter computation), take
    alpha + 1 rounds, and check as many edges as the closed form from the
    levels says."""
    rng = np.random.default_rng(900 + seed)
    for t in range(100):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 3 * n + 1))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        if t % 2:
            keep = src != dst
            src, dst = src[keep], dst[keep]
        g = gen.from_edges(n, src, dst)
        rro, rcol = gen.transpose(g)
        a = orc.ac3_jacobi2(g, rro, rcol)
        r = orc.peel2(g)
        assert np.array_equal(a.live, r.live) and np.array_equal(a.level, r.level)
        assert a.rounds == r.alpha + 1
        assert (a.edges, a.rounds) == orc.counts3two(g, rro, rcol, r)
    g = gen.rmat(12, 4, seed=seed, chain=300)
    rro, rcol = gen.transpose(g)
    a = orc.ac3_jacobi2(g, rro, rcol)
    r = orc.peel2(g)
    assert np.array_equal(a.level, r.level)
    assert (a.edges, a.rounds) == orc.counts3two(g, rro, rcol, r)


# ------------------------------------------------- vertices removed up front
def literal_runs_with_preset(adj, preset):
    """The three algorithms run step by step with the preset vertices DEAD from
    the start (vertex sampling, Section 9), counting every check:
    sequential AC-6 (Section 6.1: DoPost from a cursor, supporters handed back
    when their support dies), Jacobi AC-3 with cursor (Section 4.1 and the
    edge_index of Section 8), and AC-4 with counters from offsets (Section 5.1,
    AC4Trim* of Section 9.3; every removed vertex, preset ones included, walks
    its predecessors).  Returns (live, t6, t3, rounds, t4)."""
    n = len(adj)
    pred = [[] for _ in range(n)]
    for u in range(n):
        for w in adj[u]:
            pred[w].append(u)
    # AC-6
    live = [not preset[v] for v in range(n)]
    cur = [0] * n
    S = [[] for _ in range(n)]
    t6 = 0

    def dopost(v, Q):
        nonlocal t6
        while cur[v] < len(adj[v]):
            w = adj[v][cur[v]]
            cur[v] += 1
            t6 += 1
            if live[w]:
                S[w].append(v)
                return
        live[v] = False
        Q.append(v)

    for v in range(n):
        if not live[v]:
            continue
        Q = []
        dopost(v, Q)
        while Q:
            w = Q.pop()
            members, S[w] = S[w], []
            for u in members:
                dopost(u, Q)
    live6 = live
    # Jacobi AC-3
    INF = 1 << 60
    dround = [0 if preset[v] else INF for v in range(n)]
    cur = [0] * n
    t3 = rounds = 0
    while True:
        rounds += 1
        changed = False
        for v in range(n):
            if dround[v] != INF:
                continue
            while cur[v] < len(adj[v]):
                t3 += 1
                if dround[adj[v][cur[v]]] >= rounds:
                    break
                cur[v] += 1
            else:
                dround[v] = rounds
                changed = True
        if not changed:
            break
    # AC-4*
    cnt = [len(adj[v]) for v in range(n)]
    dead = [bool(preset[v]) for v in range(n)]
    Q = [v for v in range(n) if preset[v]] + [v for v in range(n) if not preset[v] and cnt[v] == 0]
    for v in Q:
        dead[v] = True
    t4 = 0
    while Q:
        w = Q.pop()
        for u in pred[w]:
            t4 += 1
            cnt[u] -= 1
            if cnt[u] == 0 and not dead[u]:
                dead[u] = True
                Q.append(u)
    assert [dround[v] == INF for v in range(n)] == live6 == [not d for d in dead]
    return live6, t6, t3, rounds, t4


def test_preset_exhaustive_three_vertices(orc, gen):
    n = 3
    for code in range(1 << (n * n)):
        masks = [(code >> (n * v)) & 0x7 for v in range(n)]
        adj = [[w for w in range(n) if (masks[v] >> w) & 1] for v in range(n)]
        g = gen.from_adjacency(adj)
        for pm in range(1 << n):
            preset = np.array([(pm >> v) & 1 for v in range(n)], np.uint8)
            keep = [m & ~pm for m in masks]
            want = greatest_by_subsets(n, [keep[v] if not (pm >> v) & 1 else 0
                                           for v in range(n)]) & ~pm
            r = orc.peel(g, preset=preset)
            assert sum(1 << v for v in range(n) if r.live[v]) == want, (code, pm)
            c = orc.counts(g, r, preset=preset)
            live, t6, t3, rounds, t4 = literal_runs_with_preset(adj, preset)
            assert list(r.live.astype(bool)) == live
            assert (c.T6, c.T3J, c.rounds3, c.T4s) == (t6, t3, rounds, t4), (code, pm)


@pytest.mark.parametrize("seed", range(3))
def test_preset_equals_induced_subgraph(orc, gen, seed):
    """Removing the preset vertices first is trimming the subgraph they leave:
    same live set, same peeling steps."""
    rng = np.random.default_rng(seed)
    for n, m, ratio in ((500, 700, 0.3), (4000, 5200, 0.5), (20000, 30000, 0.9)):
        g = gen.uniform(n, m, seed=seed * 11 + n)
        preset = (rng.random(n) >= ratio).astype(np.uint8)
        keep = np.flatnonzero(preset == 0)
        new_id = np.full(n, -1, np.int64)
        new_id[keep] = np.arange(keep.size)
        adj = []
        for v in keep:
            succ = g.col[g.row_off[v]:g.row_off[v + 1]]
            adj.append([int(new_id[w]) for w in succ if new_id[w] >= 0])
        sub = orc.peel(gen.from_adjacency(adj))
        r = orc.peel(g, preset=preset)
        assert (r.live[keep] == sub.live).all() and not r.live[preset == 1].any()
        assert (r.level[keep] == sub.level).all() and (r.level[preset == 1] == 0).all()
        assert r.alpha == sub.alpha and r.n_dead == sub.n_dead


@pytest.mark.parametrize("seed", range(3))
def test_preset_totals_by_literal_runs(orc, gen, seed):
    rng = np.random.default_rng(100 + seed)
    for n, m in ((60, 80), (300, 420), (2000, 2600)):
        g = gen.uniform(n, m, seed=seed * 13 + n)
        adj = [list(g.col[g.row_off[v]:g.row_off[v + 1]]) for v in range(n)]
        for ratio in (0.1, 0.5, 1.0):
            preset = (rng.random(n) >= ratio).astype(np.uint8)
            r = orc.peel(g, preset=preset)
            c = orc.counts(g, r, preset=preset)
            live, t6, t3, rounds, t4 = literal_runs_with_preset(adj, preset)
            assert list(r.live.astype(bool)) == live
            assert (c.T6, c.T3J, c.rounds3, c.T4s) == (t6, t3, rounds, t4), (n, ratio)
            assert r.rev_edges == c.T4s


# ------------------------------------------------- strongly connected components
def closure_scc(adj):
    """SCC labels by brute force: reachability by repeated squaring of the
    boolean adjacency (Warshall), then u ~ v iff each reaches the other;
    label = smallest id of the class."""
    n = len(adj)
    R = np.eye(n, dtype=bool)
    for u in range(n):
        for w in adj[u]:
            R[u, w] = True
    for k in range(n):
        R = R | (R[:, k:k + 1] & R[k:k + 1, :])
    both = R & R.T
    return np.array([int(np.flatnonzero(both[v])[0]) for v in range(n)], np.int64)


def test_scc_reference_against_closure(gen):
    from oracle.scc_ref import scc_labels
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(1, 12))
        m = int(rng.integers(0, 3 * n))
        adj = [[] for _ in range(n)]
        for _ in range(m):
            adj[int(rng.integers(n))].append(int(rng.integers(n)))
        g = gen.from_adjacency(adj)
        assert (scc_labels(g) == closure_scc(adj)).all(), adj


def test_scc_reference_closed_forms(gen):
    from oracle.scc_ref import scc_labels, summary, canonical
    # a directed cycle is one component; a path is n singletons
    n = 1000
    g = gen.from_edges(n, np.arange(n, dtype=np.int32), (np.arange(n, dtype=np.int32) + 1) % n)
    assert (scc_labels(g) == 0).all()
    g = gen.from_edges(n, np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32))
    assert (scc_labels(g) == np.arange(n)).all()
    # two 3-cycles joined by one edge stay two components
    g = gen.from_adjacency([[1], [2], [0, 3], [4], [5], [3]])
    assert list(scc_labels(g)) == [0, 0, 0, 3, 3, 3]
    assert summary(scc_labels(g)) == {"n_scc": 2, "n_single": 0, "largest": 3}
    assert list(canonical([7, 3, 7, 3, 9])) == [0, 1, 0, 1, 4]


@pytest.mark.parametrize("seed", range(2))
def test_scc_reference_versus_trimming(orc, gen, seed):
    """Vertices that two-sided trimming removes lie on no cycle, so each is a
    component of its own; a vertex with a self-loop or in a component of two
    or more vertices survives it."""
    from oracle.scc_ref import scc_labels
    g = gen.uniform(20000, 26000, seed=seed + 40)
    lab = scc_labels(g)
    size = np.bincount(lab, minlength=g.n)[lab]
    loop = np.zeros(g.n, bool)
    src = np.repeat(np.arange(g.n), np.diff(g.row_off))
    loop[src[src == g.col]] = True
    r2 = orc.peel2(g)
    on_cycle = (size > 1) | loop
    assert not (r2.live.astype(bool) == 0)[on_cycle].any()
    assert (lab[r2.live == 0] == np.flatnonzero(r2.live == 0)).all()


def test_size2_pairs_are_components(gen):
    """The pairs the size-2 check reports are exactly the strongly connected
    components of two vertices, neither with a self-loop, that no other
    remaining vertex enters or that leave to no other remaining vertex."""
    from oracle.scc_ref import scc_labels, size2_pairs
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(2, 14))
        m = int(rng.integers(1, 3 * n))
        adj = [[] for _ in range(n)]
        for _ in range(m):
            adj[int(rng.integers(n))].append(int(rng.integers(n)))
        for _ in range(int(rng.integers(0, 3))):   # plant some 2-cycles
            a, b = rng.choice(n, 2, replace=False)
            adj[int(a)].append(int(b))
            adj[int(b)].append(int(a))
        g = gen.from_adjacency(adj)
        preset = (rng.random(n) < 0.2).astype(np.uint8)
        alive = preset == 0
        partner = size2_pairs(g, preset)
        # the components of the remaining vertices
        keep = np.flatnonzero(alive)
        idx = np.full(n, -1)
        idx[keep] = np.arange(keep.size)
        sub = gen.from_adjacency([[int(idx[w]) for w in adj[v] if alive[w]] for v in keep])
        lab = scc_labels(sub)
        want = np.full(n, -1)
        for comp in np.unique(lab):
            mem = keep[lab == comp]
            if mem.size != 2:
                continue
            a, b = int(mem[0]), int(mem[1])
            if a in adj[a] or b in adj[b]:
                continue
            enters = any(alive[u] and u not in (a, b) and w in (a, b)
                         for u in range(n) for w in adj[u])
            leaves = any(w not in (a, b) and alive[w] for u in (a, b) for w in adj[u])
            if not enters or not leaves:
                want[a], want[b] = b, a
        assert (partner == want).all(), (adj, preset, partner, want)


def test_size2_pairs_hand_example(gen):
    from oracle.scc_ref import size2_pairs
    # 0 <-> 1 fed by 2 (not a source pair, but a sink pair: 0, 1 reach nothing
    # else); 3 <-> 4 with 3 -> 5: a source pair (nothing enters); 6 <-> 7 with
    # 8 -> 6 and 7 -> 8: neither
    g = gen.from_adjacency([[1], [0], [0], [4, 5], [3], [], [7], [6, 8], [6]])
    assert list(size2_pairs(g)) == [1, 0, -1, 4, 3, -1, -1, -1, -1]
    # removing 5 from the start changes nothing for 3 <-> 4; removing 2 too
    pre = np.zeros(9, np.uint8)
    pre[[2, 5]] = 1
    assert list(size2_pairs(g, pre)) == [1, 0, -1, 4, 3, -1, -1, -1, -1]
    # a self-loop on 0 breaks the pair
    g = gen.from_adjacency([[0, 1], [0]])
    assert list(size2_pairs(g)) == [-1, -1]
