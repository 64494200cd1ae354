"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

The live bitmap must be bit-identical; the traversed-edge totals must equal
the oracle's closed forms exactly (AC-6: T6, AC-4: T4*, AC-3: T3J and
alpha + 1 rounds).  Per-worker counts are schedule dependent; only their sum
is compared.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import check_all, expected, run_csr, say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def test_worked_example(ctx):
    g = gg.from_adjacency([[3, 2], [], [4, 3], [4], []])
    r, c = check_all(ctx, g, name="worked example")
    assert (c.T6, c.T4s, c.T3J) == (5, 5, 11)


@pytest.mark.parametrize("adj,name", [
    ([], "empty"),
    ([[], [], []], "edgeless"),
    ([[0]], "self-loop"),
    ([[1], [0]], "2-cycle"),
    ([[1], [2], [2], [0], []], "loop+tail"),
    ([[1, 1, 1], []], "duplicates"),
    ([[1], [0], [0], [4], []], "cycle-in-out"),
])
def test_special_cases(ctx, adj, name):
    check_all(ctx, gg.from_adjacency(adj), name=name)


@pytest.mark.parametrize("seed", range(8))
def test_random_graphs(ctx, seed):
    rng = np.random.default_rng(1000 + seed)
    for n, dens in ((97, 0.8), (1000, 1.2), (5000, 1.0), (20000, 2.5), (70001, 1.05)):
        g = gg.uniform(n, int(dens * n), seed=seed * 31 + n, drop_self=bool(rng.integers(2)))
        check_all(ctx, g, name=f"uniform n={n} seed={seed}")


def test_config0(ctx):
    g = gg.config0()
    r, c = check_all(ctx, g, name="core+tail n=65536")
    assert r.n_live == g.meta["n_core"]


def test_star_contention(ctx):
    """One hub with 10^6 supporters that dies (its only successor is a sink),
    so every supporter is handed back at once; and the same hub kept alive by
    a self-loop, so 10^6 vertices register on one list."""
    N = 1000000
    src = np.arange(1, N + 1, dtype=np.int32)
    dst = np.zeros(N, np.int32)
    g = gg.from_edges(N + 2, np.r_[src, 0], np.r_[dst, N + 1])
    check_all(ctx, g, name="dying hub")
    g = gg.from_edges(N + 2, np.r_[src, 0], np.r_[dst, 0])
    check_all(ctx, g, name="live hub")
    # every vertex points at the hub twice, then at itself: duplicates to a dying hub
    src2 = np.repeat(np.arange(1, N + 1, dtype=np.int32), 3)
    dst2 = np.stack([np.zeros(N, np.int32), np.zeros(N, np.int32),
                     np.arange(1, N + 1, dtype=np.int32)], 1).ravel()
    g = gg.from_edges(N + 2, np.r_[src2, 0], np.r_[dst2, N + 1])
    check_all(ctx, g, name="hub duplicates", algos=(6, 4))


def test_long_chain(ctx):
    n = 100000
    src = np.arange(n - 1, dtype=np.int32)
    g = gg.from_edges(n, src, src + 1)
    check_all(ctx, g, name="chain 1e5")


def test_complete_dag(ctx):
    n = 400
    i, j = np.triu_indices(n, 1)
    g = gg.from_edges(n, i.astype(np.int32), j.astype(np.int32))
    r, _ = check_all(ctx, g, name="complete DAG")
    assert r.alpha == n


def test_rmat_with_chain(ctx):
    g = gg.rmat(16, 16, seed=7, chain=3000)
    check_all(ctx, g, name="rmat16+chain")


def test_rmat_scale18(ctx):
    check_all(ctx, gg.rmat(18, 16, seed=2), algos=(6, 4), name="rmat18")


def test_schedule_invariance(ctx):
    """Block size, chunk size and worker count change the schedule, never the
    live set or the traversed-edge total."""
    import paper_2107_12720_amd as T
    g = gg.rmat(17, 8, seed=11, chain=2000)
    r, c, bm = expected(g)
    dev6 = upload(g)
    dev4 = upload(g, with_reverse=True)
    for block, chunk, workers in ((64, 64, 1), (256, 4096, 7), (1024, 65536, 0), (128, 1, 3),
                                  (512, 300, 1024)):
        opts = T.make_opts(block=block, chunk=chunk, workers=workers)
        say(f"  schedule block={block} chunk={chunk} workers={workers}")
        for a, want, dev in ((6, c.T6, dev6), (4, c.T4s, dev4)):
            got, edges, st = run_csr(ctx, g, a, opts=opts, dev=dev)
            assert np.array_equal(got, bm) and edges == want


def reverse_star(n):
    """The hub points at n vertices that are all sinks but one, and that one
    points back: the hub and its live successor survive, the hub's cursor has
    to pass n - 1 dead targets."""
    src = np.zeros(n, np.int32)
    dst = np.arange(1, n + 1, dtype=np.int32)
    return gg.from_edges(n + 1, np.r_[src, n], np.r_[dst, 0])


def test_reverse_star(ctx):
    check_all(ctx, reverse_star(300000), name="reverse star")


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_schedule_perturbation(ctx, schedule):
    """Reversed sweep chunks (1), pauses inside the race windows (2), and both:
    fifty repeats each on a dying hub with duplicate edges, a reverse star and
    R-MAT with a chain; output never changes."""
    import paper_2107_12720_amd as T
    N = 20000
    src2 = np.repeat(np.arange(1, N + 1, dtype=np.int32), 3)
    dst2 = np.stack([np.zeros(N, np.int32), np.zeros(N, np.int32),
                     np.arange(1, N + 1, dtype=np.int32)], 1).ravel()
    graphs = [("hub duplicates", gg.from_edges(N + 2, np.r_[src2, 0], np.r_[dst2, N + 1])),
              ("reverse star", reverse_star(20000)),
              ("rmat14+chain", gg.rmat(14, 16, seed=9, chain=800))]
    for name, g in graphs:
        r, c, bm = expected(g)
        dev6 = upload(g)
        dev4 = upload(g, with_reverse=True)
        say(f"  schedule={schedule} {name}: 50 repeats of AC-6 and AC-4")
        for k in range(50):
            opts = T.make_opts(schedule=schedule, chunk=(64, 4096)[k % 2], workers=(0, 37)[k % 2])
            for a, want, dev in ((6, c.T6, dev6), (4, c.T4s, dev4)):
                got, edges, st = run_csr(ctx, g, a, opts=opts, dev=dev)
                assert np.array_equal(got, bm) and edges == want, (name, a, k)


def test_repeat_stability(ctx):
    """Fifty repeats (Section 9.5 repeats every run 50 times): identical output."""
    g = gg.rmat(16, 16, seed=5, chain=500)
    r, c, bm = expected(g)
    dev = upload(g)
    for k in range(50):
        got, edges, st = run_csr(ctx, g, 6, dev=dev)
        assert np.array_equal(got, bm) and edges == c.T6, k


def test_config1_full(ctx):
    """R-MAT scale 22, edge factor 16, planted 100,000-vertex chain: AC-6 and
    AC-4 against the oracle at full size."""
    g = gg.config1()
    say(f"  config1 n={g.n} m={g.m}")
    check_all(ctx, g, algos=(6, 4, 3), name="rmat22+chain")


def test_errors(ctx):
    import torch
    import paper_2107_12720_amd as T
    g = gg.uniform(100, 300, seed=1)
    ro, col, _, _ = upload(g)
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr(4, g.n, ro, col)                     # AC-4 without G^T
    assert e.value.code == -1
    bad = col.clone()
    bad[5] = 1000                                         # target out of range
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr(6, g.n, ro, bad, opts=T.make_opts(validate=True))
    assert e.value.code == -5
    bad_ro = ro.clone()
    bad_ro[10] = bad_ro[11] + 1                           # non-monotone offsets
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr(6, g.n, bad_ro, col, opts=T.make_opts(validate=True))
    assert e.value.code == -5
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr(6, g.n, ro, col, opts=T.make_opts(block=100))
    assert e.value.code == -1
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr(6, g.n, ro, col, opts=T.make_opts(schedule=4))   # unknown flag
    assert e.value.code == -1
    table = torch.zeros(256, dtype=torch.int64, device="cuda")
    with pytest.raises(T.TrimError) as e:
        ctx.trim_implicit(4, 10, 0, 0, table)             # AC-4 has no on-the-fly form
    assert e.value.code == -4
    # a valid graph still works after the failures
    check_all(ctx, g, algos=(6,), name="after errors")
