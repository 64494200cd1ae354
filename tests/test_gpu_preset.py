"""GPU parity of trimming with vertices removed before it starts (the vertex
sampling of Section 9: unsampled vertices are set to DEAD) against the oracle.

The live bitmap must equal oracle.peel(g, preset) bit for bit, and the
traversed-edge totals its closed forms exactly: AC-6 T6 and AC-4 T4* as
defined for preset runs, AC-3 T3J with alpha + 1 rounds.
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


def run_preset(ctx, g, algo, bm_preset, opts=None, dev=None):
    import torch
    import paper_2107_12720_amd as T
    ro, col, rro, rc = dev or upload(g, with_reverse=(algo == 4))
    pd = T.to_device(bm_preset.view(np.int32)) if g.n else None
    res = ctx.trim_csr_preset(algo, g.n, ro, col if g.m else None, pd, rro,
                              rc if g.m else None, opts=opts)
    torch.cuda.synchronize()
    return (res.bitmap_numpy()[: (g.n + 31) // 32], int(res.worker_edges.sum().item()),
            res.stats_dict())


def check_preset(ctx, g, preset, bm_preset, algos=(6, 4, 3), opts=None, name=""):
    r = oracle.peel(g, preset=preset)
    c = oracle.counts(g, r, preset=preset)
    want_bm = oracle.bitmap(r.live)
    want = {6: c.T6, 4: c.T4s, 3: c.T3J}
    devs = {False: upload(g), True: upload(g, with_reverse=True)}
    for a in algos:
        say(f"  [{name}] preset AC-{a} n={g.n} m={g.m} removed first={int(preset.sum())}")
        got, edges, st = run_preset(ctx, g, a, bm_preset, opts=opts, dev=devs[a == 4])
        assert np.array_equal(got, want_bm), f"AC-{a} bitmap differs on {name}"
        assert edges == want[a] == st["edges_total"], (a, edges, want[a], st)
        assert st["n_live"] == r.n_live and st["n_dead"] == g.n - r.n_live, st
        if a == 3:
            assert st["rounds"] == c.rounds3, (st, c)
    return r, c


@pytest.mark.parametrize("seed", range(4))
def test_random_graphs(ctx, seed):
    for n, dens in ((97, 1.5), (5000, 2.0), (70001, 1.6)):
        g = gg.uniform(n, int(dens * n), seed=seed * 17 + n)
        for ratio in (0.1, 0.5, 0.9):
            preset, bm = gg.sample_vertices(n, ratio, seed=seed * 3 + n)
            check_preset(ctx, g, preset, bm, name=f"uniform n={n} ratio={ratio}")


def test_edge_cases(ctx):
    g = gg.from_adjacency([[1], [2], [0], [0], [3]])
    # nothing preset: the plain result
    preset, bm = gg.sample_vertices(g.n, 1.0)
    assert preset.sum() == 0
    check_preset(ctx, g, preset, bm, name="none preset")
    # everything preset
    preset, bm = gg.sample_vertices(g.n, 0.0)
    r, c = check_preset(ctx, g, preset, bm, name="all preset")
    assert r.n_live == 0 and c.T6 == 0 and c.rounds3 == 1
    # one vertex of the cycle preset: everything dies
    preset = np.array([0, 1, 0, 0, 0], np.uint8)
    bm = np.array([0b10], np.uint32)
    r, c = check_preset(ctx, g, preset, bm, name="cycle cut")
    assert r.n_live == 0
    # bits past n in the last word are ignored
    bm = np.array([0b10 | (0xFFFF << 5)], np.uint32)
    check_preset(ctx, g, preset, bm, name="bits past n")
    # empty graph
    g0 = gg.from_adjacency([])
    check_preset(ctx, g0, np.zeros(0, np.uint8), np.zeros(1, np.uint32), name="empty")


def test_rmat_chain_cut(ctx):
    """Presetting one vertex in the middle of the planted chain kills its
    upstream half in one go of peeling steps; AC-6 and AC-4."""
    g = gg.rmat(16, 16, seed=7, chain=3000)
    chain = g.meta["chain_ids"]
    preset = np.zeros(g.n, np.uint8)
    preset[chain[1500]] = 1
    words = (g.n + 31) // 32
    bits = np.zeros(words * 32, np.uint8)
    bits[:g.n] = preset
    bm = np.packbits(bits, bitorder="little").view(np.uint32).copy()
    check_preset(ctx, g, preset, bm, name="rmat16 chain cut")


def test_config0_sampled(ctx):
    g = gg.config0()
    for ratio in (0.3, 0.7):
        preset, bm = gg.sample_vertices(g.n, ratio, seed=5)
        check_preset(ctx, g, preset, bm, name=f"core+tail ratio={ratio}")


def test_schedules(ctx):
    import paper_2107_12720_amd as T
    g = gg.rmat(15, 16, seed=4, chain=300)
    preset, bm = gg.sample_vertices(g.n, 0.6, seed=9)
    for block, chunk, workers, sched in ((64, 64, 1, 0), (1024, 65536, 0, 1), (256, 300, 37, 3)):
        check_preset(ctx, g, preset, bm, algos=(6, 4),
                     opts=T.make_opts(block=block, chunk=chunk, workers=workers, schedule=sched),
                     name=f"block={block} chunk={chunk} workers={workers} schedule={sched}")


def test_plain_call_after_preset(ctx):
    """A plain trim_csr after a preset call on the same context is unaffected."""
    from gpu_common import check_all
    g = gg.rmat(14, 16, seed=2, chain=200)
    preset, bm = gg.sample_vertices(g.n, 0.5, seed=1)
    check_preset(ctx, g, preset, bm, name="rmat14 preset")
    check_all(ctx, g, name="rmat14 plain")


def test_config1_sampled(ctx):
    """R-MAT scale 22 with the chain, half of the vertices sampled: AC-6 and
    AC-4 at full size."""
    g = gg.config1()
    preset, bm = gg.sample_vertices(g.n, 0.5, seed=0)
    check_preset(ctx, g, preset, bm, algos=(6, 4), name="rmat22+chain ratio=0.5")


def test_errors(ctx):
    import paper_2107_12720_amd as T
    g = gg.from_adjacency([[1], [0]])
    ro, col, _, _ = upload(g)
    with pytest.raises(T.TrimError) as e:
        ctx.trim_csr_preset(6, g.n, ro, col, None)
    assert e.value.code == -1
