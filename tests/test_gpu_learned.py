"""GPU checks of the learned successor order.

* The fused forward/backward kernel against the FP64 CPU reference, which
  rounds to BF16 where the GPU feeds an MFMA (tolerance 1e-2 relative to the
  largest gradient of each parameter group; loss to 1e-4).
* The per-vertex reorder is a stable bucketed sort of each successor list.
* Training lowers the loss.
* Any order gives the same live bitmap; the traversed-edge total under the
  learned order equals the closed form on the reordered graph and is at
  least the lower bound T6min.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_12720_amd as T
    c = T.Context(0)
    yield c
    c.close()


def device_graph(g):
    import paper_2107_12720_amd as T
    return T.DeviceGraph.upload(g)


def test_gradient_vs_fp64_reference(ctx):
    import torch
    import paper_2107_12720_amd as T
    from paper_2107_12720_amd import learned
    from oracle import mlp_ref
    g = gg.rmat(12, 8, seed=4)
    r = oracle.peel(g)
    dg = device_graph(g)
    indeg, src = learned.prepare(ctx, dg)
    live = T.to_device(oracle.bitmap(r.live).view(np.int32))
    rng = np.random.default_rng(3)
    for trial in range(3):
        p = learned.init_params(seed=trial) * (1.0 + trial)
        p[256:288] = rng.normal(0, 0.1, 32)      # nonzero biases
        p[1312:1344] = rng.normal(0, 0.1, 32)
        pbf_bits = learned.to_bf16_bits(p)
        pbf = T.to_device(pbf_bits.view(np.int16))
        ids = rng.integers(0, g.m, 3000).astype(np.int64)
        grad = torch.zeros(T.MLP_PARAMS + 1, dtype=torch.float32, device="cuda")
        ctx.mlp_grad(dg, indeg, src, live, pbf, grad, len(ids), edge_ids=T.to_device(ids))
        torch.cuda.synchronize()
        gg_ = grad.cpu().numpy().astype(np.float64)
        X, s_, d_ = mlp_ref.features(g.row_off.astype(np.int64), g.col,
                                     np.bincount(g.col, minlength=g.n), ids)
        y = r.live[d_].astype(float)
        w = r.live[s_].astype(float) / len(ids)
        # the reference uses the same BF16 weights the GPU reads
        pw = pbf_bits.astype(np.uint32) << 16
        loss, ref = mlp_ref.loss_and_grad(pw.view(np.float32).astype(np.float64), X, y, w,
                                          bf16=True)
        say(f"  trial {trial}: loss gpu {gg_[-1]:.6f} ref {loss:.6f}")
        assert abs(gg_[-1] - loss) <= 1e-4 * max(1.0, abs(loss))
        for k, (o, sh) in mlp_ref.OFF.items():
            sz = int(np.prod(sh))
            a, b = gg_[o:o + sz], ref[o:o + sz]
            err = np.max(np.abs(a - b))
            assert err <= 1e-2 * np.max(np.abs(b)) + 1e-7, (k, err, np.max(np.abs(b)))


def test_adam_vs_fp64_reference(ctx):
    """Three optimiser steps of trim_mlp_adam against the FP64 Adam of
    oracle.mlp_ref (Kingma and Ba, Algorithm 1), element by element, within
    a first-order FP32 error budget carried through the steps: each FP32
    operation rounds with relative error at most u = 2^-24, so a moment
    m = b1 m' + (1 - b1) g is off by at most 3u (b1 |m'| + (1 - b1) |g|) plus
    b1 times the previous error (the two terms may cancel, so the bound is on
    the terms, not on m); the weight step lr m_hat / (sqrt(v_hat) + eps)
    inherits the moments' errors through its partial derivatives, plus 6u of
    its own, and the new weight rounds once more.  The BF16 copy must equal
    the round-to-nearest-even of the GPU's own FP32 weights, and the gradient
    buffer (loss word included) must be cleared."""
    import torch
    import paper_2107_12720_amd as T
    from paper_2107_12720_amd import learned
    from oracle import mlp_ref
    rng = np.random.default_rng(11)
    n = T.MLP_PARAMS
    u = 2.0 ** -24
    p32 = learned.init_params(seed=5).astype(np.float32)
    p32[256:288] = rng.normal(0, 0.1, 32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = dev(p32)
    PB = torch.zeros(n, dtype=torch.int16, device="cuda")
    M1 = torch.zeros(n, dtype=torch.float32, device="cuda")
    M2 = torch.zeros(n, dtype=torch.float32, device="cuda")
    lr, b1, b2, eps = [float(np.float32(x)) for x in (3e-3, 0.9, 0.999, 1e-8)]
    rp, rm, rv = p32.astype(np.float64), np.zeros(n), np.zeros(n)
    em, ev, ep = np.zeros(n), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        g = (rng.normal(0, 1, n) * 10.0 ** rng.uniform(-4, 1, n)).astype(np.float32)
        g[::97] = 0.0
        G = dev(np.r_[g, np.float32(1.5)])         # the loss word follows the gradients
        ctx.mlp_adam(P, PB, M1, M2, G, lr, step, beta1=b1, beta2=b2, eps=eps)
        torch.cuda.synchronize()
        g64 = g.astype(np.float64)
        em = b1 * em + 3 * u * (b1 * np.abs(rm) + (1 - b1) * np.abs(g64))
        ev = b2 * ev + 4 * u * (b2 * rv + (1 - b2) * g64 * g64)
        rp, rm, rv = mlp_ref.adam_step(rp, rm, rv, g64, lr, b1, b2, eps, step)
        c1, c2 = 1 / (1 - b1 ** step), 1 / (1 - b2 ** step)
        den = np.sqrt(rv * c2) + eps
        step_ = lr * rm * c1 / den
        d_dm = lr * c1 / den
        d_dv = 0.5 * lr * np.abs(rm) * c1 * np.sqrt(c2) / (den * den * np.sqrt(np.maximum(rv, 1e-300)))
        ep = ep + d_dm * em + d_dv * ev + 6 * u * np.abs(step_) + u * np.abs(rp)
        gm, gv, gp = (t.cpu().numpy().astype(np.float64) for t in (M1, M2, P))
        for name, got, ref, bud in (("m", gm, rm, em), ("v", gv, rv, ev), ("p", gp, rp, ep)):
            bad = np.abs(got - ref) > bud * 1.01 + 1e-30
            assert not bad.any(), (step, name, np.flatnonzero(bad)[:5], (got - ref)[bad][:5],
                                   bud[bad][:5])
        bits = PB.cpu().numpy().view(np.uint16)
        assert np.array_equal(bits, mlp_ref.bf16_bits(P.cpu().numpy()))
        assert not G.cpu().numpy().any()
        say(f"  step {step}: max |dp| gpu-ref {np.max(np.abs(gp - rp)):.3e}, "
            f"max budget {np.max(ep):.3e}")


def test_scores_vs_fp64_reference(ctx):
    """Every edge's logit from the scoring kernel against the FP64 forward
    pass on the same BF16 weights (FP32 accumulation against FP64: 1e-3 of
    the logit's scale), and the probabilities they give."""
    import torch
    import paper_2107_12720_amd as T
    from paper_2107_12720_amd import learned
    from oracle import mlp_ref
    g = gg.rmat(11, 8, seed=6)
    dg = device_graph(g)
    indeg, src = learned.prepare(ctx, dg)
    p = learned.init_params(seed=4) * 2.0
    p[256:288] = np.random.default_rng(1).normal(0, 0.1, 32)
    bits = learned.to_bf16_bits(p)
    scores = torch.empty(g.m, dtype=torch.float32, device="cuda")
    ctx.mlp_score(dg, indeg, src, T.to_device(bits.view(np.int16)), scores)
    torch.cuda.synchronize()
    X, _, _ = mlp_ref.features(g.row_off.astype(np.int64), g.col,
                               np.bincount(g.col, minlength=g.n), np.arange(g.m))
    pw = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    want = mlp_ref.logits(pw, X)
    got = scores.cpu().numpy().astype(np.float64)
    zerr = np.max(np.abs(got - want) / (1.0 + np.abs(want)))
    perr = np.max(np.abs(1.0 / (1.0 + np.exp(-got)) - 1.0 / (1.0 + np.exp(-want))))
    say(f"  scores: m={g.m} max |z_gpu - z_ref| / (1 + |z_ref|) = {zerr:.2e}, "
        f"max |p_gpu - p_ref| = {perr:.2e}")
    assert zerr <= 1e-3 and perr <= 2e-3


def hub_graph():
    """Random graph plus lists longer than one wavefront's share (2,048
    entries): a hub of 50,000 successors, one of exactly 2,049, one of 2,048,
    and a vertex with no successors between them."""
    rng = np.random.default_rng(7)
    n = 60000
    s0, d0 = rng.integers(0, n, 200000), rng.integers(0, n, 200000)
    keep = ~np.isin(s0, (3, 10, 11, 12))
    src, dst = [s0[keep]], [d0[keep]]
    for v, d in ((3, 50000), (10, 2049), (12, 2048)):
        src.append(np.full(d, v))
        dst.append(rng.integers(0, n, d))
    return gg.from_edges(n, np.concatenate(src), np.concatenate(dst))


def exact_tiles_graph():
    """m = 3 x 4,096 exactly, the last vertex's list of 5,000 entries ending
    at m, and vertices 0..99 without successors."""
    rng = np.random.default_rng(8)
    n = 1000
    s = np.concatenate([rng.integers(100, n - 1, 3 * 4096 - 5000), np.full(5000, n - 1)])
    return gg.from_edges(n, s, rng.integers(0, n, s.shape[0]))


@pytest.mark.parametrize("which", ["rmat13", "hubs", "exact_tiles"])
def test_order_is_stable_bucketed_permutation(ctx, which):
    import torch
    from paper_2107_12720_amd import learned
    g = {"rmat13": lambda: gg.rmat(13, 16, seed=9), "hubs": hub_graph,
         "exact_tiles": exact_tiles_graph}[which]()
    say(f"  {which}: n={g.n} m={g.m} max deg={int(np.diff(g.row_off).max())}")
    dg = device_graph(g)
    keys = torch.empty(g.m, dtype=torch.float32, device="cuda")
    ctx.edge_keys(dg, 1, keys, seed=5)
    out = torch.empty_like(dg.col)
    ctx.order_by_key(dg, keys, 0.0, 1.0, out)
    indeg, src_d = learned.prepare(ctx, dg)
    torch.cuda.synchronize()
    k = keys.cpu().numpy()
    got = out.cpu().numpy()
    scale = np.float32(16.0)
    bucket = np.clip(((np.float32(1.0) - k) * scale).astype(np.int32), 0, 15)
    src = np.repeat(np.arange(g.n), np.diff(g.row_off))
    order = np.lexsort((np.arange(g.m), bucket, src))     # stable by (src, bucket)
    assert np.array_equal(got, g.col[order])
    assert np.array_equal(src_d.cpu().numpy()[:g.m], src)
    assert np.array_equal(indeg.cpu().numpy()[:g.n], np.bincount(g.col, minlength=g.n))


def test_training_lowers_loss_and_order_keeps_live_set(ctx):
    import torch
    import paper_2107_12720_amd as T
    from paper_2107_12720_amd import learned
    from gpu_common import upload, run_csr
    graphs = []
    for seed in (1, 2):
        g = gg.rmat(14, 16, seed=seed)
        dg = device_graph(g)
        indeg, src = learned.prepare(ctx, dg)
        labels = T.to_device(oracle.bitmap(oracle.peel(g).live).view(np.int32))   # oracle labels
        graphs.append((dg, indeg, src, labels))
    tr = learned.Trainer(ctx, seed=0, lr=1e-2)
    losses = [float(tr.train_step(graphs, 1 << 14, seed=7)) for _ in range(60)]
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.mean(losses[-10:]) < 0.8 * np.mean(losses[:5])
    # evaluate on another graph
    g = gg.rmat(15, 16, seed=3)
    dg = device_graph(g)
    indeg, src = learned.prepare(ctx, dg)
    col_l, _ = learned.learned_order(ctx, dg, indeg, src, tr.pbf)
    col_h = learned.reference_order(ctx, dg, 0)
    col_r = learned.reference_order(ctx, dg, 1, seed=11)
    torch.cuda.synchronize()
    r = oracle.peel(g)
    base = oracle.counts(g, r)
    for name, col in (("learned", col_l), ("heuristic", col_h), ("random", col_r)):
        go = gg.CSR(g.n, g.row_off, col.cpu().numpy())
        # same multiset of successors per vertex
        assert np.array_equal(np.sort(go.col + np.repeat(np.arange(g.n), np.diff(g.row_off)) *
                                      np.int64(g.n)),
                              np.sort(g.col + np.repeat(np.arange(g.n), np.diff(g.row_off)) *
                                      np.int64(g.n)))
        ro = oracle.peel(go)
        c = oracle.counts(go, ro)
        res = ctx.trim_csr(6, g.n, dg.row_off, col)
        torch.cuda.synchronize()
        st = res.stats_dict()
        assert np.array_equal(res.bitmap_numpy()[:(g.n + 31) // 32], oracle.bitmap(r.live))
        assert st["edges_total"] == c.T6 and c.T6min == base.T6min <= c.T6
        say(f"  {name}: T6 {c.T6} (plain {base.T6}, min {base.T6min})")
        if name == "learned":
            t6_learned = c.T6
    # what the trained network gains over plain AC-6: fewer traversed edges
    assert t6_learned < base.T6


@pytest.mark.timeout(900)
def test_config4_full(ctx):
    """The learned-order workload at its full size, in the benchmark's setup:
    trained on oracle labels of 16 R-MAT scale-20 graphs (seeds 1..16),
    evaluated on R-MAT scale 24.  The reordered graph keeps the live set bit
    for bit, its traversed-edge total equals the closed form on the permuted
    lists and is below plain AC-6's; the scoring kernel matches the FP64
    reference on 10,000 sampled edges; sampled lists are permutations."""
    import torch
    import paper_2107_12720_amd as T
    from paper_2107_12720_amd import learned
    from oracle import mlp_ref
    say("  learned order: 16 training graphs (R-MAT 20) with oracle labels ...")
    train = []
    for seed in range(1, 17):
        g = gg.rmat(20, 16, seed=seed)
        dg = device_graph(g)
        indeg, src = learned.prepare(ctx, dg)
        labels = T.to_device(oracle.bitmap(oracle.peel(g).live).view(np.int32))
        train.append((dg, indeg, src, labels))
    tr = learned.Trainer(ctx, seed=0, lr=5e-3)
    losses = [float(tr.train_step(train, 1 << 14, seed=1)) for _ in range(300)]
    say(f"  loss {losses[0]:.4f} -> {np.mean(losses[-10:]):.4f}")
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:5])
    del train
    say("  evaluation graph R-MAT 24 ...")
    g = gg.rmat(24, 16, seed=0)
    dg = device_graph(g)
    indeg, src = learned.prepare(ctx, dg)
    col_l, scores = learned.learned_order(ctx, dg, indeg, src, tr.pbf)
    res = ctx.trim_csr(6, g.n, dg.row_off, col_l)
    torch.cuda.synchronize()
    r = oracle.peel(g)
    base = oracle.counts(g, r)
    assert np.array_equal(res.bitmap_numpy()[:(g.n + 31) // 32], oracle.bitmap(r.live))
    go = gg.CSR(g.n, g.row_off, col_l.cpu().numpy())
    c = oracle.counts(go, r)   # the levels do not depend on the order
    st = res.stats_dict()
    say(f"  T6 learned {c.T6}, plain {base.T6}, min {base.T6min}")
    assert st["edges_total"] == c.T6 and base.T6min <= c.T6 < base.T6
    rng = np.random.default_rng(24)
    for v in rng.integers(0, g.n, 10000):
        a, b = g.row_off[v], g.row_off[v + 1]
        assert np.array_equal(np.sort(go.col[a:b]), np.sort(g.col[a:b])), int(v)
    ids = rng.integers(0, g.m, 10000)
    X, _, _ = mlp_ref.features(g.row_off.astype(np.int64), g.col,
                               np.bincount(g.col, minlength=g.n), ids)
    bits = tr.pbf.cpu().numpy().view(np.uint16)
    pw = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    want = mlp_ref.logits(pw, X)
    got = scores.cpu().numpy()[ids].astype(np.float64)
    err = np.max(np.abs(got - want) / (1.0 + np.abs(want)))
    say(f"  sampled logits: max |z_gpu - z_ref| / (1 + |z_ref|) = {err:.2e}")
    assert err <= 1e-3
