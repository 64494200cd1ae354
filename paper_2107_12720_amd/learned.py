"""Learned successor order for AC-6: training and ordering driver.

Host-side orchestration only: every computation (features, forward,
backward, Adam, scoring, reordering) runs in the HIP kernels of libtrim
(mlp.hip, order.hip); this module allocates device buffers and loops over
steps.

Labels are the live sets of the training graphs (the caller supplies them:
the tests and the benchmark use the CPU oracle's).  Training minimises the
binary cross-entropy of "target is live" over edges whose source is live.
The order sorts each list by the network's logit in 16 levels; the range the
levels span is chosen on the training graphs (choose_logit_range), as is the
out-degree heuristic's (choose_degree_range) when the two are compared.
"""
from __future__ import annotations

import numpy as np

NPARAM = 1377
OFFSETS = {"W1": (0, 256), "b1": (256, 32), "W2": (288, 1024), "b2": (1312, 32),
           "w3": (1344, 32), "b3": (1376, 1)}


def init_params(seed: int = 0) -> np.ndarray:
    """Deterministic initial weights: uniform +-sqrt(6/(fan_in+fan_out)), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, np.float32)
    for k, (fi, fo) in (("W1", (8, 32)), ("W2", (32, 32)), ("w3", (32, 1))):
        o, size = OFFSETS[k]
        lim = np.sqrt(6.0 / (fi + fo))
        p[o:o + size] = rng.uniform(-lim, lim, size)
    return p


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 to BF16 (nearest even); uint16 bit patterns (initial copy only)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


class Trainer:
    """FP32 master weights, BF16 copy, Adam moments and a gradient buffer on the GPU."""

    def __init__(self, ctx, seed: int = 0, lr: float = 3e-3):
        import torch
        self.ctx, self.lr = ctx, lr
        p = init_params(seed)
        dev = torch.device("cuda", ctx.device)
        self.p32 = torch.from_numpy(p).to(dev)
        self.pbf = torch.from_numpy(to_bf16_bits(p).view(np.int16)).to(dev)
        self.m1 = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
        self.m2 = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(NPARAM + 1, dtype=torch.float32, device=dev)
        self.step = 0
        self.losses = []

    def train_step(self, graphs, batch: int, seed: int = 1):
        """One Adam step on `batch` hashed edge samples from each graph in `graphs`
        (a list of (DeviceGraph, indeg, src, live_bitmap))."""
        self.step += 1
        for gi, (dg, indeg, src, live) in enumerate(graphs):
            # the gradient is the sum of the graphs' mean losses
            self.ctx.mlp_grad(dg, indeg, src, live, self.pbf, self.grad, batch,
                              seed=seed * 1000003 + gi, step=self.step)
        loss = self.grad[NPARAM:].clone() / len(graphs)
        self.ctx.mlp_adam(self.p32, self.pbf, self.m1, self.m2, self.grad, self.lr, self.step)
        return loss


def prepare(ctx, dg):
    """(indeg, src) device arrays of a DeviceGraph."""
    import torch
    indeg = torch.empty(max(dg.n, 1), dtype=torch.int32, device="cuda")
    src = torch.empty(max(dg.m, 1), dtype=torch.int32, device="cuda")
    ctx.mlp_prepare(dg, indeg, src)
    return indeg, src


# The reorder sorts each list into 16 equal levels of its key over [lo, hi]
# (larger keys first).  Candidate ranges, chosen on the training graphs only.
LOGIT_RANGES = [(lo, hi) for lo in (-8.0, -4.0, 0.0, 4.0, 8.0) for hi in (12.0, 16.0, 24.0, 32.0)]
DEGREE_RANGES = [(lo, hi) for lo in (0.0, 1.0) for hi in (4.0, 6.0, 8.0, 10.0, 12.0, 16.0)]
DEFAULT_LOGIT_RANGE = (0.0, 24.0)


def learned_order(ctx, dg, indeg, src, pbf, key_range=DEFAULT_LOGIT_RANGE):
    """(col_out, scores): successor lists reordered by the network's logit of
    the target staying live, in 16 levels over key_range."""
    import torch
    scores = torch.empty(max(dg.m, 1), dtype=torch.float32, device="cuda")
    ctx.mlp_score(dg, indeg, src, pbf, scores)
    col_out = torch.empty_like(dg.col)
    ctx.order_by_key(dg, scores, float(key_range[0]), float(key_range[1]), col_out)
    return col_out, scores


def _t6_total(ctx, graphs, order):
    """Sum over graphs of AC-6's traversed edges with the lists that
    order(dg, indeg, src) returns."""
    total = 0
    for dg, indeg, src, _ in graphs:
        col = order(dg, indeg, src)
        total += ctx.trim_csr(6, dg.n, dg.row_off, col).stats_dict()["edges_total"]
    return total


def choose_logit_range(ctx, graphs, pbf, ranges=LOGIT_RANGES):
    """The key range with the fewest traversed edges on the training graphs."""
    return min(ranges, key=lambda r: _t6_total(
        ctx, graphs, lambda dg, i, s: learned_order(ctx, dg, i, s, pbf, r)[0]))


def choose_degree_range(ctx, graphs, ranges=DEGREE_RANGES):
    """The same choice for the out-degree heuristic (its key is
    log1p(target out-degree))."""
    return min(ranges, key=lambda r: _t6_total(
        ctx, graphs, lambda dg, i, s: reference_order(ctx, dg, 0, key_range=r)))


def reference_order(ctx, dg, kind: int, seed: int = 0, key_range=None):
    """kind 0: larger target out-degree first (heuristic; key log1p(out-degree),
    default range [0, log1p(m)]); kind 1: random order."""
    import torch
    keys = torch.empty(max(dg.m, 1), dtype=torch.float32, device="cuda")
    ctx.edge_keys(dg, kind, keys, seed=seed)
    if key_range is not None:
        lo, hi = float(key_range[0]), float(key_range[1])
    else:
        lo, hi = (0.0, float(np.log1p(dg.m))) if kind == 0 else (0.0, 1.0)
    col_out = torch.empty_like(dg.col)
    ctx.order_by_key(dg, keys, lo, hi, col_out)
    return col_out
