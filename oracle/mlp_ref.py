"""FP64 CPU reference of the edge-scoring network -- TEST INFRASTRUCTURE ONLY.

Written from the network's definition, sharing no code with the GPU kernels:
8 edge features -> 32 -> 32 -> 1 with ReLU, binary cross-entropy of "target
is live" averaged over the sampled edges (weight 0 when the source is not
live).  Parameter vector (1,377 values): W1[32][8], b1[32], W2[32][32]
(W2[out][in]), b2[32], w3[32], b3.

With ``bf16=True`` the reference rounds, as the GPU does, every value that
enters a BF16 matrix product (weights, features, layer-1 activations, dZ2 and
dZ1); arithmetic is FP64 throughout.  With ``bf16=False`` everything is FP64,
which the finite-difference pin uses.  ``adam_step`` is the optimiser's
update in FP64.
"""
from __future__ import annotations

import numpy as np

OFF = {"W1": (0, (32, 8)), "b1": (256, (32,)), "W2": (288, (32, 32)), "b2": (1312, (32,)),
       "w3": (1344, (32,)), "b3": (1376, (1,))}
NPARAM = 1377
MASK64 = (1 << 64) - 1


def bf16_round(x) -> np.ndarray:
    """Round to BF16 (round to nearest even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def unpack(p):
    return {k: np.asarray(p[o:o + int(np.prod(s))], np.float64).reshape(s)
            for k, (o, s) in OFF.items()}


def splitmix_fin(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finalizer on uint64 arrays (Steele, Lea, Flood 2014)."""
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def features(row_off, col, indeg, edges) -> np.ndarray:
    """Feature rows (FP32 arithmetic, as the GPU computes them) of edge ids."""
    edges = np.asarray(edges, np.int64)
    src = np.searchsorted(row_off, edges, side="right") - 1
    dst = col[edges]
    deg = np.diff(row_off).astype(np.float32)
    lu = np.log1p(deg[src]).astype(np.float32)
    lw = np.log1p(deg[dst]).astype(np.float32)
    h = splitmix_fin((edges - row_off[src]).astype(np.uint64))
    pm = lambda b: np.where((h >> np.uint64(b)) & np.uint64(1), 1.0, -1.0).astype(np.float32)
    X = np.stack([lu, np.log1p(indeg[src].astype(np.float32)), lw,
                  np.log1p(indeg[dst].astype(np.float32)), (lu - lw).astype(np.float32),
                  pm(0), pm(1), pm(2)], 1)
    return X.astype(np.float64), src, dst


def logits(params, X, bf16=True):
    """Network output (logit) for feature rows X, with the same BF16 rounding
    points as loss_and_grad."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    P = unpack(r(params) if bf16 else params)
    h1 = r(np.maximum(r(X) @ P["W1"].T + P["b1"], 0.0))
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    return h2 @ P["w3"] + P["b3"][0]


def loss_and_grad(params, X, y, w, bf16=True):
    """(loss, grad[1377]) of sum_e w_e * BCE(s_e, y_e) for feature rows X."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    P = unpack(r(params) if bf16 else params)
    Xb = r(X)
    z1 = Xb @ P["W1"].T + P["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ P["w3"] + P["b3"][0]
    loss = np.sum(w * (np.maximum(s, 0) - s * y + np.log1p(np.exp(-np.abs(s)))))
    gs = w * (1.0 / (1.0 + np.exp(-s)) - y)
    g = {}
    g["w3"] = gs @ h2
    g["b3"] = np.array([gs.sum()])
    dz2 = gs[:, None] * P["w3"][None, :] * (z2 > 0)
    g["b2"] = dz2.sum(0)
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ h1
    dh1 = dz2r @ P["W2"]
    dz1 = dh1 * (z1 > 0)
    g["b1"] = dz1.sum(0)
    g["W1"] = r(dz1).T @ Xb
    grad = np.zeros(NPARAM)
    for k, (o, sh) in OFF.items():
        grad[o:o + int(np.prod(sh))] = g[k].ravel()
    return loss, grad


def adam_step(params, m, v, grad, lr, beta1, beta2, eps, step):
    """One Adam update in FP64 (Kingma and Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1): the moment estimates
    m <- beta1 m + (1 - beta1) g and v <- beta2 v + (1 - beta2) g^2, their
    bias-corrected values m / (1 - beta1^t) and v / (1 - beta2^t), and the
    step params - lr * m_hat / (sqrt(v_hat) + eps).  Returns (params, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v
