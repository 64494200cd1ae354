"""Strongly connected components -- TEST INFRASTRUCTURE ONLY.

The partition of V into strongly connected components, which FW-BW SCC
decomposition (Section 1.1, the application of graph trimming) computes:
u and v are in one component iff each reaches the other.  The partition is
unique, so it is the plain definition that any decomposition must match.
It is computed with scipy's strong-component routine (a library primitive)
and given as canonical labels: every vertex is labelled with the smallest
vertex id of its component.  Shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np


def canonical(labels) -> np.ndarray:
    """Relabel a partition so that every vertex carries the smallest vertex id
    of its class (labels are arbitrary ints; equal ints = one class)."""
    labels = np.asarray(labels, dtype=np.int64)
    n = labels.shape[0]
    if n == 0:
        return np.zeros(0, np.int64)
    uniq, inv = np.unique(labels, return_inverse=True)
    first = np.full(uniq.shape[0], n, np.int64)
    np.minimum.at(first, inv, np.arange(n, dtype=np.int64))
    return first[inv]


def scc_labels(g) -> np.ndarray:
    """Canonical SCC labels of the CSR graph g (int64[n])."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    n = g.n
    if n == 0:
        return np.zeros(0, np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_off.astype(np.int64)))
    A = sp.csr_matrix((np.ones(g.m, np.int8), (src, g.col.astype(np.int64))), shape=(n, n))
    _, lab = connected_components(A, directed=True, connection="strong")
    return canonical(lab)


def size2_pairs(g, preset=None) -> np.ndarray:
    """Size-2 SCC trimming (the pattern check that follows size-1 trimming,
    Section 1.1): among the vertices not preset as removed, u and v != u are
    a pair iff each is the other's only remaining predecessor (nothing else
    reaches the pair) or each is the other's only remaining successor (the
    pair reaches nothing else); such a pair is a component of its own.
    Returns partner[u] = v for paired vertices, -1 otherwise.  Plain sets,
    one vertex at a time."""
    n = g.n
    alive = np.ones(n, bool) if preset is None else ~np.asarray(preset, bool)
    ro = g.row_off.astype(np.int64)
    rro = np.zeros(n + 1, np.int64)
    np.add.at(rro, g.col.astype(np.int64) + 1, 1)
    rro = np.cumsum(rro)
    order = np.argsort(g.col, kind="stable")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(ro))[order]
    only_in = np.full(n, -1, np.int64)
    only_out = np.full(n, -1, np.int64)
    for u in range(n):
        if not alive[u]:
            continue
        preds = {int(x) for x in src[rro[u]:rro[u + 1]] if alive[x]}
        succs = {int(x) for x in g.col[ro[u]:ro[u + 1]] if alive[x]}
        if len(preds) == 1 and u not in preds:
            only_in[u] = preds.pop()
        if len(succs) == 1 and u not in succs:
            only_out[u] = succs.pop()
    partner = np.full(n, -1, np.int64)
    for u in range(n):
        for only in (only_in, only_out):
            v = only[u]
            if v >= 0 and only[v] == u:
                partner[u] = v
    return partner


def summary(labels) -> dict:
    """Number of components, of size-1 components, and the largest size."""
    labels = np.asarray(labels)
    if labels.size == 0:
        return {"n_scc": 0, "n_single": 0, "largest": 0}
    _, cnt = np.unique(labels, return_counts=True)
    return {"n_scc": int(cnt.size), "n_single": int((cnt == 1).sum()), "largest": int(cnt.max())}
