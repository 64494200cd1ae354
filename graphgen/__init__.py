"""Seeded synthetic input graphs for the trimming workloads.

This package only builds inputs: CSR arrays, packed batches and the
parameters of the implicit (hash-generated) graph.  It holds none of the
trimming arithmetic; the GPU library and the CPU oracle both consume what it
produces.  All draws are counter based (SplitMix64 streams), so every graph is
a pure function of its parameters and seed.

Workloads (the paper's benchmark graphs are not available; these synthetic
graphs stand in for them, see the Graph Benchmarks part of Section 9):

* ``core_tail``  -- a random core with out-degree 8 plus a DAG tail whose last
  1 % are sinks (n = 65,536 by default);
* ``rmat``       -- R-MAT (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), optionally
  with a planted chain that forces deep sequential peeling;
* ``implicit``   -- n = 2^28 vertices whose successors come from a hash:
  deg(v) is Zipf(2.1) clamped at 256 with 20 % zero-degree vertices;
* ``batch``      -- thousands of core+tail graphs packed into one CSR.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None

MASK64 = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile libgraphgen.so next to its source (plain C, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        u8p = ctypes.c_void_p
        L.gg_fin64.restype = ctypes.c_uint64
        L.gg_fin64.argtypes = [ctypes.c_uint64]
        L.gg_draw.restype = ctypes.c_uint64
        L.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.gg_core_tail.restype = ctypes.c_int64
        L.gg_core_tail.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]
        L.gg_uniform_edges.restype = None
        L.gg_uniform_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        L.gg_rmat_edges.restype = None
        L.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, i32p, i32p, ctypes.c_int]
        L.gg_chain_ids.restype = ctypes.c_int
        L.gg_chain_ids.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, i32p]
        L.gg_csr.restype = ctypes.c_int64
        L.gg_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_int, u8p,
                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, i32p, ctypes.c_void_p,
                             ctypes.c_int]
        L.gg_transpose.restype = None
        L.gg_transpose.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p]
        L.gg_zipf_table.restype = None
        L.gg_zipf_table.argtypes = [ctypes.c_double, ctypes.c_int, u64p]
        L.gg_batch_params.restype = None
        L.gg_batch_params.argtypes = [ctypes.c_uint64, ctypes.c_int64] + [ctypes.c_double] * 6 + [
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """A directed graph in CSR form (int32 offsets and targets)."""
    n: int
    row_off: np.ndarray
    col: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_off[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_off.astype(np.int64))


def from_edges(n: int, src, dst, drop_self: bool = False, drop_src=None, extra_src=None,
               extra_dst=None, nthreads: int = 0, meta=None) -> CSR:
    """Stable CSR build (sources sorted, successor order = edge-list order)."""
    L = lib()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m0 = src.shape[0]
    ds = None if drop_src is None else np.ascontiguousarray(drop_src, dtype=np.uint8)
    xs = np.zeros(0, np.int32) if extra_src is None else np.ascontiguousarray(extra_src, np.int32)
    xd = np.zeros(0, np.int32) if extra_dst is None else np.ascontiguousarray(extra_dst, np.int32)
    row_off = np.zeros(n + 1, np.int32)
    m = L.gg_csr(n, m0, src, dst, int(drop_self), _ptr(ds), xs.shape[0], _ptr(xs), _ptr(xd),
                 row_off, None, nthreads)
    if m < 0 or m >= 2 ** 31:
        raise ValueError(f"edge count {m} does not fit int32 CSR")
    col = np.empty(m, np.int32)
    L.gg_csr(n, m0, src, dst, int(drop_self), _ptr(ds), xs.shape[0], _ptr(xs), _ptr(xd),
             row_off, _ptr(col), nthreads)
    return CSR(n, row_off, col, dict(meta or {}))


def from_adjacency(adj) -> CSR:
    """CSR from a list of successor lists (small hand-written graphs)."""
    n = len(adj)
    row_off = np.zeros(n + 1, np.int32)
    row_off[1:] = np.cumsum([len(a) for a in adj])
    col = np.array([w for a in adj for w in a], dtype=np.int32)
    return CSR(n, row_off, col)


def core_tail(n: int = 65536, seed: int = 0, core_frac: float = 0.7, core_deg: int = 8,
              tail_lambda: float = 3.0, sink_frac: float = 0.01, core_lambda: float = 0.0,
              drop_self: bool = True, min_sink: int = 0) -> CSR:
    """Random core + DAG tail.  With the defaults: n_core = floor(0.7 n) vertices of
    out-degree 8 (targets uniform in the core, self-loops dropped); the tail has
    Poisson(3) out-degrees to uniformly chosen higher-indexed vertices; the last
    floor(0.01 n) vertices are sinks.  core_deg < 0 draws core degrees from
    Poisson(core_lambda) instead."""
    L = lib()
    n_core = int(math.floor(core_frac * n))
    n_sink = max(min_sink, int(math.floor(sink_frac * n)))
    row_off = np.zeros(n + 1, np.int32)
    m = L.gg_core_tail(n, n_core, n_sink, core_deg, core_lambda, tail_lambda, seed & MASK64,
                       int(drop_self), _ptr(row_off), None)
    col = np.empty(m, np.int32)
    L.gg_core_tail(n, n_core, n_sink, core_deg, core_lambda, tail_lambda, seed & MASK64,
                   int(drop_self), _ptr(row_off), _ptr(col))
    return CSR(n, row_off, col, dict(kind="core_tail", n_core=n_core, n_sink=n_sink, seed=seed))


def uniform(n: int, m: int, seed: int = 0, drop_self: bool = False) -> CSR:
    """m uniform random edges (duplicates, and self-loops unless dropped)."""
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    lib().gg_uniform_edges(n, m, seed & MASK64, src, dst)
    return from_edges(n, src, dst, drop_self=drop_self, nthreads=1,
                      meta=dict(kind="uniform", seed=seed))


def rmat(scale: int, edge_factor: int = 16, seed: int = 0, chain: int = 0,
         abc=(0.57, 0.19, 0.19), nthreads: int = 0) -> CSR:
    """R-MAT graph on 2^scale vertices with edge_factor * 2^scale generated edges,
    self-loops removed, duplicates kept.  With chain = L > 0, L distinct seeded
    vertices c_0..c_{L-1} lose all their out-edges and get c_i -> c_{i+1}; the
    last one is a sink, so peeling needs at least L steps."""
    n = 1 << scale
    m0 = edge_factor * n
    src = np.empty(m0, np.int32)
    dst = np.empty(m0, np.int32)
    a, b, c = abc
    lib().gg_rmat_edges(scale, m0, seed & MASK64, a, b, c, src, dst, nthreads)
    drop = None
    xs = xd = None
    chain_ids = None
    if chain > 0:
        chain_ids = np.empty(chain, np.int32)
        if lib().gg_chain_ids(n, chain, seed & MASK64, chain_ids) != 0:
            raise ValueError("chain longer than the vertex count")
        drop = np.zeros(n, np.uint8)
        drop[chain_ids] = 1
        xs, xd = chain_ids[:-1].copy(), chain_ids[1:].copy()
    g = from_edges(n, src, dst, drop_self=True, drop_src=drop, extra_src=xs, extra_dst=xd,
                   nthreads=nthreads,
                   meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor, seed=seed,
                             chain=chain))
    del src, dst
    if chain_ids is not None:
        g.meta["chain_ids"] = chain_ids
    return g


def sample_vertices(n: int, ratio: float, seed: int = 0):
    """Vertex sampling of the scalability experiments: each vertex is kept with
    probability `ratio`; the others are to be removed before trimming.
    Returns (preset uint8[n], 1 = not sampled; the same flags as a uint32
    bitmap of ceil(n/32) words, bit v % 32 of word v // 32)."""
    rng = np.random.default_rng([seed & MASK64, 0x5653414D])   # stream tag "VSAM"
    preset = (rng.random(n) >= ratio).astype(np.uint8)
    words = (n + 31) // 32
    bits = np.zeros(max(words, 1) * 32, np.uint8)
    bits[:n] = preset
    bm = np.packbits(bits, bitorder="little").view(np.uint32)[:max(words, 1)].copy()
    return preset, bm


def sample_edges(g: CSR, ratio: float, seed: int = 0) -> CSR:
    """Edge sampling of the scalability experiments: each edge is kept with
    probability `ratio`, in its list order; the others are dropped."""
    rng = np.random.default_rng([seed & MASK64, 0x4553414D])   # stream tag "ESAM"
    keep = rng.random(g.m) < ratio
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_off.astype(np.int64)))
    cnt = np.bincount(src[keep], minlength=g.n)
    row_off = np.zeros(g.n + 1, np.int32)
    np.cumsum(cnt, out=row_off[1:])
    return CSR(g.n, row_off, g.col[keep].astype(np.int32),
               dict(g.meta, edge_sample=ratio, edge_sample_seed=seed))


def transpose(g: CSR):
    """(rrow_off, rcol): the transposed graph G^T in CSR form."""
    rrow_off = np.zeros(g.n + 1, np.int32)
    rcol = np.empty(g.m, np.int32)
    lib().gg_transpose(g.n, g.row_off, g.col, rrow_off, rcol)
    return rrow_off, rcol


# ---------------------------------------------------------------- implicit
@dataclass
class Implicit:
    """Parameters of the hash-generated graph G = (V, POST).

    n = 2^log2n.  deg(v) = 0 when fin64(seed ^ T_ZERO ^ (v << 8)) < zero_thr,
    else 1 + #{j : fin64(seed ^ T_DEG ^ (v << 8)) >= table[j], j < 255}
    (Zipf(s) clamped at 256 by inverse CDF).  Successor i of v is
    fin64(seed ^ T_NBR ^ ((v << 8) | i)) & (n - 1).  fin64 is the SplitMix64
    finalizer; self-loops and duplicates are kept."""
    log2n: int
    seed: int
    zero_thr: int
    table: np.ndarray          # uint64[256]
    s: float = 2.1
    zero_frac: float = 0.2

    @property
    def n(self) -> int:
        return 1 << self.log2n


# tags xored into the hash input; shared constants of the workload definition
IMPLICIT_TAG_ZERO = 0x5A45524F00000000   # "ZERO"
IMPLICIT_TAG_DEG = 0x4445470000000000    # "DEG"
IMPLICIT_TAG_NBR = 0x4E42520000000000    # "NBR"


def zipf_table(s: float = 2.1, cap: int = 256) -> np.ndarray:
    t = np.zeros(cap, np.uint64)
    lib().gg_zipf_table(s, cap, t)
    return t


def implicit(log2n: int = 28, seed: int = 0, s: float = 2.1, cap: int = 256,
             zero_frac: float = 0.2) -> Implicit:
    if cap != 256:
        raise ValueError("the implicit graph uses a 256-entry degree table")
    thr = int(math.floor(zero_frac * 2.0 ** 64))
    return Implicit(log2n, seed & MASK64, min(thr, MASK64), zipf_table(s, cap), s, zero_frac)


def fin64(z: int) -> int:
    return int(lib().gg_fin64(z & MASK64))


# ------------------------------------------------------------------ batches
@dataclass
class Batch:
    """Packed multi-graph CSR: graph g owns vertices [vbase[g], vbase[g+1]) and
    edges [ebase[g], ebase[g+1]); row_off is absolute into col; col holds
    graph-local target ids."""
    vbase: np.ndarray   # int64[G+1]
    ebase: np.ndarray   # int64[G+1]
    row_off: np.ndarray  # int32[sum n + 1]
    col: np.ndarray      # int32[sum m]
    params: list

    @property
    def G(self) -> int:
        return self.vbase.shape[0] - 1

    def graph(self, g: int) -> CSR:
        v0, v1 = int(self.vbase[g]), int(self.vbase[g + 1])
        e0, e1 = int(self.ebase[g]), int(self.ebase[g + 1])
        ro = (self.row_off[v0:v1 + 1] - e0).astype(np.int32)
        return CSR(v1 - v0, ro, self.col[e0:e1].copy())

    def bitmap_base(self) -> np.ndarray:
        """Word offset of each graph's live bitmap (graphs start on word boundaries)."""
        words = (np.diff(self.vbase) + 31) // 32
        bb = np.zeros(self.G + 1, np.int64)
        bb[1:] = np.cumsum(words)
        return bb


def batch(G: int = 4096, seed: int = 0, n_range=(100, 100000), d_range=(1.0, 8.0),
          f_range=(0.1, 0.6)) -> Batch:
    """G independent core+tail graphs: n log-uniform in n_range, mean out-degree
    d uniform in d_range (core and tail degrees Poisson(d), core targets uniform
    in the core), tail fraction f uniform in f_range, the last max(1, floor(0.01 n))
    vertices are sinks, self-loops dropped."""
    L = lib()
    n_ = ctypes.c_int32()
    d_ = ctypes.c_double()
    f_ = ctypes.c_double()
    s_ = ctypes.c_uint64()
    params = []
    for g in range(G):
        L.gg_batch_params(seed & MASK64, g, float(n_range[0]), float(n_range[1]), d_range[0],
                          d_range[1], f_range[0], f_range[1], ctypes.byref(n_), ctypes.byref(d_),
                          ctypes.byref(f_), ctypes.byref(s_))
        params.append((n_.value, d_.value, f_.value, s_.value))
    vbase = np.zeros(G + 1, np.int64)
    vbase[1:] = np.cumsum([p[0] for p in params])
    row_parts, col_parts = [], []
    ebase = np.zeros(G + 1, np.int64)
    for g, (n, d, f, gs) in enumerate(params):
        n_tail = int(math.floor(f * n))
        n_core = n - n_tail
        n_sink = max(1, int(math.floor(0.01 * n)))
        ro = np.zeros(n + 1, np.int32)
        m = L.gg_core_tail(n, n_core, n_sink, -1, d, d, gs, 1, _ptr(ro), None)
        c = np.empty(m, np.int32)
        L.gg_core_tail(n, n_core, n_sink, -1, d, d, gs, 1, _ptr(ro), _ptr(c))
        ebase[g + 1] = ebase[g] + m
        row_parts.append(ro[:-1].astype(np.int64) + ebase[g])
        col_parts.append(c)
    if ebase[-1] >= 2 ** 31:
        raise ValueError("packed batch exceeds int32 edge offsets")
    row_off = np.empty(int(vbase[-1]) + 1, np.int32)
    row_off[:-1] = np.concatenate(row_parts)
    row_off[-1] = ebase[-1]
    col = np.concatenate(col_parts).astype(np.int32)
    return Batch(vbase, ebase, row_off, col, params)


# ------------------------------------------------------------ named configs
def config0(seed: int = 0) -> CSR:
    """n = 65,536 core+tail graph, seed 0."""
    return core_tail(65536, seed)


def config1(seed: int = 0, nthreads: int = 0) -> CSR:
    """R-MAT scale 22, edge factor 16, with a planted 100,000-vertex chain."""
    return rmat(22, 16, seed, chain=100000, nthreads=nthreads)


def config2_explicit(seed: int = 0, nthreads: int = 0) -> CSR:
    """R-MAT scale 26, edge factor 16 (about 1.07e9 edges)."""
    return rmat(26, 16, seed, nthreads=nthreads)
