"""CPU oracle for graph trimming -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The GPU library never calls it, and
it shares no code with the GPU path: liboracle.so is built from
``oracle/oracle.c`` alone.

Paper: "Efficient Parallel Graph Trimming by Arc-Consistency" (arXiv
2107.12720).  What each routine follows:

* :func:`peel` -- the trimmed graph (Def. Trimmed Graph, Section 2) and the
  peeling step of every removed vertex (Def. of alpha, Section 2.4), computed
  with the out-degree counters over G^T of the sequential AC-4-based algorithm
  (Section 5.1), counters taken from CSR offsets (AC4Trim*, Section 9.3).
* :func:`ac6_seq` -- the sequential AC-6-based algorithm (Section 6.1), run
  literally, counting successor checks.
* :func:`ac3` -- the AC-3-based algorithm (Section 4.1) with the edge_index
  cursor (Section 8); ``jacobi=True`` reads the statuses of the start of each
  repetition.
* :func:`counts` -- closed forms of the traversed-edge totals.
* :func:`implicit_csr` -- materialises the hash-generated graph with the
  oracle's own SplitMix64 implementation.
* :func:`peel` and :func:`counts` with ``preset`` -- some vertices set to DEAD
  before trimming starts (the vertex sampling of the scalability experiments,
  Section 9).
* :func:`peel2` -- two-sided trimming, the first improvement listed in
  Section 4.1: a vertex must also keep a live predecessor (checked over G^T);
  two counters per vertex, removed vertices processed in peeling-step order.
* :func:`counts2` -- totals of the two-sided algorithms for a final live set.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so from oracle.c (gcc, -O2, OpenMP for batches only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = load(_SO)
    return _lib


def swap_library(L):
    """Make every oracle function call the library handle ``L`` (from
    :func:`load`); returns the handle in use before.  The mutation pins use it
    to run the pins against copies of oracle.c with planted mistakes."""
    global _lib
    old = lib()
    _lib = L
    return old


def load(path: str):
    """Open a build of oracle.c and declare its functions."""
    L = ctypes.CDLL(path)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    L.or_peel.restype = ctypes.c_int64
    L.or_peel.argtypes = [ctypes.c_int32, i32p, i32p, u8p, i32p, i32p, i64p]
    for f in (L.or_ac6_seq, L.or_ac3_jacobi, L.or_ac3_inplace):
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_int32, i32p, i32p, u8p, i64p]
    L.or_counts.restype = ctypes.c_int64
    L.or_counts.argtypes = [ctypes.c_int32, i32p, i32p, u8p, i32p, ctypes.c_int32, i64p]
    L.or_implicit_deg.restype = ctypes.c_int32
    L.or_implicit_deg.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p, ctypes.c_uint64]
    L.or_implicit_nbr.restype = ctypes.c_int32
    L.or_implicit_nbr.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.c_uint64]
    L.or_implicit_csr.restype = ctypes.c_int64
    L.or_implicit_csr.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u64p, i32p,
                                  ctypes.c_void_p]
    L.or_batch_peel.restype = ctypes.c_int64
    L.or_batch_peel.argtypes = [ctypes.c_int64, i64p, i32p, i32p, u8p, i64p, ctypes.c_int]
    L.or_peel_preset.restype = ctypes.c_int64
    L.or_peel_preset.argtypes = [ctypes.c_int32, i32p, i32p, u8p, u8p, i32p, i32p, i64p]
    L.or_counts_preset.restype = ctypes.c_int64
    L.or_counts_preset.argtypes = [ctypes.c_int32, i32p, i32p, u8p, u8p, i32p,
                                   ctypes.c_int32, i64p]
    L.or_peel2.restype = ctypes.c_int64
    L.or_peel2.argtypes = [ctypes.c_int32, i32p, i32p, u8p, i32p, i32p, i64p]
    L.or_counts2.restype = ctypes.c_int64
    L.or_counts2.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, u8p, i64p]
    L.or_ac3_jacobi2.restype = ctypes.c_int64
    L.or_ac3_jacobi2.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, u8p, i32p, i64p]
    L.or_counts3two.restype = ctypes.c_int64
    L.or_counts3two.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, u8p, i32p, i64p]
    L.or_ac6_deferred.restype = ctypes.c_int64
    L.or_ac6_deferred.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, u8p, i64p]
    L.or_counts_deferred.restype = ctypes.c_int64
    L.or_counts_deferred.argtypes = [ctypes.c_int32, i32p, i32p, u8p, i32p, ctypes.c_int32,
                                     ctypes.c_int32, i64p]
    L.or_num_threads.restype = ctypes.c_int
    L.or_fin64.restype = ctypes.c_uint64
    L.or_fin64.argtypes = [ctypes.c_uint64]
    return L


def num_threads() -> int:
    return int(lib().or_num_threads())


@dataclass
class PeelResult:
    live: np.ndarray      # uint8[n], 1 = LIVE
    level: np.ndarray     # int32[n], peeling step (0 for live vertices)
    order: np.ndarray     # int32[n_dead], removal order
    alpha: int
    n_live: int
    rev_edges: int        # reverse edges traversed during propagation

    @property
    def n_dead(self) -> int:
        return int(self.order.shape[0])


@dataclass
class Counts:
    T6: int
    T4s: int
    T4: int
    T3J: int
    rounds3: int
    T6min: int
    m: int
    n_live: int


def _csr(g):
    return (np.ascontiguousarray(g.row_off, dtype=np.int32),
            np.ascontiguousarray(g.col, dtype=np.int32))


def _preset(g, preset):
    p = np.ascontiguousarray(preset, dtype=np.uint8)
    if p.shape != (g.n,):
        raise ValueError("preset must hold one flag per vertex")
    return p


def peel(g, preset=None) -> PeelResult:
    """Greatest vertex set in which every vertex keeps a live successor, plus the
    peeling step of every other vertex.  With ``preset`` (one flag per vertex),
    the flagged vertices are DEAD from the start (level 0, not in ``order``)."""
    ro, col = _csr(g)
    live = np.empty(g.n, np.uint8)
    level = np.empty(g.n, np.int32)
    order = np.empty(max(g.n, 1), np.int32)
    st = np.zeros(3, np.int64)
    if preset is not None:
        nd = lib().or_peel_preset(g.n, ro, col, _preset(g, preset), live, level, order, st)
    else:
        nd = lib().or_peel(g.n, ro, col, live, level, order, st)
    if nd < 0:
        raise MemoryError("oracle peel: allocation failed")
    return PeelResult(live, level, order[:nd].copy(), int(st[0]), int(st[1]), int(st[2]))


@dataclass
class Counts2:
    T6live: int     # two-sided AC-6 checks made by the vertices that stay live
    dead_lo: int    # least checks the removed vertices can make
    dead_hi: int    # most checks the removed vertices can make
    T4two: int      # two-sided AC-4: edges walked, both directions
    n_live: int


def peel2(g) -> PeelResult:
    """Greatest vertex set in which every vertex keeps a live successor and a
    live predecessor, plus the peeling step of every other vertex.
    ``rev_edges`` counts the edges walked in both directions."""
    ro, col = _csr(g)
    live = np.empty(g.n, np.uint8)
    level = np.empty(g.n, np.int32)
    order = np.empty(max(g.n, 1), np.int32)
    st = np.zeros(3, np.int64)
    nd = lib().or_peel2(g.n, ro, col, live, level, order, st)
    if nd < 0:
        raise MemoryError("oracle peel2: allocation failed")
    return PeelResult(live, level, order[:nd].copy(), int(st[0]), int(st[1]), int(st[2]))


def counts2(g, rrow_off, rcol, live) -> Counts2:
    """Totals of the two-sided algorithms for the live set ``live``, with G^T
    given as (rrow_off, rcol) in the order the in-side scans use."""
    ro, col = _csr(g)
    rro = np.ascontiguousarray(rrow_off, dtype=np.int32)
    rc = np.ascontiguousarray(rcol, dtype=np.int32)
    out = np.zeros(5, np.int64)
    r = lib().or_counts2(g.n, ro, col, rro, rc, np.ascontiguousarray(live, np.uint8), out)
    if r != 0:
        raise ValueError(f"oracle counts2: live vertex {-r - 1} lacks a live neighbour")
    return Counts2(*[int(x) for x in out])


@dataclass
class Ac3Two:
    live: np.ndarray    # uint8, 1 = LIVE
    level: np.ndarray   # int32 removal round, 0 for live vertices
    edges: int          # traversed edges (successor and predecessor checks)
    rounds: int
    n_live: int


def ac3_jacobi2(g, rrow_off, rcol) -> Ac3Two:
    """The two-sided AC-3 rounds run literally (successors first, then
    predecessors, statuses of the round's start); G^T is (rrow_off, rcol) in
    the order the predecessor scans use."""
    ro, col = _csr(g)
    rro = np.ascontiguousarray(rrow_off, dtype=np.int32)
    rc = np.ascontiguousarray(rcol, dtype=np.int32)
    live = np.empty(g.n, np.uint8)
    level = np.empty(g.n, np.int32)
    st = np.zeros(3, np.int64)
    if lib().or_ac3_jacobi2(g.n, ro, col, rro, rc, live, level, st) < 0:
        raise MemoryError("oracle ac3_jacobi2: allocation failed")
    return Ac3Two(live, level, int(st[0]), int(st[1]), int(st[2]))


def counts3two(g, rrow_off, rcol, res: PeelResult):
    """Closed-form (total, rounds) of the two-sided AC-3 rounds from the
    two-sided peeling result ``res`` (:func:`peel2`)."""
    ro, col = _csr(g)
    rro = np.ascontiguousarray(rrow_off, dtype=np.int32)
    rc = np.ascontiguousarray(rcol, dtype=np.int32)
    out = np.zeros(2, np.int64)
    r = lib().or_counts3two(g.n, ro, col, rro, rc, np.ascontiguousarray(res.live, np.uint8),
                            np.ascontiguousarray(res.level, np.int32), out)
    if r != 0:
        raise ValueError(f"oracle counts3two: vertex {-r - 1} inconsistent with the levels")
    return int(out[0]), int(out[1])


def counts(g, res: PeelResult, preset=None) -> Counts:
    """Closed-form traversed-edge totals for the given (oracle) result; pass the
    same ``preset`` as to :func:`peel`."""
    ro, col = _csr(g)
    out = np.zeros(8, np.int64)
    if preset is not None:
        rc = lib().or_counts_preset(g.n, ro, col, _preset(g, preset), res.live, res.level,
                                    res.alpha, out)
    else:
        rc = lib().or_counts(g.n, ro, col, res.live, res.level, res.alpha, out)
    if rc != 0:
        raise ValueError(f"oracle counts: live vertex {-rc - 1} has no live successor")
    return Counts(*[int(x) for x in out])


def ac6_seq(g):
    """(live, traversed_edges, |Q| high-water) of the sequential AC-6 algorithm."""
    ro, col = _csr(g)
    live = np.empty(g.n, np.uint8)
    st = np.zeros(3, np.int64)
    if lib().or_ac6_seq(g.n, ro, col, live, st) < 0:
        raise MemoryError("oracle ac6: allocation failed")
    return live, int(st[0]), int(st[2])


def ac3(g, jacobi: bool = True):
    """(live, traversed_edges, rounds) of the AC-3-based algorithm with cursor."""
    ro, col = _csr(g)
    live = np.empty(g.n, np.uint8)
    st = np.zeros(3, np.int64)
    f = lib().or_ac3_jacobi if jacobi else lib().or_ac3_inplace
    if f(g.n, ro, col, live, st) < 0:
        raise MemoryError("oracle ac3: allocation failed")
    return live, int(st[0]), int(st[1])


@dataclass
class Deferred:
    live: np.ndarray      # uint8[n], 1 = LIVE
    edges: int            # traversed edges, cursor re-checks included
    rounds: int           # rounds run (the last one registers supports unless the
                          # fixed point came first)
    rechecks: int         # cursor re-checks of rounds 2..


def ac6_deferred(g, rounds: int) -> Deferred:
    """AC-3 rounds with cursor for up to ``rounds - 1`` repetitions, then AC-6
    from the vertices still live, run literally (oracle.c or_ac6_deferred)."""
    ro, col = _csr(g)
    live = np.empty(g.n, np.uint8)
    st = np.zeros(4, np.int64)
    if lib().or_ac6_deferred(g.n, ro, col, int(rounds), live, st) < 0:
        raise MemoryError("oracle ac6_deferred: allocation failed")
    return Deferred(live, int(st[0]), int(st[1]), int(st[3]))


def counts_deferred(g, res: PeelResult, rounds: int):
    """(total, rounds, rechecks) of :func:`ac6_deferred` in closed form from the
    peeling levels (rounds >= 2)."""
    ro, col = _csr(g)
    out = np.zeros(3, np.int64)
    rc = lib().or_counts_deferred(g.n, ro, col, res.live, res.level, res.alpha, int(rounds),
                                  out)
    if rc != 0:
        raise ValueError(f"oracle counts: live vertex {-rc - 1} has no live successor")
    return int(out[0]), int(out[1]), int(out[2])


def bitmap(live: np.ndarray) -> np.ndarray:
    """LIVE bitmap: bit (v % 32) of uint32 word v // 32 is set iff v is LIVE."""
    n = live.shape[0]
    words = (n + 31) // 32
    bits = np.zeros(words * 32, np.uint8)
    bits[:n] = live != 0
    return np.packbits(bits, bitorder="little").view(np.uint32).copy()


def fin64(z: int) -> int:
    """The oracle's SplitMix64 finalizer."""
    return int(lib().or_fin64(z & ((1 << 64) - 1)))


def implicit_deg(imp, v: int) -> int:
    return int(lib().or_implicit_deg(imp.seed, imp.zero_thr, imp.table, v))


def implicit_nbr(imp, v: int, i: int) -> int:
    return int(lib().or_implicit_nbr(imp.seed, imp.log2n, v, i))


def implicit_csr(imp):
    """(row_off, col) of the implicit graph, generated by the oracle's own hash."""
    n = 1 << imp.log2n
    ro = np.zeros(n + 1, np.int32)
    m = lib().or_implicit_csr(imp.log2n, imp.seed, imp.zero_thr, imp.table, ro, None)
    if m >= 2 ** 31:
        raise ValueError("implicit graph too large for int32 CSR")
    col = np.empty(m, np.int32)
    lib().or_implicit_csr(imp.log2n, imp.seed, imp.zero_thr, imp.table, ro,
                          col.ctypes.data_as(ctypes.c_void_p))
    return ro, col


def batch_peel(b, nthreads: int = 0):
    """(live uint8[sum n], n_live int64[G], alpha int64[G]) of every graph in a
    packed batch, one graph per thread."""
    G = b.G
    live = np.empty(int(b.vbase[-1]), np.uint8)
    out = np.zeros(2 * G, np.int64)
    if lib().or_batch_peel(G, np.ascontiguousarray(b.vbase, np.int64),
                           np.ascontiguousarray(b.row_off, np.int32),
                           np.ascontiguousarray(b.col, np.int32), live, out, nthreads) != 0:
        raise MemoryError("oracle batch: allocation failed")
    return live, out[:G].copy(), out[G:].copy()
