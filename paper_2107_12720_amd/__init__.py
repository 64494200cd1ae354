"""Python binding of libtrim: parallel graph trimming on MI355X (gfx950).

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``libtrim.so`` (built from ``csrc/`` by ``build.py``); PyTorch is
used only for device memory and streams.  There is no fallback: if the
library is missing or no GPU is present, calls raise :class:`TrimError`.

The functions mirror the C ABI in ``include/trim.h``:

* :meth:`Context.trim_csr`      -- AC-6 / AC-4 / AC-3 on an explicit CSR graph;
* :meth:`Context.trim_implicit` -- AC-6 / AC-3 on the hash-generated graph;
* :meth:`Context.trim_batch`    -- AC-6 on many packed graphs in one launch
  sequence (optionally replayed from a captured HIP graph);
* :meth:`Context.num_workers`   -- the worker count P (size of worker_edges).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrim.so")

AC3, AC4, AC6 = 3, 4, 6
ALGOS = {"ac3": AC3, "ac4": AC4, "ac6": AC6}
STATUS = {0: "TRIM_OK", -1: "TRIM_E_INVAL", -2: "TRIM_E_NOMEM", -3: "TRIM_E_HIP",
          -4: "TRIM_E_UNSUPPORTED", -5: "TRIM_E_BADGRAPH", -6: "TRIM_E_STALLED"}
EXPORTS = ("trim_version", "trim_last_error", "trim_ctx_create", "trim_ctx_destroy",
           "trim_ctx_mem_used", "trim_ctx_status", "trim_max_workers",
           "trim_num_workers", "trim_csr", "trim_csr_preset", "trim_csr_two_sided",
           "trim_scc", "trim_size2", "trim_implicit", "trim_batch",
           "trim_ctx_set_timing", "trim_ctx_kernel_times", "trim_mlp_prepare", "trim_mlp_grad",
           "trim_mlp_adam", "trim_mlp_score", "trim_edge_keys", "trim_order_by_key",
           "trim_csr_noalloc")
MLP_PARAMS = 1377
STATS_FIELDS = ("edges_total", "n_live", "n_dead", "rounds", "queued", "edges_sweep", "closes",
                "joins", "visited", "graph_edges", "q_highwater", "edges_live", "stalled",
                "forest", "jump_rounds", "work_items", "phases", "rechecks")
STATS_WORDS = 18
ABI_VERSION = 3
MAX_ROUNDS = 64
DEFAULT_BUDGET = 1 << 22


class TrimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("budget", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rounds", ctypes.c_int32)]


class CsrDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("row_off", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("rrow_off", ctypes.c_void_p), ("rcol", ctypes.c_void_p)]


class SccStats(ctypes.Structure):
    _fields_ = [("n_scc", ctypes.c_int64), ("trimmed", ctypes.c_int64), ("giant", ctypes.c_int64),
                ("trims", ctypes.c_int32), ("color_rounds", ctypes.c_int32),
                ("color_sweeps", ctypes.c_int32), ("search_levels", ctypes.c_int32),
                ("search_edges", ctypes.c_int64), ("search_ors", ctypes.c_int64),
                ("trim_ms", ctypes.c_double),
                ("search_ms", ctypes.c_double), ("color_ms", ctypes.c_double),
                ("paired", ctypes.c_int64), ("size2_ms", ctypes.c_double)]


class ImplicitDesc(ctypes.Structure):
    _fields_ = [("log2n", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("zero_thr", ctypes.c_uint64), ("deg_table", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libtrim.so (raises TrimError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TrimError(-3, f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.trim_version.restype = ctypes.c_int
        L.trim_last_error.restype = ctypes.c_char_p
        L.trim_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_uint64]
        L.trim_ctx_destroy.argtypes = [vp]
        L.trim_ctx_mem_used.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.trim_ctx_status.argtypes = [vp, vp]
        L.trim_max_workers.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32)]
        L.trim_num_workers.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Opts),
                                       ctypes.POINTER(i32)]
        L.trim_csr.argtypes = [vp, ctypes.c_int, ctypes.POINTER(CsrDesc), ctypes.POINTER(Opts),
                               vp, vp, vp, vp]
        L.trim_scc.argtypes = [vp, ctypes.POINTER(CsrDesc), ctypes.POINTER(Opts), vp,
                               ctypes.POINTER(SccStats), vp]
        L.trim_size2.argtypes = [vp, ctypes.POINTER(CsrDesc), vp, vp,
                                 ctypes.POINTER(ctypes.c_int64), vp]
        L.trim_csr_preset.argtypes = [vp, ctypes.c_int, ctypes.POINTER(CsrDesc), vp,
                                      ctypes.POINTER(Opts), vp, vp, vp, vp]
        L.trim_csr_two_sided.argtypes = [vp, ctypes.c_int, ctypes.POINTER(CsrDesc),
                                         ctypes.POINTER(Opts), vp, vp, vp, vp]
        L.trim_implicit.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ImplicitDesc),
                                    ctypes.POINTER(Opts), vp, vp, vp, vp]
        L.trim_batch.argtypes = [vp, i32, vp, vp, vp, ctypes.c_int64, ctypes.c_int64, vp,
                                 ctypes.POINTER(Opts), vp, vp, vp, vp]
        L.trim_ctx_set_timing.argtypes = [vp, ctypes.c_int]
        L.trim_ctx_kernel_times.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                            ctypes.POINTER(ctypes.c_float)]
        csr_p = ctypes.POINTER(CsrDesc)
        f32 = ctypes.c_float
        L.trim_mlp_prepare.argtypes = [vp, csr_p, vp, vp, vp]
        L.trim_mlp_grad.argtypes = [vp, csr_p, vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_uint64,
                                    i32, vp, vp]
        L.trim_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
        L.trim_mlp_score.argtypes = [vp, csr_p, vp, vp, vp, vp, vp]
        L.trim_edge_keys.argtypes = [vp, csr_p, i32, ctypes.c_uint64, vp, vp]
        L.trim_order_by_key.argtypes = [vp, csr_p, vp, f32, f32, vp, vp]
        L.trim_csr_noalloc.argtypes = [csr_p, ctypes.POINTER(Opts), vp, vp, vp, vp]
        for f in ("trim_ctx_create", "trim_ctx_destroy", "trim_ctx_mem_used", "trim_ctx_status",
                  "trim_max_workers", "trim_num_workers", "trim_csr",
                  "trim_csr_preset", "trim_csr_two_sided", "trim_scc", "trim_size2",
                  "trim_implicit", "trim_batch", "trim_ctx_set_timing", "trim_ctx_kernel_times",
                  "trim_mlp_prepare", "trim_mlp_grad", "trim_mlp_adam", "trim_mlp_score",
                  "trim_edge_keys", "trim_order_by_key", "trim_csr_noalloc"):
            getattr(L, f).restype = ctypes.c_int
        if L.trim_version() != ABI_VERSION:
            raise TrimError(-3, f"{LIB_PATH} has ABI {L.trim_version()}, expected "
                                f"{ABI_VERSION}; rebuild it")
        _lib = L
    return _lib


def last_error() -> str:
    return lib().trim_last_error().decode()


def _check(code: int):
    if code != 0:
        raise TrimError(code, last_error())


SCHED_REVERSE = 1
SCHED_JITTER = 2


FLAG_STEPWISE = 1
FLAG_BATCH_UNION = 2
FLAG_FOREST = 4


def make_opts(block=0, workers=0, chunk=0, validate=False, graph=False, schedule=0,
              budget=0, flags=0, rounds=0) -> Opts:
    return Opts(block, workers, chunk, int(bool(validate)), int(bool(graph)), int(schedule),
                int(budget), int(flags), int(rounds))


def _dev_ptr(t, dtype, name, allow_none=False):
    import torch
    if t is None:
        if allow_none:
            return None
        raise TrimError(-1, f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TrimError(-1, f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TrimError(-1, f"{name} must be a contiguous {dtype} tensor")
    return t.data_ptr()


def _stream_handle(stream, device):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class TrimResult:
    live_bitmap: "object"    # torch.int32 tensor of ceil(n/32) words (uint32 bit patterns)
    worker_edges: "object"   # torch.int64 tensor of P counts (or per-graph counts)
    stats: "object"          # torch.int64 tensor of STATS_WORDS words (trim_stats_t)

    def stats_dict(self) -> dict:
        s = self.stats.cpu().numpy().view(np.uint64)
        return {k: int(s[i]) for i, k in enumerate(STATS_FIELDS)}

    def bitmap_numpy(self) -> np.ndarray:
        return self.live_bitmap.cpu().numpy().view(np.uint32)


# Contexts still open at interpreter exit are destroyed by an exit hook, while
# the HIP runtime is certainly alive, instead of by __del__ during module
# teardown (whose order against the runtime's and a profiler's own teardown is
# not fixed).
_open_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_open_contexts():
    for c in list(_open_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A libtrim context bound to one GPU; owns the call's working memory.
    ``mem_budget`` caps the device memory it may hold (bytes, 0 = no cap)."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise TrimError(-3, "no GPU available; libtrim has no CPU path")
        self.device = device
        self._h = ctypes.c_void_p()
        _check(lib().trim_ctx_create(ctypes.byref(self._h), device, int(mem_budget)))
        _open_contexts.add(self)

    def close(self):
        if self._h:
            lib().trim_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()
        _open_contexts.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def mem_used(self) -> int:
        """Device memory the context holds (bytes)."""
        b = ctypes.c_uint64()
        _check(lib().trim_ctx_mem_used(self._h, ctypes.byref(b)))
        return int(b.value)

    def status(self, stream=None) -> int:
        """Wait for the stream; the watchdog status of the last trimming call
        (0, or -6 = TRIM_E_STALLED when it was abandoned)."""
        return int(lib().trim_ctx_status(self._h, _stream_handle(stream, self.device)))

    def check(self, stream=None):
        """As status(), raising TrimError when the last call did not finish."""
        _check(self.status(stream))

    def max_workers(self, algo: int = AC6) -> int:
        P = ctypes.c_int32()
        _check(lib().trim_max_workers(self._h, int(ALGOS.get(algo, algo)), ctypes.byref(P)))
        return P.value

    def set_timing(self, enable=True):
        """Record HIP events around each kernel of later calls (same stream).
        `enable`: False / 0 off, True / 1 the last call, k <= 64 the last k
        calls."""
        _check(lib().trim_ctx_set_timing(self._h, int(enable)))

    def kernel_times(self) -> list:
        """[(kernel name, ms)] of the kept calls, in call order; waits for the
        last of them to finish."""
        cap = 16 * 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_float * cap)()
        k = lib().trim_ctx_kernel_times(self._h, cap, names, ms)
        if k < 0:
            raise TrimError(k, last_error())
        return [(names[i].decode(), float(ms[i])) for i in range(k)]

    def num_workers(self, algo: int = AC6, opts: Opts | None = None) -> int:
        P = ctypes.c_int32()
        _check(lib().trim_num_workers(self._h, int(algo), ctypes.byref(opts or Opts()),
                                      ctypes.byref(P)))
        return P.value

    def _outputs(self, n_words, P, live_bitmap, worker_edges, stats):
        import torch
        dev = torch.device("cuda", self.device)
        if live_bitmap is None:
            live_bitmap = torch.empty(max(n_words, 1), dtype=torch.int32, device=dev)
        if worker_edges is None:
            worker_edges = torch.empty(max(P, 1), dtype=torch.int64, device=dev)
        if stats is None:
            stats = torch.empty(STATS_WORDS, dtype=torch.int64, device=dev)
        return live_bitmap, worker_edges, stats

    def trim_csr(self, algo, n, row_off, col, rrow_off=None, rcol=None, *, live_bitmap=None,
                 worker_edges=None, stats=None, opts: Opts | None = None,
                 stream=None) -> TrimResult:
        """Trim the CSR graph (row_off, col: int32 device tensors) with algo 3/4/6."""
        import torch
        algo = ALGOS.get(algo, algo)
        opts = opts or Opts()
        m = int(col.numel()) if col is not None else 0
        d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                    _dev_ptr(col, torch.int32, "col") if m else None,
                    _dev_ptr(rrow_off, torch.int32, "rrow_off", allow_none=True),
                    _dev_ptr(rcol, torch.int32, "rcol", allow_none=True) if m else None)
        P = self.num_workers(algo, opts)
        lb, we, st = self._outputs((int(n) + 31) // 32, P, live_bitmap, worker_edges, stats)
        _check(lib().trim_csr(self._h, int(algo), ctypes.byref(d), ctypes.byref(opts),
                              ctypes.c_void_p(lb.data_ptr()), ctypes.c_void_p(we.data_ptr()),
                              ctypes.c_void_p(st.data_ptr()), _stream_handle(stream, self.device)))
        return TrimResult(lb, we, st)

    def trim_scc(self, n, row_off, col, rrow_off, rcol, *, label=None,
                 opts: Opts | None = None, stream=None):
        """Strongly connected components by forward-backward search with
        trimming.  Returns (label int32 device tensor, stats dict); label[v] is
        the id of one vertex of v's component.  Synchronises the stream."""
        import torch
        opts = opts or Opts()
        m = int(col.numel()) if col is not None else 0
        d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                    _dev_ptr(col, torch.int32, "col") if m else None,
                    _dev_ptr(rrow_off, torch.int32, "rrow_off"),
                    _dev_ptr(rcol, torch.int32, "rcol") if m else None)
        if label is None:
            label = torch.empty(max(int(n), 1), dtype=torch.int32,
                                device=torch.device("cuda", self.device))
        st = SccStats()
        _check(lib().trim_scc(self._h, ctypes.byref(d), ctypes.byref(opts),
                              ctypes.c_void_p(label.data_ptr()), ctypes.byref(st),
                              _stream_handle(stream, self.device)))
        return label, {k: (float if t is ctypes.c_double else int)(getattr(st, k))
                       for k, t in SccStats._fields_}

    def trim_size2(self, n, row_off, col, rrow_off, rcol, preset_dead=None, *, partner=None,
                   stream=None):
        """Size-2 check: (partner int32 device tensor, number of paired
        vertices); partner[u] = v for a component {u, v} of two, else -1."""
        import torch
        m = int(col.numel()) if col is not None else 0
        d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                    _dev_ptr(col, torch.int32, "col") if m else None,
                    _dev_ptr(rrow_off, torch.int32, "rrow_off"),
                    _dev_ptr(rcol, torch.int32, "rcol") if m else None)
        pd = _dev_ptr(preset_dead, torch.int32, "preset_dead", allow_none=True)
        if partner is None:
            partner = torch.empty(max(int(n), 1), dtype=torch.int32,
                                  device=torch.device("cuda", self.device))
        np_ = ctypes.c_int64()
        _check(lib().trim_size2(self._h, ctypes.byref(d), pd, ctypes.c_void_p(partner.data_ptr()),
                                ctypes.byref(np_), _stream_handle(stream, self.device)))
        return partner, int(np_.value)

    def trim_csr_preset(self, algo, n, row_off, col, preset_dead, rrow_off=None, rcol=None, *,
                        live_bitmap=None, worker_edges=None, stats=None,
                        opts: Opts | None = None, stream=None) -> TrimResult:
        """Trim with the vertices set in ``preset_dead`` (int32 device bitmap of
        ceil(n/32) words) removed from the start; algo 3/4/6."""
        import torch
        algo = ALGOS.get(algo, algo)
        opts = opts or Opts()
        m = int(col.numel()) if col is not None else 0
        d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                    _dev_ptr(col, torch.int32, "col") if m else None,
                    _dev_ptr(rrow_off, torch.int32, "rrow_off", allow_none=True),
                    _dev_ptr(rcol, torch.int32, "rcol", allow_none=True) if m else None)
        pd = _dev_ptr(preset_dead, torch.int32, "preset_dead", allow_none=int(n) == 0)
        P = self.num_workers(algo, opts)
        lb, we, st = self._outputs((int(n) + 31) // 32, P, live_bitmap, worker_edges, stats)
        _check(lib().trim_csr_preset(self._h, int(algo), ctypes.byref(d), pd, ctypes.byref(opts),
                                     ctypes.c_void_p(lb.data_ptr()),
                                     ctypes.c_void_p(we.data_ptr()),
                                     ctypes.c_void_p(st.data_ptr()),
                                     _stream_handle(stream, self.device)))
        return TrimResult(lb, we, st)

    def trim_csr_two_sided(self, algo, n, row_off, col, rrow_off, rcol, *, live_bitmap=None,
                           worker_edges=None, stats=None, opts: Opts | None = None,
                           stream=None) -> TrimResult:
        """Two-sided trimming (a vertex needs a live successor and a live
        predecessor) of the CSR graph and its transpose, algo 3, 4 or 6."""
        import torch
        algo = ALGOS.get(algo, algo)
        opts = opts or Opts()
        m = int(col.numel()) if col is not None else 0
        d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                    _dev_ptr(col, torch.int32, "col") if m else None,
                    _dev_ptr(rrow_off, torch.int32, "rrow_off"),
                    _dev_ptr(rcol, torch.int32, "rcol") if m else None)
        P = self.num_workers(algo, opts) if algo in (AC3, AC4, AC6) else 1
        lb, we, st = self._outputs((int(n) + 31) // 32, P, live_bitmap, worker_edges, stats)
        _check(lib().trim_csr_two_sided(self._h, int(algo), ctypes.byref(d), ctypes.byref(opts),
                                        ctypes.c_void_p(lb.data_ptr()),
                                        ctypes.c_void_p(we.data_ptr()),
                                        ctypes.c_void_p(st.data_ptr()),
                                        _stream_handle(stream, self.device)))
        return TrimResult(lb, we, st)

    def trim_implicit(self, algo, log2n, seed, zero_thr, deg_table, *, live_bitmap=None,
                      worker_edges=None, stats=None, opts: Opts | None = None,
                      stream=None) -> TrimResult:
        """Trim the hash-generated graph G = (V, POST) with n = 2^log2n (algo 3 or 6)."""
        import torch
        algo = ALGOS.get(algo, algo)
        opts = opts or Opts()
        d = ImplicitDesc(int(log2n), int(seed) & (2 ** 64 - 1), int(zero_thr) & (2 ** 64 - 1),
                         _dev_ptr(deg_table, torch.int64, "deg_table"))
        P = self.num_workers(algo, opts) if algo in (AC3, AC6) else 1
        lb, we, st = self._outputs(((1 << int(log2n)) + 31) // 32, P, live_bitmap, worker_edges,
                                   stats)
        _check(lib().trim_implicit(self._h, int(algo), ctypes.byref(d), ctypes.byref(opts),
                                   ctypes.c_void_p(lb.data_ptr()), ctypes.c_void_p(we.data_ptr()),
                                   ctypes.c_void_p(st.data_ptr()),
                                   _stream_handle(stream, self.device)))
        return TrimResult(lb, we, st)

    def trim_batch(self, vbase, row_off, col, bitmap_base, total_n, total_m, *, live_bitmaps=None,
                   graph_edges=None, stats=None, opts: Opts | None = None,
                   stream=None) -> TrimResult:
        """AC-6 on the packed batch (vbase, bitmap_base: int64 device tensors of G+1)."""
        import torch
        opts = opts or Opts()
        G = int(vbase.numel()) - 1
        if live_bitmaps is None:
            raise TrimError(-1, "live_bitmaps must be preallocated (bitmap_base[G] words)")
        lb, ge, st = self._outputs(0, G, live_bitmaps, graph_edges, stats)
        _check(lib().trim_batch(self._h, G, _dev_ptr(vbase, torch.int64, "vbase"),
                                _dev_ptr(row_off, torch.int32, "row_off"),
                                _dev_ptr(col, torch.int32, "col") if total_m else None,
                                int(total_n), int(total_m),
                                _dev_ptr(bitmap_base, torch.int64, "bitmap_base"),
                                ctypes.byref(opts), ctypes.c_void_p(lb.data_ptr()),
                                ctypes.c_void_p(ge.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                                _stream_handle(stream, self.device)))
        return TrimResult(lb, ge, st)


NOALLOC_MAX_N = 1 << 20
NOALLOC_WORKERS = 512


def trim_csr_noalloc(n, row_off, col, *, live_bitmap=None, worker_edges=None, stats=None,
                     opts: Opts | None = None, stream=None, device: int = 0) -> TrimResult:
    """AC-6 through trim_csr_noalloc: no context, working memory in the
    library's fixed per-GPU array (n <= NOALLOC_MAX_N).  Outputs that are not
    given are allocated here by torch, before the call."""
    import torch
    opts = opts or Opts()
    m = int(col.numel()) if col is not None else 0
    d = CsrDesc(int(n), m, _dev_ptr(row_off, torch.int32, "row_off"),
                _dev_ptr(col, torch.int32, "col") if m else None, None, None)
    dev = torch.device("cuda", device)
    P = opts.workers if opts.workers > 0 else NOALLOC_WORKERS
    if live_bitmap is None:
        live_bitmap = torch.empty(max((int(n) + 31) // 32, 1), dtype=torch.int32, device=dev)
    if worker_edges is None:
        worker_edges = torch.empty(max(P, 1), dtype=torch.int64, device=dev)
    if stats is None:
        stats = torch.empty(STATS_WORDS, dtype=torch.int64, device=dev)
    with torch.cuda.device(device):
        _check(lib().trim_csr_noalloc(ctypes.byref(d), ctypes.byref(opts),
                                      ctypes.c_void_p(live_bitmap.data_ptr()),
                                      ctypes.c_void_p(worker_edges.data_ptr()),
                                      ctypes.c_void_p(stats.data_ptr()),
                                      _stream_handle(stream, device)))
    return TrimResult(live_bitmap, worker_edges, stats)


class DeviceGraph:
    """An explicit CSR graph resident on the GPU (int32 row_off and col)."""

    def __init__(self, n, row_off, col, rrow_off=None, rcol=None):
        self.n, self.row_off, self.col = int(n), row_off, col
        self.rrow_off, self.rcol = rrow_off, rcol
        self.m = int(col.numel()) if col is not None else 0

    def desc(self) -> CsrDesc:
        import torch
        return CsrDesc(self.n, self.m, _dev_ptr(self.row_off, torch.int32, "row_off"),
                       _dev_ptr(self.col, torch.int32, "col") if self.m else None,
                       _dev_ptr(self.rrow_off, torch.int32, "rrow_off", allow_none=True),
                       _dev_ptr(self.rcol, torch.int32, "rcol", allow_none=True)
                       if self.m else None)

    @staticmethod
    def upload(g, device: int = 0) -> "DeviceGraph":
        return DeviceGraph(g.n, to_device(g.row_off, device),
                           to_device(g.col, device) if g.m else None)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _mlp_methods():
    def mlp_prepare(self, dg: DeviceGraph, indeg, src, stream=None):
        d = dg.desc()
        _check(lib().trim_mlp_prepare(self._h, ctypes.byref(d), _ptr(indeg), _ptr(src),
                                      _stream_handle(stream, self.device)))

    def mlp_grad(self, dg: DeviceGraph, indeg, src, live_bitmap, params_bf16, grad, count,
                 edge_ids=None, seed=0, step=0, stream=None):
        d = dg.desc()
        _check(lib().trim_mlp_grad(self._h, ctypes.byref(d), _ptr(indeg), _ptr(src),
                                   _ptr(live_bitmap), _ptr(params_bf16), _ptr(edge_ids),
                                   int(count), int(seed) & (2 ** 64 - 1), int(step), _ptr(grad),
                                   _stream_handle(stream, self.device)))

    def mlp_adam(self, params, params_bf16, m1, m2, grad, lr, step, beta1=0.9, beta2=0.999,
                 eps=1e-8, stream=None):
        _check(lib().trim_mlp_adam(self._h, _ptr(params), _ptr(params_bf16), _ptr(m1), _ptr(m2),
                                   _ptr(grad), float(lr), float(beta1), float(beta2), float(eps),
                                   int(step), _stream_handle(stream, self.device)))

    def mlp_score(self, dg: DeviceGraph, indeg, src, params_bf16, scores, stream=None):
        d = dg.desc()
        _check(lib().trim_mlp_score(self._h, ctypes.byref(d), _ptr(indeg), _ptr(src),
                                    _ptr(params_bf16), _ptr(scores),
                                    _stream_handle(stream, self.device)))

    def edge_keys(self, dg: DeviceGraph, kind, keys, seed=0, stream=None):
        d = dg.desc()
        _check(lib().trim_edge_keys(self._h, ctypes.byref(d), int(kind),
                                    int(seed) & (2 ** 64 - 1), _ptr(keys),
                                    _stream_handle(stream, self.device)))

    def order_by_key(self, dg: DeviceGraph, keys, lo, hi, col_out, stream=None):
        d = dg.desc()
        _check(lib().trim_order_by_key(self._h, ctypes.byref(d), _ptr(keys), float(lo), float(hi),
                                       _ptr(col_out), _stream_handle(stream, self.device)))

    for f in (mlp_prepare, mlp_grad, mlp_adam, mlp_score, edge_keys, order_by_key):
        setattr(Context, f.__name__, f)


_mlp_methods()


def to_device(a: np.ndarray, device: int = 0):
    """numpy array -> contiguous device tensor (int32/int64 views kept)."""
    import torch
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", device))
