"""The C-ABI library loads and exports every declared symbol; argument errors
are reported without a GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "trim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trim_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_calls():
    import paper_2107_12720_amd as T
    assert declared_functions() == sorted(T.EXPORTS)


def test_library_exports_every_declared_symbol():
    import paper_2107_12720_amd as T
    L = T.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.trim_version() == T.ABI_VERSION == 3


def test_null_arguments_rejected():
    import paper_2107_12720_amd as T
    L = T.lib()
    assert L.trim_csr(None, 6, None, None, None, None, None, None) == -1
    assert "NULL" in T.last_error()
    assert L.trim_ctx_create(None, 0, 0) == -1
    assert L.trim_ctx_status(None, None) == -1
    assert L.trim_max_workers(None, 6, ctypes.byref(ctypes.c_int32())) == -1
    assert L.trim_ctx_mem_used(None, ctypes.byref(ctypes.c_uint64())) == -1
    P = ctypes.c_int32()
    assert L.trim_num_workers(None, 6, None, ctypes.byref(P)) == -1
    assert L.trim_batch(None, 1, None, None, None, 0, 0, None, None, None, None, None, None) == -1
    assert L.trim_csr_two_sided(None, 6, None, None, None, None, None, None) == -1
    assert "NULL" in T.last_error()
    assert L.trim_csr_preset(None, 6, None, None, None, None, None, None, None) == -1
    assert L.trim_scc(None, None, None, None, None, None) == -1
    assert L.trim_size2(None, None, None, None, None, None) == -1
    assert "NULL" in T.last_error()
    assert L.trim_ctx_destroy(None) == 0


def test_no_gpu_context_fails_cleanly():
    import torch
    import paper_2107_12720_amd as T
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = T.lib().trim_ctx_create(ctypes.byref(h), 0, 0)
    assert rc in (-1, -3) and not h.value
    with pytest.raises(T.TrimError):
        T.Context(0)


def test_opts_layout_matches_header():
    import paper_2107_12720_amd as T
    assert ctypes.sizeof(T.Opts) == 36
    assert [f for f, _ in T.Opts._fields_] == ["block", "workers", "chunk", "validate", "graph",
                                               "schedule", "budget", "flags", "rounds"]
    # trim_stats_t: the header's uint64 words, the named fields first, in order
    text = open(os.path.join(ROOT, "include", "trim.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} trim_stats_t;", text).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"uint64_t\s+(\w+)(?:\[(\d+)\])?;", body)
    assert sum(int(k or 1) for _, k in fields) == T.STATS_WORDS == 18
    assert tuple(f for f, _ in fields) == T.STATS_FIELDS
    assert ctypes.sizeof(T.CsrDesc) == 48
    assert ctypes.sizeof(T.ImplicitDesc) == 32


def test_noalloc_refuses_late_registration_before_any_gpu_call():
    """trim_csr_noalloc takes opts.rounds 0 or 1 only; the refusal comes from
    the argument checks, before the device is touched (host stand-ins for the
    pointers are never dereferenced)."""
    import paper_2107_12720_amd as T
    L = T.lib()
    dummy = (ctypes.c_int32 * 4)()
    g = T.CsrDesc(1, 0, ctypes.cast(dummy, ctypes.c_void_p), None, None, None)
    o = T.make_opts(rounds=2)
    rc = L.trim_csr_noalloc(ctypes.byref(g), ctypes.byref(o), ctypes.cast(dummy, ctypes.c_void_p),
                            ctypes.cast(dummy, ctypes.c_void_p), None, None)
    assert rc == -1 and "rounds" in T.last_error()
    o = T.make_opts(rounds=T.MAX_ROUNDS + 1)
    rc = L.trim_csr_noalloc(ctypes.byref(g), ctypes.byref(o), ctypes.cast(dummy, ctypes.c_void_p),
                            ctypes.cast(dummy, ctypes.c_void_p), None, None)
    assert rc == -1 and "rounds" in T.last_error()

