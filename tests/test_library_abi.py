"""The HIP library loads on the CPU and exports every entry point that
include/burr.h declares (no compute calls: there may be no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "burr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(burr_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_2411_12365_amd as burr
    lib = burr.lib()
    names = declared()
    assert "burr_build" in names and "burr_query" in names
    for name in names:
        assert hasattr(lib, name), name


def test_default_params_and_error_strings():
    import paper_2411_12365_amd as burr
    lib = burr.lib()
    p = burr._CParams()
    lib.burr_default_params(ctypes.byref(p))
    assert (p.abi_version, p.bucket, p.load_num, p.load_den, p.layers, p.t_lo, p.t_hi) == \
        (2, 64, 97, 100, 3, 16, 32)
    assert lib.burr_error_string(burr.BURR_E_UNSOLVABLE).startswith(b"final layer")


def test_invalid_arguments_fail_without_touching_the_device():
    import paper_2411_12365_amd as burr
    lib = burr.lib()
    p = burr.Params(bucket=128).c(None)
    assert lib.burr_build(None, None, 10, 8, ctypes.byref(p)) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    p = burr.Params().c(None)
    assert lib.burr_build(None, None, 10, 0, ctypes.byref(p)) is None
    assert lib.burr_import(b"not an export", 13, None) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    for bad in (dict(threshold_mode=2), dict(cut_strategy=4)):
        p = burr.Params(**bad).c(None)
        assert lib.burr_build(None, None, 0, 8, ctypes.byref(p)) is None
        assert lib.burr_last_error() == burr.BURR_E_INVALID


def test_invalid_batch_arguments_fail_without_touching_the_device():
    import numpy as np
    import paper_2411_12365_amd as burr
    lib = burr.lib()
    p = burr.Params().c(None)
    off = np.array([0, 5, 3], dtype=np.uint64)      # decreasing
    rs = np.array([8, 8], dtype=np.uint32)
    fake = ctypes.c_void_p(0x1000)                  # never dereferenced
    assert lib.burr_build_batch(fake, fake, off.ctypes.data, rs.ctypes.data, 2,
                                ctypes.byref(p)) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    off = np.array([0, 3, 5], dtype=np.uint64)
    rs0 = np.array([8, 0], dtype=np.uint32)         # r = 0
    assert lib.burr_build_batch(fake, fake, off.ctypes.data, rs0.ctypes.data, 2,
                                ctypes.byref(p)) is None
    assert lib.burr_build_batch(fake, fake, off.ctypes.data, rs.ctypes.data, 0,
                                ctypes.byref(p)) is None
    off1 = np.array([1, 3, 5], dtype=np.uint64)     # does not start at 0
    assert lib.burr_build_batch(fake, fake, off1.ctypes.data, rs.ctypes.data, 2,
                                ctypes.byref(p)) is None
    assert lib.burr_build_batch(None, fake, off.ctypes.data, rs.ctypes.data, 2,
                                ctypes.byref(p)) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    assert lib.burr_batch_size(None) == 0
    assert lib.burr_batch_member(None, 0) is None


def test_invalid_tuning_arguments_fail_without_touching_the_device():
    import numpy as np
    import paper_2411_12365_amd as burr
    lib = burr.lib()
    p = burr.Params().c(None)
    off = np.array([0, 3, 5], dtype=np.uint64)
    rs = np.array([8, 8], dtype=np.uint32)
    fake = ctypes.c_void_p(0x1000)                  # never dereferenced
    for table in ([], [dict(n_max=100, minbpt=0)],                    # empty, zero minbpt
                  [dict(n_max=100, minbpt=4), dict(n_max=100, minbpt=8)]):  # not ascending
        arr = burr._tune_array(table) if table else None
        assert lib.burr_build_batch_tuned(fake, fake, off.ctypes.data, rs.ctypes.data, 2,
                                          ctypes.byref(p), arr, len(table)) is None
        assert lib.burr_last_error() == burr.BURR_E_INVALID
    # a valid table does not excuse invalid offsets
    arr = burr._tune_array([dict(n_max=100, minbpt=4)])
    bad = np.array([0, 5, 3], dtype=np.uint64)
    assert lib.burr_build_batch_tuned(fake, fake, bad.ctypes.data, rs.ctypes.data, 2,
                                      ctypes.byref(p), arr, 1) is None
    out = (burr._CTuneEntry * 2)()
    nm = np.array([1000, 500], dtype=np.uint64)     # not ascending
    cand = np.array([4, 16], dtype=np.uint32)
    assert lib.burr_autotune(ctypes.byref(p), 8, None, 0, nm.ctypes.data, 2, cand.ctypes.data,
                             2, 10_000, 1, out) == burr.BURR_E_INVALID
    nm = np.array([500, 1000], dtype=np.uint64)
    zero = np.array([4, 0], dtype=np.uint32)
    assert lib.burr_autotune(ctypes.byref(p), 8, None, 0, nm.ctypes.data, 2, zero.ctypes.data,
                             2, 10_000, 1, out) == burr.BURR_E_INVALID
    assert lib.burr_autotune(ctypes.byref(p), 0, None, 0, nm.ctypes.data, 2, cand.ctypes.data,
                             2, 10_000, 1, out) == burr.BURR_E_INVALID
    sizes = np.array([100, 200], dtype=np.uint64)  # a size sample of length 0
    assert lib.burr_autotune(ctypes.byref(p), 8, sizes.ctypes.data, 0, nm.ctypes.data, 2,
                             cand.ctypes.data, 2, 0, 1, out) == burr.BURR_E_INVALID


def test_python_binding_fails_loudly_without_library(monkeypatch):
    import paper_2411_12365_amd as burr
    monkeypatch.setattr(burr, "_lib", None)
    monkeypatch.setattr(burr, "LIB_PATH", "/nonexistent/libburr.so")
    try:
        burr.lib()
    except RuntimeError as e:
        assert "missing" in str(e)
    else:
        raise AssertionError("expected a failure")
