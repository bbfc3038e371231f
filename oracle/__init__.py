"""ctypes wrapper of the CPU oracle (``burr_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check the HIP library. The product package never
imports this module.

The oracle is plain sequential C written from the paper's definitions
(arXiv 2411.12365, Sec. 2 and Sec. 3); see the comments in burr_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "burr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libburr_oracle.so")

OK = 0
E_INVALID = -1
E_NOMEM = -2
E_UNSOLVABLE = -3


def compile_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libburr_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("bucket", ctypes.c_uint32),
        ("load_num", ctypes.c_uint32),
        ("load_den", ctypes.c_uint32),
        ("final_num", ctypes.c_uint32),
        ("final_den", ctypes.c_uint32),
        ("layers", ctypes.c_uint32),
        ("t_lo", ctypes.c_uint32),
        ("t_hi", ctypes.c_uint32),
        ("ranges", ctypes.c_uint32),
        ("minbpt", ctypes.c_uint32),
        ("final_attempts", ctypes.c_uint32),
        ("filter_mode", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("threshold_mode", ctypes.c_uint32),
        ("cut_strategy", ctypes.c_uint32),
        ("cut_search", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
    ]


class _LayerInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("n", "m", "nbuckets", "nranges", "bumped", "forced", "pivots",
                 "redundant", "steps")]


class _FinalInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("n", "m", "attempt", "steps")]


@dataclass
class Params:
    """Construction parameters (same meaning as the library's burr_params)."""
    bucket: int = 64
    load_num: int = 97
    load_den: int = 100
    final_num: int = 110
    final_den: int = 100
    layers: int = 3
    t_lo: int = 16
    t_hi: int = 32
    ranges: int = 1
    minbpt: int = 16
    final_attempts: int = 16
    filter_mode: int = 0
    seed: int = 0
    threshold_mode: int = 0   # 0: 2-bit, 1: 1+-bit thresholds
    cut_strategy: int = 0     # 0: equal split, 1 minbump, 2 maxprev, 3 diff
    cut_search: int = 0       # buckets searched around each equal-split cut

    def _c(self) -> _Params:
        return _Params(**asdict(self), pad=0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            compile_oracle(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.ref_fmix64.restype = u64
        L.ref_fmix64.argtypes = [u64]
        L.ref_fastrange.restype = u64
        L.ref_fastrange.argtypes = [u64, u64]
        L.ref_hash.restype = None
        L.ref_hash.argtypes = [u64, u32, u64, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.ref_fingerprint.restype = u32
        L.ref_fingerprint.argtypes = [u64, u32, u64]
        L.ref_build.restype = ctypes.c_int
        L.ref_build.argtypes = [vp, vp, u64, u32, ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        L.ref_free.restype = None
        L.ref_free.argtypes = [vp]
        L.ref_query.restype = ctypes.c_int
        L.ref_query.argtypes = [vp, vp, u64, vp]
        L.ref_export.restype = ctypes.c_int
        L.ref_export.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
        L.ref_layers_built.restype = u32
        L.ref_layers_built.argtypes = [vp]
        L.ref_get_layer_info.restype = ctypes.c_int
        L.ref_get_layer_info.argtypes = [vp, u32, ctypes.POINTER(_LayerInfo)]
        L.ref_get_final_info.restype = ctypes.c_int
        L.ref_get_final_info.argtypes = [vp, ctypes.POINTER(_FinalInfo)]
        L.ref_build_mt.restype = ctypes.c_int
        L.ref_build_mt.argtypes = [vp, vp, u64, u32, ctypes.POINTER(_Params), u32,
                                   ctypes.POINTER(vp)]
        L.ref_build_from.restype = ctypes.c_int
        L.ref_build_from.argtypes = [vp, vp, u64, u32, ctypes.POINTER(_Params), u32, u32,
                                     ctypes.POINTER(vp)]
        L.ref_layer_cuts.restype = u64
        L.ref_layer_cuts.argtypes = [vp, u32, vp, u64]
        for fn in ("ref_layer_keys", "ref_layer_codes", "ref_layer_solution"):
            getattr(L, fn).restype = u64
            getattr(L, fn).argtypes = [vp, u32, vp, u64]
        p64 = ctypes.POINTER(u64)
        L.ref_layer_geometry.restype = None
        L.ref_layer_geometry.argtypes = [ctypes.POINTER(_Params), u64, p64, p64, p64]
        L.ref_range_buckets.restype = None
        L.ref_range_buckets.argtypes = [u64, u64, u64, p64, p64]
        L.ref_start_buckets.restype = None
        L.ref_start_buckets.argtypes = [vp, u64, u32, u64, u64, u32, vp]
        L.ref_layer_range.restype = ctypes.c_int
        L.ref_layer_range.argtypes = [ctypes.POINTER(_Params), u32, u32, u64, u64, vp, vp, u64,
                                      vp, vp, vp, p64]
        _lib = L
    return _lib


def value_dtype(r: int):
    return np.uint8 if r <= 8 else (np.uint16 if r <= 16 else np.uint32)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


class RefBurr:
    """A structure built by the oracle."""

    def __init__(self, handle: int, r: int, params: Params, n: int):
        self._h = ctypes.c_void_p(handle)
        self.r = r
        self.params = params
        self.n = n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ref_free(h)
            self._h = None

    @property
    def layers_built(self) -> int:
        return int(lib().ref_layers_built(self._h))

    def query(self, keys: np.ndarray) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(len(keys), dtype=value_dtype(self.r))
        rc = lib().ref_query(self._h, keys.ctypes.data, len(keys), out.ctypes.data)
        if rc != OK:
            raise OracleError(rc)
        return out

    def export(self) -> bytes:
        need = ctypes.c_uint64(0)
        lib().ref_export(self._h, None, 0, ctypes.byref(need))
        buf = (ctypes.c_uint8 * need.value)()
        rc = lib().ref_export(self._h, buf, need.value, ctypes.byref(need))
        if rc != OK:
            raise OracleError(rc)
        return bytes(buf)

    def layer_info(self, layer: int) -> dict:
        info = _LayerInfo()
        rc = lib().ref_get_layer_info(self._h, layer, ctypes.byref(info))
        if rc != OK:
            raise OracleError(rc)
        return {f: int(getattr(info, f)) for f, _ in _LayerInfo._fields_}

    def final_info(self) -> dict:
        info = _FinalInfo()
        lib().ref_get_final_info(self._h, ctypes.byref(info))
        return {f: int(getattr(info, f)) for f, _ in _FinalInfo._fields_}

    def layer_keys(self, layer: int) -> np.ndarray:
        n = lib().ref_layer_keys(self._h, layer, None, 0)
        out = np.zeros(n, dtype=np.uint64)
        lib().ref_layer_keys(self._h, layer, out.ctypes.data, n)
        return out

    def layer_codes(self, layer: int) -> np.ndarray:
        n = lib().ref_layer_codes(self._h, layer, None, 0)
        out = np.zeros(n, dtype=np.uint8)
        lib().ref_layer_codes(self._h, layer, out.ctypes.data, n)
        return out

    def layer_cuts(self, layer: int) -> np.ndarray:
        n = lib().ref_layer_cuts(self._h, layer, None, 0)
        out = np.zeros(n, dtype=np.uint64)
        lib().ref_layer_cuts(self._h, layer, out.ctypes.data, n)
        return out

    def layer_solution(self, layer: int) -> np.ndarray:
        n = lib().ref_layer_solution(self._h, layer, None, 0)
        out = np.zeros(n, dtype=np.uint32)
        lib().ref_layer_solution(self._h, layer, out.ctypes.data, n)
        return out


def build(keys: np.ndarray, values: np.ndarray | None, r: int,
          params: Params | None = None, threads: int = 1,
          first_layer: int = 0) -> RefBurr:
    """Build with the oracle. threads > 1 (or 0: every CPU) uses the
    range-parallel driver, which gives the same structure; first_layer > 0
    builds only the layers from that one on, from keys that enter it.
    Raises OracleError on failure."""
    params = params or Params()
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vptr = None
    if values is not None:
        values = np.ascontiguousarray(values, dtype=value_dtype(r))
        vptr = values.ctypes.data
    h = ctypes.c_void_p(0)
    cp = params._c()
    kptr = keys.ctypes.data if len(keys) else None
    if first_layer:
        rc = lib().ref_build_from(kptr, vptr, len(keys), r, ctypes.byref(cp), first_layer,
                                  threads if threads else os.cpu_count(), ctypes.byref(h))
    elif threads == 1:
        rc = lib().ref_build(kptr, vptr, len(keys), r, ctypes.byref(cp), ctypes.byref(h))
    else:
        rc = lib().ref_build_mt(kptr, vptr, len(keys), r, ctypes.byref(cp), threads,
                                ctypes.byref(h))
    if rc != OK:
        raise OracleError(rc)
    return RefBurr(h.value, r, params, len(keys))


def fmix64(x: int) -> int:
    return int(lib().ref_fmix64(x))


def fastrange(h: int, n: int) -> int:
    return int(lib().ref_fastrange(h, n))


def hash_key(key: int, layer: int, m: int, seed: int) -> tuple[int, int]:
    s = ctypes.c_uint64(0)
    c = ctypes.c_uint64(0)
    lib().ref_hash(key, layer, m, seed, ctypes.byref(s), ctypes.byref(c))
    return int(s.value), int(c.value)


def fingerprint(key: int, r: int, seed: int) -> int:
    return int(lib().ref_fingerprint(key, r, seed))


def layer_geometry(params: Params, nkeys: int) -> tuple[int, int, int]:
    """(slots m, buckets, ranges) of a BuRR layer entered by nkeys keys."""
    m, B, R = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    cp = params._c()
    lib().ref_layer_geometry(ctypes.byref(cp), nkeys, ctypes.byref(m), ctypes.byref(B),
                             ctypes.byref(R))
    return int(m.value), int(B.value), int(R.value)


def range_buckets(nbuckets: int, nranges: int, rho: int) -> tuple[int, int]:
    """Buckets [first, last) of range rho."""
    f, l = ctypes.c_uint64(0), ctypes.c_uint64(0)
    lib().ref_range_buckets(nbuckets, nranges, rho, ctypes.byref(f), ctypes.byref(l))
    return int(f.value), int(l.value)


def start_buckets(keys: np.ndarray, layer: int, m: int, params: Params) -> np.ndarray:
    """Start bucket of every key in layer `layer` of m slots (u32)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty(len(keys), dtype=np.uint32)
    if len(keys):
        lib().ref_start_buckets(keys.ctypes.data, len(keys), layer, m, params.seed,
                                params.bucket, out.ctypes.data)
    return out


def layer_range(keys: np.ndarray, values: np.ndarray | None, r: int, params: Params,
                layer: int, n_layer: int, rho: int) -> dict:
    """Range rho of layer `layer` (entered by n_layer keys) solved on its own
    from the keys that start in it: threshold codes per bucket, the range's
    column-interleaved solution words and its bumped keys."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    m, B, R = layer_geometry(params, n_layer)
    first, last = range_buckets(B, R, rho)
    codes = np.zeros(last - first, dtype=np.uint8)
    W = np.zeros((last - first) * params.bucket // 64 * r + 1, dtype=np.uint64)
    bumped = np.zeros(len(keys) + 1, dtype=np.uint64)
    nb = ctypes.c_uint64(0)
    vptr = None
    if values is not None:
        values = np.ascontiguousarray(values, dtype=value_dtype(r))
        vptr = values.ctypes.data
    cp = params._c()
    rc = lib().ref_layer_range(ctypes.byref(cp), r, layer, n_layer, rho,
                               keys.ctypes.data if len(keys) else None, vptr, len(keys),
                               codes.ctypes.data, W.ctypes.data, bumped.ctypes.data,
                               ctypes.byref(nb))
    if rc != OK:
        raise OracleError(rc)
    return {"first": first, "last": last, "codes": codes, "W": W[:-1],
            "bumped": bumped[:int(nb.value)]}
