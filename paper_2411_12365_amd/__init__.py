"""MI355X Bumped Ribbon Retrieval (BuRR) - Python binding of libburr.so.

Argument marshalling only: every step of construction and query runs in the
HIP kernels behind the C ABI declared in include/burr.h. Tensors must live
on the GPU; PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import asdict, dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libburr.so")

BURR_OK = 0
BURR_E_INVALID = -1
BURR_E_NOMEM = -2
BURR_E_UNSOLVABLE = -3
BURR_E_DEVICE = -4
BURR_E_BUDGET = -5
BURR_E_EVICTED = -6
BURR_SERVER_EVICT_LRU = 1
BURR_SERVER_NO_DEVICE = 2
BURR_REQ_BUILD = 1
BURR_REQ_QUERY = 2
BURR_FLAG_KEEP_LAYER_KEYS = 1
BURR_FLAG_NO_WORKSPACE_CACHE = 2
ABI_VERSION = 2
BURR_THRESH_2BIT = 0
BURR_THRESH_1PLUS = 1
BURR_CUT_EQUAL = 0
BURR_CUT_MINBUMP = 1
BURR_CUT_MAXPREV = 2
BURR_CUT_DIFF = 3

_EXPORTS = ("burr_default_params", "burr_build", "burr_query", "burr_contains", "burr_free",
            "burr_get_stats", "burr_export", "burr_import", "burr_debug_layer_keys",
            "burr_last_error", "burr_error_string", "burr_build_batch", "burr_batch_size",
            "burr_batch_member", "burr_batch_free", "burr_estimate_build_bytes",
            "burr_server_default_config", "burr_server_create", "burr_server_submit_build",
            "burr_server_submit_query", "burr_server_poll", "burr_server_drain",
            "burr_server_drop", "burr_server_handle", "burr_server_get_info",
            "burr_server_destroy", "burr_release_workspaces", "burr_build_batch_tuned",
            "burr_autotune", "burr_build_noalloc")


class BurrError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = _lib_error_string(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


class _CParams(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("bucket", ctypes.c_uint32),
        ("load_num", ctypes.c_uint32), ("load_den", ctypes.c_uint32),
        ("final_num", ctypes.c_uint32), ("final_den", ctypes.c_uint32),
        ("layers", ctypes.c_uint32), ("t_lo", ctypes.c_uint32), ("t_hi", ctypes.c_uint32),
        ("ranges", ctypes.c_uint32), ("minbpt", ctypes.c_uint32),
        ("final_attempts", ctypes.c_uint32), ("filter_mode", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p),
        ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("alloc_ctx", ctypes.c_void_p),
        ("threshold_mode", ctypes.c_uint32), ("cut_strategy", ctypes.c_uint32),
        ("cut_search", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


class _CLayerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("n", "m", "nbuckets", "nranges", "bumped",
                                                "steps")] + \
               [(f, ctypes.c_double) for f in ("ms_sort", "ms_solve", "ms_backsub", "ms_gather")]


class _CStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("r", ctypes.c_uint32), ("layers_built", ctypes.c_uint32),
        ("layer", _CLayerStats * 32), ("final_n", ctypes.c_uint64), ("final_m", ctypes.c_uint64),
        ("final_attempt", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
        ("ms_sort", ctypes.c_double), ("ms_solve", ctypes.c_double),
        ("ms_final", ctypes.c_double), ("ms_total", ctypes.c_double),
    ]


class _CTuneEntry(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_uint64), ("minbpt", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("ns_per_key", ctypes.c_double),
                ("bits_per_key", ctypes.c_double)]


class _CServerConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("workers", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("max_batch_keys", ctypes.c_uint64)]


class _CCompletion(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("struct_id", ctypes.c_uint64),
                ("kind", ctypes.c_uint32), ("status", ctypes.c_int32), ("n", ctypes.c_uint64),
                ("batch_id", ctypes.c_uint64), ("t_submit_ms", ctypes.c_double),
                ("t_start_ms", ctypes.c_double), ("t_end_ms", ctypes.c_double)]


class _CServerInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "resident_bytes", "inflight_bytes", "peak_bytes", "resident", "pending", "running",
        "completed", "evictions", "batches")]


@dataclass
class Params:
    """burr_params without the stream/allocator fields."""
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
    flags: int = 0
    seed: int = 0
    threshold_mode: int = 0   # BURR_THRESH_2BIT / BURR_THRESH_1PLUS
    cut_strategy: int = 0     # BURR_CUT_EQUAL / MINBUMP / MAXPREV / DIFF
    cut_search: int = 0       # buckets searched per cut

    def c(self, stream: int | None = None, allocator: "TorchAllocator | None" = None) -> _CParams:
        cp = _CParams(abi_version=ABI_VERSION, stream=stream, alloc=None, free=None,
                      alloc_ctx=None, **asdict(self))
        if allocator is not None:
            cp.alloc = ctypes.cast(allocator._alloc_cb, ctypes.c_void_p)
            cp.free = ctypes.cast(allocator._free_cb, ctypes.c_void_p)
        return cp


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator: passed
    as burr_params.alloc/free, every workspace buffer and table of a build
    then lives in torch-managed memory (stream-ordered on the build's stream)
    instead of the library's own hipMalloc cache or HIP's pool. Counts the
    bytes it has handed out and not yet taken back."""

    def __init__(self, device=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else \
            torch.device(device).index or 0
        self.live = {}          # pointer -> bytes
        self.allocations = 0    # calls that returned memory
        self.peak = 0

        def _alloc(nbytes, stream, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                         int(stream or 0))
            except Exception:  # reported by the library as BURR_E_NOMEM
                return None
            self.live[ptr] = int(nbytes)
            self.allocations += 1
            self.peak = max(self.peak, sum(self.live.values()))
            return ptr

        def _free(ptr, stream, ctx):
            if ptr:
                self.live.pop(ptr, None)
                torch.cuda.caching_allocator_delete(ptr)

        # kept referenced for as long as the allocator lives
        self._alloc_cb = _ALLOC_FN(_alloc)
        self._free_cb = _FREE_FN(_free)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())


_lib = None


def lib():
    """Load libburr.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                               "python paper_2411_12365_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.burr_default_params.argtypes = [ctypes.POINTER(_CParams)]
        L.burr_default_params.restype = None
        L.burr_build.argtypes = [vp, vp, u64, u32, ctypes.POINTER(_CParams)]
        L.burr_build.restype = vp
        L.burr_build_noalloc.argtypes = [vp, vp, u64, u32, ctypes.POINTER(_CParams), vp,
                                         ctypes.c_size_t]
        L.burr_build_noalloc.restype = vp
        L.burr_query.argtypes = [vp, vp, u64, vp, vp]
        L.burr_query.restype = i32
        L.burr_contains.argtypes = [vp, vp, u64, vp, vp]
        L.burr_contains.restype = i32
        L.burr_free.argtypes = [vp]
        L.burr_free.restype = None
        L.burr_get_stats.argtypes = [vp, ctypes.POINTER(_CStats)]
        L.burr_get_stats.restype = i32
        L.burr_export.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.burr_export.restype = i32
        L.burr_import.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(_CParams)]
        L.burr_import.restype = vp
        L.burr_debug_layer_keys.argtypes = [vp, u32, vp, u64]
        L.burr_debug_layer_keys.restype = ctypes.c_int64
        L.burr_build_batch.argtypes = [vp, vp, vp, vp, u32, ctypes.POINTER(_CParams)]
        L.burr_build_batch.restype = vp
        L.burr_build_batch_tuned.argtypes = [vp, vp, vp, vp, u32, ctypes.POINTER(_CParams),
                                             ctypes.POINTER(_CTuneEntry), u32]
        L.burr_build_batch_tuned.restype = vp
        L.burr_autotune.argtypes = [ctypes.POINTER(_CParams), u32, vp, u64, vp, u32, vp, u32,
                                    u64, u32, ctypes.POINTER(_CTuneEntry)]
        L.burr_autotune.restype = ctypes.c_int
        L.burr_batch_size.argtypes = [vp]
        L.burr_batch_size.restype = u32
        L.burr_batch_member.argtypes = [vp, u32]
        L.burr_batch_member.restype = vp
        L.burr_batch_free.argtypes = [vp]
        L.burr_batch_free.restype = None
        L.burr_estimate_build_bytes.argtypes = [u64, u32, ctypes.POINTER(_CParams),
                                                ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.burr_estimate_build_bytes.restype = i32
        L.burr_server_default_config.argtypes = [ctypes.POINTER(_CServerConfig)]
        L.burr_server_default_config.restype = None
        L.burr_server_create.argtypes = [ctypes.POINTER(_CServerConfig), ctypes.POINTER(_CParams)]
        L.burr_server_create.restype = vp
        L.burr_server_submit_build.argtypes = [vp, vp, vp, u64, u32, ctypes.POINTER(u64)]
        L.burr_server_submit_build.restype = i32
        L.burr_server_submit_query.argtypes = [vp, u64, vp, u64, vp, ctypes.POINTER(u64)]
        L.burr_server_submit_query.restype = i32
        L.burr_server_poll.argtypes = [vp, ctypes.POINTER(_CCompletion), u32,
                                       ctypes.POINTER(u32), ctypes.c_int64]
        L.burr_server_poll.restype = i32
        L.burr_server_drain.argtypes = [vp]
        L.burr_server_drain.restype = i32
        L.burr_server_drop.argtypes = [vp, u64]
        L.burr_server_drop.restype = i32
        L.burr_server_handle.argtypes = [vp, u64]
        L.burr_server_handle.restype = vp
        L.burr_server_get_info.argtypes = [vp, ctypes.POINTER(_CServerInfo)]
        L.burr_server_get_info.restype = i32
        L.burr_server_destroy.argtypes = [vp]
        L.burr_server_destroy.restype = None
        L.burr_release_workspaces.argtypes = []
        L.burr_release_workspaces.restype = None
        L.burr_last_error.argtypes = []
        L.burr_last_error.restype = i32
        L.burr_error_string.argtypes = [i32]
        L.burr_error_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _lib_error_string(code: int) -> str:
    try:
        return lib().burr_error_string(code).decode()
    except Exception:  # library missing: still report the code
        return "error"


def _stream_of(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check_tensor(t, name: str, dtypes):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")


def value_dtype(r: int):
    import torch
    return torch.uint8 if r <= 8 else (torch.uint16 if r <= 16 else torch.uint32)


class Handle:
    """A structure built on the GPU; owns its device memory until free().
    A batch member's handle owns nothing: it keeps its batch alive."""

    def __init__(self, ptr: int, r: int, params: Params, batch: "Batch | None" = None,
                 allocator: TorchAllocator | None = None):
        self._h = ptr
        self.r = r
        self.params = params
        self._batch = batch
        self._allocator = allocator  # frees through it, so it must outlive the handle

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None):
            if self._batch is None:
                lib().burr_free(self._h)
            self._h = None
            self._batch = None

    def query(self, keys, out=None, stream=None):
        return burr_query(self, keys, out, stream)

    def contains(self, keys, out=None, stream=None):
        return burr_contains(self, keys, out, stream)

    def export(self) -> bytes:
        return burr_export(self)

    def stats(self) -> dict:
        return burr_get_stats(self)

    def layer_keys(self, layer: int):
        return burr_debug_layer_keys(self, layer)


def burr_build(keys, values, r: int, params: Params | None = None, stream=None,
               allocator: TorchAllocator | None = None) -> Handle:
    """keys: int64/uint64 GPU tensor (bit pattern of u64 keys); values: GPU
    tensor of uint8/uint16/uint32 (by r) or None in filter mode. With an
    allocator (TorchAllocator), the build's device memory comes from PyTorch."""
    import torch
    params = params or Params()
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    vptr = None
    if values is not None:
        _check_tensor(values, "values", (value_dtype(r),))
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        vptr = values.data_ptr()
    cp = params.c(_stream_of(stream), allocator)
    h = lib().burr_build(keys.data_ptr() if keys.numel() else None, vptr, keys.numel(), r,
                         ctypes.byref(cp))
    if not h:
        raise BurrError(lib().burr_last_error(), "burr_build")
    return Handle(h, r, params, allocator=allocator)


def burr_build_noalloc(keys, values, r: int, table, params: Params | None = None,
                       stream=None) -> Handle:
    """burr_build without any device allocation by the library: temporary
    buffers come from its fixed scratch array, the tables go to `table` (a
    caller-owned uint8 GPU tensor, kept alive by the handle)."""
    import torch
    params = params or Params()
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    _check_tensor(table, "table", (torch.uint8,))
    vptr = None
    if values is not None:
        _check_tensor(values, "values", (value_dtype(r),))
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        vptr = values.data_ptr()
    cp = params.c(_stream_of(stream))
    h = lib().burr_build_noalloc(keys.data_ptr() if keys.numel() else None, vptr, keys.numel(),
                                 r, ctypes.byref(cp), table.data_ptr(), table.numel())
    if not h:
        raise BurrError(lib().burr_last_error(), "burr_build_noalloc")
    hd = Handle(h, r, params)
    hd._table = table
    return hd


class Batch:
    """Independent structures built together by burr_build_batch."""

    def __init__(self, ptr: int, rs, params: Params, allocator: TorchAllocator | None = None):
        self._b = ptr
        self.rs = rs
        self.params = params
        self._allocator = allocator

    def __del__(self):
        self.free()

    def __len__(self):
        return lib().burr_batch_size(self._b) if self._b else 0

    def member(self, i: int) -> Handle:
        return burr_batch_member(self, i)

    def free(self):
        if getattr(self, "_b", None):
            lib().burr_batch_free(self._b)
            self._b = None


def _batch_args(keys, values, offsets, rs):
    import numpy as np
    import torch
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    rr = np.ascontiguousarray(np.asarray(rs, dtype=np.uint32))
    if len(rr) == 0 or off.shape != (len(rr) + 1,):
        raise ValueError("offsets must hold len(rs)+1 entries")
    if int(off[-1]) != keys.numel():
        raise ValueError("offsets[-1] must equal the number of keys")
    vptr = None
    if values is not None:
        _check_tensor(values, "values", (value_dtype(int(rr.max())),))
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        vptr = values.data_ptr() if values.numel() else None
    return (keys.data_ptr() if keys.numel() else None), vptr, off, rr


def burr_build_batch(keys, values, offsets, rs, params: Params | None = None,
                     stream=None, allocator: TorchAllocator | None = None) -> Batch:
    """keys: GPU int64/uint64 tensor holding every structure's keys back to
    back; offsets: host sequence of len(rs)+1 key offsets (offsets[0] = 0);
    rs: value bits per structure; values: GPU tensor laid out like keys with
    the value dtype of max(rs), or None in filter mode."""
    params = params or Params()
    kptr, vptr, off, rr = _batch_args(keys, values, offsets, rs)
    cp = params.c(_stream_of(stream), allocator)
    b = lib().burr_build_batch(kptr, vptr, off.ctypes.data, rr.ctypes.data, len(rr),
                               ctypes.byref(cp))
    if not b:
        raise BurrError(lib().burr_last_error(), "burr_build_batch")
    return Batch(b, rr, params, allocator)


def _tune_array(table):
    arr = (_CTuneEntry * len(table))()
    for i, e in enumerate(table):
        arr[i].n_max = int(e["n_max"])
        arr[i].minbpt = int(e["minbpt"])
        arr[i].ns_per_key = float(e.get("ns_per_key", 0.0))
        arr[i].bits_per_key = float(e.get("bits_per_key", 0.0))
    return arr


def burr_build_batch_tuned(keys, values, offsets, rs, table, params: Params | None = None,
                           stream=None) -> Batch:
    """burr_build_batch with each structure's minimum buckets per range from
    the size class of `table` (a list of dicts with n_max and minbpt, as
    returned by burr_autotune) that holds its key count."""
    params = params or Params()
    kptr, vptr, off, rr = _batch_args(keys, values, offsets, rs)
    arr = _tune_array(table)
    cp = params.c(_stream_of(stream))
    b = lib().burr_build_batch_tuned(kptr, vptr, off.ctypes.data, rr.ctypes.data, len(rr),
                                     ctypes.byref(cp), arr, len(table))
    if not b:
        raise BurrError(lib().burr_last_error(), "burr_build_batch_tuned")
    return Batch(b, rr, params)


def burr_autotune(r: int, n_max, candidates, keys_per_trial: int = 0, reps: int = 2,
                  params: Params | None = None, stream=None, sizes=None) -> list[dict]:
    """Picks, per size class (upper bounds n_max, ascending), the minimum
    buckets per range among `candidates`: on whole batches of the structure
    sizes `sizes` (coordinate descent), or, without sizes, timing each class
    alone on batches of about keys_per_trial keys. Returns the table for
    burr_build_batch_tuned."""
    import numpy as np
    params = params or Params()
    nm = np.ascontiguousarray(np.asarray(n_max, dtype=np.uint64))
    cand = np.ascontiguousarray(np.asarray(candidates, dtype=np.uint32))
    sz = None if sizes is None else np.ascontiguousarray(np.asarray(sizes, dtype=np.uint64))
    out = (_CTuneEntry * max(len(nm), 1))()
    cp = params.c(_stream_of(stream))
    rc = lib().burr_autotune(ctypes.byref(cp), r, None if sz is None else sz.ctypes.data,
                             0 if sz is None else len(sz), nm.ctypes.data, len(nm),
                             cand.ctypes.data, len(cand), keys_per_trial, reps, out)
    if rc != BURR_OK:
        raise BurrError(rc, "burr_autotune")
    return [{f: getattr(out[i], f) for f in ("n_max", "minbpt", "ns_per_key", "bits_per_key")}
            for i in range(len(nm))]


def burr_batch_size(b: Batch) -> int:
    return len(b)


def burr_batch_member(b: Batch, i: int) -> Handle:
    h = lib().burr_batch_member(b._b, i)
    if not h:
        raise BurrError(lib().burr_last_error(), "burr_batch_member")
    return Handle(h, int(b.rs[i]), b.params, batch=b)


def burr_batch_free(b: Batch):
    b.free()


def burr_query(h: Handle, keys, out=None, stream=None):
    import torch
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    if out is None:
        out = torch.empty(keys.numel(), dtype=value_dtype(h.r), device=keys.device)
    _check_tensor(out, "out", (value_dtype(h.r),))
    rc = lib().burr_query(h._h, keys.data_ptr() if keys.numel() else None, keys.numel(),
                          out.data_ptr() if out.numel() else None, _stream_of(stream))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_query")
    return out


def burr_contains(h: Handle, keys, out=None, stream=None):
    import torch
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
    rc = lib().burr_contains(h._h, keys.data_ptr() if keys.numel() else None, keys.numel(),
                             out.data_ptr() if out.numel() else None, _stream_of(stream))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_contains")
    return out


def burr_free(h: Handle):
    h.free()


def burr_get_stats(h: Handle) -> dict:
    st = _CStats()
    rc = lib().burr_get_stats(h._h, ctypes.byref(st))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_get_stats")
    layers = [{f: getattr(st.layer[i], f) for f, _ in _CLayerStats._fields_}
              for i in range(st.layers_built)]
    return dict(n=st.n, r=st.r, layers_built=st.layers_built, layers=layers,
                final_n=st.final_n, final_m=st.final_m, final_attempt=st.final_attempt,
                table_bytes=st.table_bytes, ms_sort=st.ms_sort, ms_solve=st.ms_solve,
                ms_final=st.ms_final, ms_total=st.ms_total)


def burr_export(h: Handle) -> bytes:
    need = ctypes.c_size_t(0)
    rc = lib().burr_export(h._h, None, 0, ctypes.byref(need))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_export")
    buf = (ctypes.c_uint8 * need.value)()
    rc = lib().burr_export(h._h, buf, need.value, ctypes.byref(need))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_export")
    return bytes(buf)


def burr_import(data: bytes, stream=None) -> Handle:
    cp = Params().c(_stream_of(stream))
    h = lib().burr_import(data, len(data), ctypes.byref(cp))
    if not h:
        raise BurrError(lib().burr_last_error(), "burr_import")
    r = int.from_bytes(data[20:24], "little")
    return Handle(h, r, Params())


def burr_debug_layer_keys(h: Handle, layer: int):
    import numpy as np
    n = lib().burr_debug_layer_keys(h._h, layer, None, 0)
    if n < 0:
        raise BurrError(int(n), "burr_debug_layer_keys")
    out = np.zeros(n, dtype=np.uint64)
    if n:
        lib().burr_debug_layer_keys(h._h, layer, out.ctypes.data, n)
    return out


def burr_estimate_build_bytes(n: int, r: int, params: Params | None = None):
    """(table bytes, workspace bytes) the library expects a build to hold."""
    cp = (params or Params()).c(None)
    tb, wb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = lib().burr_estimate_build_bytes(n, r, ctypes.byref(cp), ctypes.byref(tb),
                                         ctypes.byref(wb))
    if rc != BURR_OK:
        raise BurrError(rc, "burr_estimate_build_bytes")
    return tb.value, wb.value


def burr_release_workspaces():
    """Free the device workspace the library keeps between builds."""
    lib().burr_release_workspaces()


class Server:
    """Request loop with resident structures (burr_server_* in include/burr.h).

    submit_build/submit_query return request ids at once; poll() returns
    completions. The tensors of a request are kept referenced here until its
    completion has been polled, so the library never sees freed memory."""

    def __init__(self, budget_bytes: int = 0, workers: int = 4, max_batch: int = 1024,
                 max_batch_keys: int = 1 << 28, evict_lru: bool = False,
                 params: Params | None = None, no_device: bool = False):
        self.params = params or Params()
        cfg = _CServerConfig()
        lib().burr_server_default_config(ctypes.byref(cfg))
        cfg.workers = workers
        cfg.budget_bytes = budget_bytes
        cfg.max_batch = max_batch
        cfg.max_batch_keys = max_batch_keys
        cfg.flags = (BURR_SERVER_EVICT_LRU if evict_lru else 0) | \
            (BURR_SERVER_NO_DEVICE if no_device else 0)
        cp = self.params.c(None)
        self._s = lib().burr_server_create(ctypes.byref(cfg), ctypes.byref(cp))
        if not self._s:
            raise BurrError(lib().burr_last_error(), "burr_server_create")
        self._live = {}
        self._r = {}

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_s", None):
            lib().burr_server_destroy(self._s)
            self._s = None
            self._live.clear()

    def submit_build(self, keys, values, r: int) -> int:
        import torch
        _check_tensor(keys, "keys", (torch.int64, torch.uint64))
        vptr = None
        if values is not None and not self.params.filter_mode:
            _check_tensor(values, "values", (value_dtype(r),))
            if values.numel() != keys.numel():
                raise ValueError("keys and values differ in length")
            vptr = values.data_ptr() if values.numel() else None
        rid = ctypes.c_uint64(0)
        rc = lib().burr_server_submit_build(self._s, keys.data_ptr() if keys.numel() else None,
                                            vptr, keys.numel(), r, ctypes.byref(rid))
        if rc != BURR_OK:
            raise BurrError(rc, "burr_server_submit_build")
        self._live[rid.value] = (keys, values)
        self._r[rid.value] = r
        return rid.value

    def submit_query(self, struct_id: int, keys, out=None):
        """Returns (request id, out tensor); out is valid after completion."""
        import torch
        _check_tensor(keys, "keys", (torch.int64, torch.uint64))
        r = self._r.get(struct_id, 8)
        if out is None:
            out = torch.empty(keys.numel(), dtype=value_dtype(r), device=keys.device)
        rid = ctypes.c_uint64(0)
        rc = lib().burr_server_submit_query(self._s, struct_id,
                                            keys.data_ptr() if keys.numel() else None,
                                            keys.numel(), out.data_ptr() if out.numel() else None,
                                            ctypes.byref(rid))
        if rc != BURR_OK:
            raise BurrError(rc, "burr_server_submit_query")
        self._live[rid.value] = (keys, out)
        return rid.value, out

    def poll(self, max_items: int = 4096, timeout_ms: int = 0) -> list:
        buf = (_CCompletion * max_items)()
        got = ctypes.c_uint32(0)
        rc = lib().burr_server_poll(self._s, buf, max_items, ctypes.byref(got), timeout_ms)
        if rc != BURR_OK:
            raise BurrError(rc, "burr_server_poll")
        out = []
        for i in range(got.value):
            c = {f: getattr(buf[i], f) for f, _ in _CCompletion._fields_}
            self._live.pop(c["req_id"], None)
            out.append(c)
        return out

    def drain(self):
        lib().burr_server_drain(self._s)

    def drop(self, struct_id: int):
        rc = lib().burr_server_drop(self._s, struct_id)
        if rc != BURR_OK:
            raise BurrError(rc, "burr_server_drop")

    def handle(self, struct_id: int):
        h = lib().burr_server_handle(self._s, struct_id)
        return Handle(h, self._r[struct_id], self.params, batch=self) if h else None

    def info(self) -> dict:
        st = _CServerInfo()
        lib().burr_server_get_info(self._s, ctypes.byref(st))
        return {f: getattr(st, f) for f, _ in _CServerInfo._fields_}


# short aliases
build = burr_build
build_batch = burr_build_batch
build_noalloc = burr_build_noalloc
build_batch_tuned = burr_build_batch_tuned
autotune = burr_autotune
import_ = burr_import
