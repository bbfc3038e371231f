"""GPU: the C ABI's memory contract (§ boundary of the library).

- allocator callbacks: with burr_params.alloc/free backed by PyTorch's
  caching allocator, every device buffer of a build (workspace and tables)
  comes from the callbacks, the structure equals the oracle's, and freeing
  it hands every byte back;
- import of crafted export bytes whose sizes would overflow the table size
  computation is rejected (BURR_E_INVALID) before anything is allocated; no
  query is run on such buffers.
"""
import struct

import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W
from tests.gpu_compare import check_handle, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _burr():
    import paper_2411_12365_amd as burr
    return burr


def test_build_through_torch_allocator():
    burr = _burr()
    n, r, kw = 200_000, 8, dict(ranges=64, seed=3)
    keys, vals = W.keys(n, 71), W.values(n, r, 72)
    print(f"[boundary] torch allocator n={n}", flush=True)
    alloc = burr.TorchAllocator()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    kd, vd = to_dev(keys), to_dev(vals)
    base = torch.cuda.memory_allocated()
    h = burr.build(kd, vd, r, burr.Params(flags=burr.BURR_FLAG_KEEP_LAYER_KEYS, **kw),
                   allocator=alloc)
    st = h.stats()
    # workspace buffers and tables all came through the callbacks; what the
    # handle still holds (its tables) is torch memory
    assert alloc.allocations >= 10
    assert alloc.live_bytes >= st["table_bytes"] > 0
    held = torch.cuda.memory_allocated() - base  # torch rounds blocks up to 512 bytes
    assert alloc.live_bytes <= held <= alloc.live_bytes + 512 * len(alloc.live)
    ref = oracle.build(keys, vals, r, oracle.Params(**kw))
    check_handle(h, ref, keys)
    h.free()
    torch.cuda.synchronize()
    assert alloc.live_bytes == 0
    assert torch.cuda.memory_allocated() == base
    del kd, vd
    assert torch.cuda.memory_allocated() == before


def test_batch_through_torch_allocator():
    burr = _burr()
    sizes = [0, 150, 3000, 20000]
    rs = np.array([8, 1, 3, 8], dtype=np.uint32)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = W.keys(int(offs[-1]), 73)
    vals = W.values(int(offs[-1]), 8, 74)
    print("[boundary] torch allocator batch", flush=True)
    alloc = burr.TorchAllocator()
    b = burr.build_batch(to_dev(keys), to_dev(vals), offs, rs, burr.Params(ranges=16),
                         allocator=alloc)
    assert alloc.allocations >= 10 and alloc.live_bytes > 0
    for i, sz in enumerate(sizes):
        lo, hi, ri = int(offs[i]), int(offs[i + 1]), int(rs[i])
        ref = oracle.build(keys[lo:hi], vals[lo:hi] & ((1 << ri) - 1), ri,
                           oracle.Params(ranges=16))
        assert b.member(i).export() == ref.export(), f"member {i}"
    b.free()
    torch.cuda.synchronize()
    assert alloc.live_bytes == 0


def _header(r=8, built=0, layers=3, bucket=64, n=5, seed=0):
    hdr = [2, 64, bucket, r, 97, 100, 110, 100, layers, 16, 32, 1, 16, 16, 0, built, 0, 0, 0, 0]
    return struct.pack("<Q20IQQ", 0x3170786552527542, *hdr, seed, n)


def test_import_rejects_sizes_that_would_overflow():
    burr = _burr()
    lib = burr.lib()
    print("[boundary] crafted imports", flush=True)
    # final layer m = 64 * (2^56 + 1) with r = 32: m/64 * 32 words wraps to 32
    m_bad = 64 * ((1 << 56) + 1)
    buf = _header(r=32) + struct.pack("<3Q", 5, m_bad, 0) + bytes(32 * 8)
    assert lib.burr_import(buf, len(buf), None) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    # a BuRR layer with the same wrap in its solution words
    buf = _header(r=32, built=1) + struct.pack("<3Q", 5, m_bad, 1) + bytes(64 * 8)
    assert lib.burr_import(buf, len(buf), None) is None
    assert lib.burr_last_error() == burr.BURR_E_INVALID
    # more layers built than the parameters allow, and an invalid bucket size
    for hb in (_header(built=4, layers=3), _header(bucket=128)):
        buf = hb + bytes(64)
        assert lib.burr_import(buf, len(buf), None) is None
        assert lib.burr_last_error() == burr.BURR_E_INVALID
    # a genuine export still imports
    keys, vals = W.keys(1000, 75), W.values(1000, 8, 76)
    ref = oracle.build(keys, vals, 8, oracle.Params())
    h = burr.import_(ref.export())
    assert h.export() == ref.export()
    got = h.query(to_dev(keys)).cpu().numpy()
    assert np.array_equal(got, vals)
    h.free()
