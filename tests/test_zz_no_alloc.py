"""GPU: burr_build_noalloc (a build whose temporary buffers come from the
library's fixed scratch array and whose tables go to caller memory) gives
the export bytes and query results of burr_build, on two calls in a row, the
second with fewer keys, and rejects inputs beyond the array's size."""
import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W
from tests.gpu_compare import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _burr():
    import paper_2411_12365_amd as burr
    return burr


@pytest.mark.parametrize("r", [8, 16])
def test_noalloc_equals_build_two_calls(r):
    burr = _burr()
    for n, kw in ((1_000_000, dict(ranges=64, seed=5)), (30_000, dict(ranges=16, seed=6))):
        print(f"[noalloc] r={r} n={n} {kw}", flush=True)
        keys, vals = W.keys(n, 80 + n % 7), W.values(n, r, 81)
        kd, vd = to_dev(keys), to_dev(vals)
        params = burr.Params(**kw)
        tb, _ = burr.burr_estimate_build_bytes(n, r, params)
        table = torch.empty(tb, dtype=torch.uint8, device="cuda")
        h = burr.build_noalloc(kd, vd, r, table, params)
        ref = burr.build(kd, vd, r, params)
        assert h.export() == ref.export()
        q = np.concatenate([keys[:50_000], W.non_members(n, 50_000, 9)])
        qd = to_dev(q)
        assert torch.equal(h.query(qd), ref.query(qd))
        if n <= 30_000:  # small enough for the oracle within the test
            o = oracle.build(keys, vals, r, oracle.Params(**kw))
            assert h.export() == o.export()
        h.free()
        ref.free()


def test_noalloc_filter_and_empty():
    burr = _burr()
    params = burr.Params(ranges=8, filter_mode=1)
    table = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    keys = W.keys(20_000, 90)
    print("[noalloc] filter", flush=True)
    h = burr.build_noalloc(to_dev(keys), None, 8, table, params)
    o = oracle.build(keys, None, 8, oracle.Params(ranges=8, filter_mode=1))
    assert h.export() == o.export()
    h.free()
    print("[noalloc] empty", flush=True)
    e = burr.build_noalloc(to_dev(np.zeros(0, np.uint64)), to_dev(np.zeros(0, np.uint8)), 8,
                           table, burr.Params())
    assert e.export() == oracle.build(np.zeros(0, np.uint64), np.zeros(0, np.uint8), 8,
                                      oracle.Params()).export()
    e.free()


def test_noalloc_rejects_what_does_not_fit():
    burr = _burr()
    table = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    big = torch.zeros(4_000_000, dtype=torch.int64, device="cuda")   # never read: rejected first
    vals = torch.zeros(4_000_000, dtype=torch.uint8, device="cuda")
    print("[noalloc] too many keys", flush=True)
    with pytest.raises(burr.BurrError) as ei:
        burr.build_noalloc(big, vals, 8, table, burr.Params())
    assert ei.value.code == burr.BURR_E_INVALID
    # a table too small for the structure: a clean error, and the next call works
    keys, v = W.keys(100_000, 91), W.values(100_000, 8, 92)
    print("[noalloc] table too small", flush=True)
    with pytest.raises(burr.BurrError) as ei:
        burr.build_noalloc(to_dev(keys), to_dev(v), 8, table, burr.Params(ranges=16))
    assert ei.value.code == burr.BURR_E_NOMEM
    tb, _ = burr.burr_estimate_build_bytes(100_000, 8, burr.Params(ranges=16))
    table = torch.empty(tb, dtype=torch.uint8, device="cuda")
    h = burr.build_noalloc(to_dev(keys), to_dev(v), 8, table, burr.Params(ranges=16))
    o = oracle.build(keys, v, 8, oracle.Params(ranges=16))
    assert h.export() == o.export()
    h.free()
