"""GPU: the request loop gives every request the result it gets alone.

Builds and queries are submitted together so that they run concurrently on
the workers' streams and small builds get packed into batched builds; every
structure must export the same bytes as a standalone burr_build of its keys
(and as the oracle's, for a few), and every query must return what a
standalone query returns."""
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


def _wait_all(srv, expect):
    done = {}
    while len(done) < expect:
        for c in srv.poll(timeout_ms=2000):
            done[c["req_id"]] = c
        if srv.info()["pending"] == 0 and srv.info()["running"] == 0:
            for c in srv.poll():
                done[c["req_id"]] = c
            break
    return done


def test_alone_equals_mix():
    burr = _burr()
    params = burr.Params(ranges=1 << 10)
    sizes = [1000, 250_000, 3000, 40_000, 0, 120_000, 777, 2_000, 60_000, 5, 500_000, 9_000]
    rs = [8, 8, 3, 8, 8, 13, 1, 8, 16, 2, 8, 5]
    srv = burr.Server(workers=4, params=params)
    reqs = []
    for i, (n, r) in enumerate(zip(sizes, rs)):
        k = W.keys(n, 300 + i)
        v = W.values(n, r, 400 + i)
        reqs.append((k, v, r, to_dev(k), to_dev(v)))
    print(f"[server] {len(sizes)} builds, {sum(sizes)} keys", flush=True)
    ids = [srv.submit_build(dk, dv, r) for (_, _, r, dk, dv) in reqs]
    # queries interleaved with the builds: members and non-members
    queries = []
    for j in range(30):
        t = j % len(ids)
        k = reqs[t][0]
        q = np.concatenate([k[: 3000], W.non_members(max(len(k), 1), 2000, 500 + j)])
        dq = to_dev(q)
        rid, out = srv.submit_query(ids[t], dq)
        queries.append((rid, t, q, out))
    done = _wait_all(srv, len(ids) + len(queries))
    assert all(done[i]["status"] == 0 for i in ids)
    assert all(done[rid]["status"] == 0 for rid, *_ in queries)
    for i, (k, v, r, dk, dv) in enumerate(reqs):
        alone = burr.build(dk, dv, r, params)
        assert srv.handle(ids[i]).export() == alone.export(), f"structure {i}"
        if len(k) <= 3000:
            ref = oracle.build(k, v, r, oracle.Params(ranges=1 << 10))
            assert alone.export() == ref.export()
        for rid, t, q, out in queries:
            if t == i:
                assert torch.equal(out, alone.query(to_dev(q))), f"query {rid}"
    info = srv.info()
    srv.close()
    assert info["resident"] == len(ids)


def test_small_builds_are_packed_and_stay_exact():
    burr = _burr()
    params = burr.Params()
    srv = burr.Server(workers=2, params=params)
    keys = W.keys(400 * 1500, 77)
    vals = W.values(400 * 1500, 8, 78)
    dk, dv = to_dev(keys), to_dev(vals)
    ids = [srv.submit_build(dk[i * 1500:(i + 1) * 1500], dv[i * 1500:(i + 1) * 1500], 8)
           for i in range(400)]
    done = _wait_all(srv, len(ids))
    batches = {done[i]["batch_id"] for i in ids}
    print(f"[server] 400 builds in {len(batches)} batched builds", flush=True)
    assert len(batches) < 400
    for i in range(0, 400, 37):
        h = srv.handle(ids[i])
        ref = oracle.build(keys[i * 1500:(i + 1) * 1500], vals[i * 1500:(i + 1) * 1500], 8,
                           oracle.Params())
        assert h.export() == ref.export()
    srv.close()


def test_bad_request_fails_alone_in_a_packed_build():
    burr = _burr()
    srv = burr.Server(workers=2)
    keys = W.keys(30 * 2000, 88)
    vals = W.values(30 * 2000, 8, 89)
    keys[5 * 2000 + 7] = keys[5 * 2000 + 8]  # request 5: one key with two values
    vals[5 * 2000 + 7] = vals[5 * 2000 + 8] ^ 1
    dk, dv = to_dev(keys), to_dev(vals)
    ids = [srv.submit_build(dk[i * 2000:(i + 1) * 2000], dv[i * 2000:(i + 1) * 2000], 8)
           for i in range(30)]
    done = _wait_all(srv, 30)
    assert done[ids[5]]["status"] == burr.BURR_E_UNSOLVABLE
    assert all(done[ids[i]]["status"] == 0 for i in range(30) if i != 5)
    got = srv.handle(ids[6]).query(dk[6 * 2000:7 * 2000])
    assert torch.equal(got, dv[6 * 2000:7 * 2000])
    srv.close()


def test_budget_and_eviction_on_device():
    burr = _burr()
    tb, wb = burr.burr_estimate_build_bytes(200_000, 8)
    budget = 3 * tb + wb + tb // 2
    srv = burr.Server(workers=2, budget_bytes=budget, evict_lru=True)
    keys = [to_dev(W.keys(200_000, 90 + i)) for i in range(5)]
    vals = [to_dev(W.values(200_000, 8, 95 + i)) for i in range(5)]
    ids = []
    for i in range(5):
        ids.append(srv.submit_build(keys[i], vals[i], 8))
        _wait_all(srv, 1)
    info = srv.info()
    assert info["peak_bytes"] <= budget and info["evictions"] >= 1
    # the newest structures are resident and exact
    got = srv.handle(ids[4]).query(keys[4])
    assert torch.equal(got, vals[4])
    rid, out = srv.submit_query(ids[0], keys[0])
    c = _wait_all(srv, 1)
    assert c[rid]["status"] == burr.BURR_E_EVICTED
    srv.close()
