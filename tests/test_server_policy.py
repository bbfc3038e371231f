"""Admission and scheduling policy of the request loop, on the CPU.

The server runs in scheduling-only mode (BURR_SERVER_NO_DEVICE): the same
queueing, packing, budget and eviction code as on the GPU, with requests that
complete after a short sleep instead of device work. Pointers passed here
are placeholders that this mode never dereferences."""
import ctypes
import time

import pytest

KEYS, VALS, OUT = 0x10000, 0x20000, 0x30000


def _burr():
    import paper_2411_12365_amd as burr
    return burr


class Sim:
    def __init__(self, budget=0, workers=4, evict=False, max_batch=1024):
        burr = _burr()
        self.burr = burr
        self.lib = burr.lib()
        cfg = burr._CServerConfig()
        self.lib.burr_server_default_config(ctypes.byref(cfg))
        cfg.workers = workers
        cfg.budget_bytes = budget
        cfg.max_batch = max_batch
        cfg.flags = burr.BURR_SERVER_NO_DEVICE | (burr.BURR_SERVER_EVICT_LRU if evict else 0)
        self.cp = burr.Params().c(None)
        self.s = self.lib.burr_server_create(ctypes.byref(cfg), ctypes.byref(self.cp))
        assert self.s
        self.done = {}

    def build(self, n, r=8):
        rid = ctypes.c_uint64(0)
        rc = self.lib.burr_server_submit_build(self.s, KEYS, VALS, n, r, ctypes.byref(rid))
        return rc, rid.value

    def query(self, sid, n):
        rid = ctypes.c_uint64(0)
        rc = self.lib.burr_server_submit_query(self.s, sid, KEYS, n, OUT, ctypes.byref(rid))
        assert rc == 0
        return rid.value

    def poll_all(self):
        self.lib.burr_server_drain(self.s)
        buf = (self.burr._CCompletion * 4096)()
        got = ctypes.c_uint32(0)
        while True:
            self.lib.burr_server_poll(self.s, buf, 4096, ctypes.byref(got), 0)
            for i in range(got.value):
                c = {f: getattr(buf[i], f) for f, _ in self.burr._CCompletion._fields_}
                self.done[c["req_id"]] = c
            if got.value < 4096:
                break
        return self.done

    def info(self):
        st = self.burr._CServerInfo()
        self.lib.burr_server_get_info(self.s, ctypes.byref(st))
        return {f: getattr(st, f) for f, _ in self.burr._CServerInfo._fields_}

    def close(self):
        self.lib.burr_server_destroy(self.s)


def est(n, r=8):
    return _burr().burr_estimate_build_bytes(n, r)


def test_estimates_grow_with_n_and_r():
    t1, w1 = est(10_000, 1)
    t8, w8 = est(10_000, 8)
    T8, W8 = est(1_000_000, 8)
    assert 0 < t1 < t8 < T8 and 0 < w1 <= w8 < W8
    # the layer-0 table alone is m0 * r bits
    assert t8 >= (10_000 * 97 // 100) * 8 // 8


def test_every_request_completes_and_queries_follow_their_build():
    sim = Sim()
    ids = [sim.build(n)[1] for n in (1000, 50_000, 200, 0, 120_000)]
    qs = [(sim.query(sid, 5000), sid) for sid in ids for _ in range(2)]
    done = sim.poll_all()
    sim.close()
    for sid in ids:
        assert done[sid]["status"] == 0 and done[sid]["kind"] == 1
    for qid, sid in qs:
        c = done[qid]
        assert c["status"] == 0 and c["kind"] == 2 and c["struct_id"] == sid
        assert c["t_start_ms"] >= done[sid]["t_end_ms"] - 1e-6
        assert c["t_end_ms"] >= c["t_start_ms"] >= c["t_submit_ms"]


def test_builds_are_admitted_in_arrival_order_and_packed():
    sim = Sim(workers=2)
    ids = [sim.build(2000 + 10 * i)[1] for i in range(300)]
    done = sim.poll_all()
    info = sim.info()
    sim.close()
    starts = [done[i]["t_start_ms"] for i in ids]
    assert starts == sorted(starts)
    batches = {done[i]["batch_id"] for i in ids}
    assert len(batches) < len(ids)  # requests waiting together share a build
    assert info["batches"] == len(batches)


def test_budget_is_never_exceeded_and_oversize_is_rejected():
    tb, wb = est(100_000)
    budget = 3 * (tb + wb)
    sim = Sim(budget=budget, workers=4)
    rc, _ = sim.build(50_000_000)
    assert rc == _burr().BURR_E_BUDGET
    ids = [sim.build(100_000)[1] for _ in range(20)]
    done = sim.poll_all()
    info = sim.info()
    sim.close()
    assert all(done[i]["status"] == 0 for i in ids)
    assert info["peak_bytes"] <= budget
    assert info["resident"] == 20


def test_build_that_can_never_fit_fails_instead_of_waiting():
    tb, wb = est(100_000)
    budget = 2 * tb + wb + tb // 2
    sim = Sim(budget=budget, workers=2)
    a = sim.build(100_000)[1]
    b = sim.build(100_000)[1]
    sim.poll_all()
    c = sim.build(100_000)[1]  # resident tables leave no room, nothing to evict
    done = sim.poll_all()
    sim.close()
    assert done[a]["status"] == 0 and done[b]["status"] == 0
    assert done[c]["status"] == _burr().BURR_E_BUDGET


def test_lru_eviction_under_pressure():
    burr = _burr()
    tb, wb = est(100_000)
    budget = 3 * tb + wb + tb // 2
    sim = Sim(budget=budget, workers=2, evict=True)
    ids = []
    for _ in range(3):  # one at a time: one structure per batch
        ids.append(sim.build(100_000)[1])
        sim.poll_all()
    q1 = sim.query(ids[0], 1000)  # structure 0 becomes the most recently used
    sim.poll_all()
    d = sim.build(100_000)[1]     # needs room: evicts structure 1 (least recent)
    sim.poll_all()
    q0, q1b, q2 = sim.query(ids[0], 10), sim.query(ids[1], 10), sim.query(ids[2], 10)
    done = sim.poll_all()
    info = sim.info()
    sim.close()
    assert done[q1]["status"] == 0 and done[d]["status"] == 0
    assert done[q0]["status"] == 0 and done[q2]["status"] == 0
    assert done[q1b]["status"] == burr.BURR_E_EVICTED
    assert info["evictions"] == 1 and info["peak_bytes"] <= budget


def test_queries_are_not_held_behind_builds():
    sim = Sim(workers=2)
    a = sim.build(1000)[1]
    sim.poll_all()
    big = sim.build(200_000_000)[1]  # about 0.4 s of simulated work
    time.sleep(0.05)
    q = sim.query(a, 1000)
    done = sim.poll_all()
    sim.close()
    assert done[q]["t_end_ms"] < done[big]["t_end_ms"]


def test_drop_and_unknown_targets():
    burr = _burr()
    sim = Sim()
    a = sim.build(1000)[1]
    sim.poll_all()
    assert sim.lib.burr_server_drop(sim.s, a) == 0
    q = sim.query(a, 10)
    u = sim.query(123456, 10)
    done = sim.poll_all()
    info = sim.info()
    sim.close()
    assert done[q]["status"] == burr.BURR_E_EVICTED
    assert done[u]["status"] == burr.BURR_E_EVICTED
    assert info["resident_bytes"] == 0 and info["resident"] == 0


def test_invalid_submissions():
    burr = _burr()
    sim = Sim()
    rid = ctypes.c_uint64(0)
    assert sim.lib.burr_server_submit_build(sim.s, None, VALS, 10, 8, ctypes.byref(rid)) == \
        burr.BURR_E_INVALID
    assert sim.lib.burr_server_submit_build(sim.s, KEYS, VALS, 10, 0, ctypes.byref(rid)) == \
        burr.BURR_E_INVALID
    assert sim.lib.burr_server_submit_query(sim.s, 1, KEYS, 10, None, ctypes.byref(rid)) == \
        burr.BURR_E_INVALID
    sim.close()


def test_destroy_waits_for_pending_requests():
    sim = Sim(workers=1)
    t0 = time.perf_counter()
    for _ in range(5):
        sim.build(10_000_000)  # about 20 ms of simulated work each, run one by one
    sim.close()  # returns only after the builds ran
    assert time.perf_counter() - t0 >= 0.09


@pytest.mark.parametrize("workers", [1, 3])
def test_worker_counts(workers):
    sim = Sim(workers=workers)
    ids = [sim.build(5000)[1] for _ in range(10)]
    qs = [sim.query(i, 100) for i in ids]
    done = sim.poll_all()
    sim.close()
    assert all(done[i]["status"] == 0 for i in ids + qs)
