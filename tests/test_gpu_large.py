"""GPU: the full-size workloads - the 1B-key filter build (2^18 ranges, r = 16
and r = 1), the 100M-key retrieval build (2^16 ranges, r = 8) and the
200,000-structure batch.

The oracle cannot build a billion keys within a test, so this checks
(1) properties that hold at any size: every member is found, the
false-positive rate of non-members matches 2^-r (Sec. 1: a retrieval
structure of r-bit fingerprints is a filter), and each layer's geometry
follows its closed form; and (2) exact parity on sampled layer-0 ranges: the
oracle solves each sampled range alone from the keys that start in it
(ranges are independent, Sec. 3), and its threshold codes, solution words
and bumped keys must equal the library's; batch members sampled across the
size range must export exactly the oracle's structure of their own keys."""
import struct

import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 1_000_000_000
RANGES = 1 << 18
SEED_KEYS = 3
CHUNK = 100_000_000


def _burr():
    import paper_2411_12365_amd as burr
    return burr


@pytest.fixture(scope="module")
def big():
    dev = torch.device("cuda:0")
    print(f"[large] generating {N} keys on the device", flush=True)
    keys_dev = W.keys_device(N, SEED_KEYS, dev)
    keys = keys_dev.cpu().numpy().view(np.uint64)
    for lo in (0, 123_456_789, N - 1000):  # the device stream is the numpy stream
        assert np.array_equal(keys[lo:lo + 1000], W.keys(1000, SEED_KEYS, lo))
    op = oracle.Params(ranges=RANGES, filter_mode=1)
    m, B, R = oracle.layer_geometry(op, N)
    assert (m, B, R) == (970_000_000, 15_156_250, RANGES)
    print("[large] oracle start buckets of every key", flush=True)
    sb = oracle.start_buckets(keys, 0, m, op)
    # sampled ranges: both ends, the middle and a few random ones
    rng = np.random.default_rng(33)
    rhos = sorted({0, 1, R // 2, R - 2, R - 1, *rng.integers(0, R, 3).tolist()})
    lut = np.full(B, -1, dtype=np.int8)
    bounds = []
    for i, rho in enumerate(rhos):
        first, last = oracle.range_buckets(B, R, rho)
        lut[first:last] = i
        bounds.append((first, last))
    tag = lut[sb]
    sel = np.flatnonzero(tag >= 0)
    members = {rho: keys[sel[tag[sel] == i]] for i, rho in enumerate(rhos)}
    yield dict(keys_dev=keys_dev, keys=keys, op=op, m=m, B=B, R=R, rhos=rhos,
               bounds=bounds, members=members, lut=lut)
    del keys_dev
    _burr().burr_release_workspaces()
    torch.cuda.empty_cache()


def _layer0(buf: bytes, r: int):
    """Layer-0 codes and solution words of a canonical export."""
    off = 8 + 16 * 4 + 16
    n0, m0, R0 = struct.unpack_from("<3Q", buf, off)
    off += 24
    B = m0 // 64
    ncode = (B + 31) // 32
    codes = np.frombuffer(buf, dtype=np.uint64, count=ncode, offset=off)
    off += ncode * 8
    words = np.frombuffer(buf, dtype=np.uint64, count=(m0 // 64) * r, offset=off)
    return n0, m0, R0, codes, words


@pytest.mark.parametrize("r", [16, 1])
def test_billion_key_filter(big, r):
    burr = _burr()
    params = burr.Params(ranges=RANGES, filter_mode=1, flags=burr.BURR_FLAG_KEEP_LAYER_KEYS)
    print(f"[large] build r={r}", flush=True)
    h = burr.build(big["keys_dev"], None, r, params)
    st = h.stats()

    # geometry of every layer follows the closed form of its key count
    n_l = N
    for li, L in enumerate(st["layers"]):
        m, B, R = oracle.layer_geometry(big["op"], n_l)
        assert (L["n"], L["m"], L["nranges"]) == (n_l, m, R), f"layer {li}"
        assert 0 < L["bumped"] < 0.15 * n_l
        n_l = L["bumped"]
    assert st["final_n"] == n_l

    # every member is found
    print("[large] members", flush=True)
    for lo in range(0, N, CHUNK):
        assert bool(h.contains(big["keys_dev"][lo:lo + CHUNK]).all()), f"members {lo}"

    # false positives of a billion non-members: Binomial(1e9, 2^-r)
    print("[large] non-members", flush=True)
    fp = 0
    dev = big["keys_dev"].device
    for lo in range(0, N, CHUNK):
        q = W.keys_device(CHUNK, SEED_KEYS, dev, start=N + lo)
        fp += int(h.contains(q).sum())
        del q
    p = 2.0 ** -r
    mean, sd = N * p, (N * p * (1 - p)) ** 0.5
    print(f"[large] r={r}: {fp} false positives, expected {mean:.0f} +- {sd:.0f}", flush=True)
    assert abs(fp - mean) <= 6 * sd

    # sampled ranges: exact codes, solution words and bump sets
    print("[large] sampled ranges", flush=True)
    n0, m0, R0, codes, words = _layer0(h.export(), r)
    assert (n0, m0, R0) == (N, big["m"], big["R"])
    bumped_gpu = h.layer_keys(1)
    bsb = oracle.start_buckets(bumped_gpu, 0, big["m"], big["op"])
    btag = big["lut"][bsb]
    for i, rho in enumerate(big["rhos"]):
        first, last = big["bounds"][i]
        ref = oracle.layer_range(big["members"][rho], None, r, big["op"], 0, N, rho)
        beta = np.arange(first, last, dtype=np.uint64)
        got_codes = (codes[beta // 32] >> (2 * (beta % 32))) & 3
        assert np.array_equal(got_codes.astype(np.uint8), ref["codes"]), f"codes, range {rho}"
        assert np.array_equal(words[first * r:last * r], ref["W"]), f"words, range {rho}"
        assert set(bumped_gpu[btag == i].tolist()) == set(ref["bumped"].tolist()), \
            f"bumped keys, range {rho}"
    h.free()


def _sampled_ranges(keys, op, n, R_expect, seed):
    m, B, R = oracle.layer_geometry(op, n)
    assert R == R_expect
    sb = oracle.start_buckets(keys, 0, m, op)
    rng = np.random.default_rng(seed)
    rhos = sorted({0, 1, R // 2, R - 2, R - 1, *rng.integers(0, R, 3).tolist()})
    lut = np.full(B, -1, dtype=np.int8)
    bounds = []
    for i, rho in enumerate(rhos):
        first, last = oracle.range_buckets(B, R, rho)
        lut[first:last] = i
        bounds.append((first, last))
    return m, B, R, rhos, bounds, lut, lut[sb]


def test_hundred_million_key_retrieval():
    burr = _burr()
    n, R_expect, r = 100_000_000, 1 << 16, 8
    dev = torch.device("cuda:0")
    print(f"[large] {n} keys, r={r}, {R_expect} ranges", flush=True)
    keys_dev = W.keys_device(n, 2, dev)
    vals_dev = (W.splitmix64_device(1002, 0, n, dev) & 0xFF).to(torch.uint8)
    keys = keys_dev.cpu().numpy().view(np.uint64)
    vals = vals_dev.cpu().numpy()
    assert np.array_equal(vals[:1000], W.values(1000, r, 1002))
    op = oracle.Params(ranges=R_expect)
    m, B, R, rhos, bounds, lut, tag = _sampled_ranges(keys, op, n, R_expect, 22)
    h = burr.build(keys_dev, vals_dev, r,
                   burr.Params(ranges=R_expect, flags=burr.BURR_FLAG_KEEP_LAYER_KEYS))
    for lo in range(0, n, CHUNK):
        assert torch.equal(h.query(keys_dev[lo:lo + CHUNK]), vals_dev[lo:lo + CHUNK])
    n0, m0, R0, codes, words = _layer0(h.export(), r)
    assert (n0, m0, R0) == (n, m, R)
    bumped_gpu = h.layer_keys(1)
    btag = lut[oracle.start_buckets(bumped_gpu, 0, m, op)]
    sel = np.flatnonzero(tag >= 0)
    for i, rho in enumerate(rhos):
        first, last = bounds[i]
        idx = sel[tag[sel] == i]
        ref = oracle.layer_range(keys[idx], vals[idx], r, op, 0, n, rho)
        beta = np.arange(first, last, dtype=np.uint64)
        got_codes = (codes[beta // 32] >> (2 * (beta % 32))) & 3
        assert np.array_equal(got_codes.astype(np.uint8), ref["codes"]), f"codes, range {rho}"
        assert np.array_equal(words[first * r:last * r], ref["W"]), f"words, range {rho}"
        assert set(bumped_gpu[btag == i].tolist()) == set(ref["bumped"].tolist()), \
            f"bumped keys, range {rho}"
    h.free()


def test_two_hundred_thousand_structure_batch():
    burr = _burr()
    count = 200_000
    sizes = W.batch_sizes(count, 4)
    rs = np.random.default_rng(4).integers(1, 4, size=count).astype(np.uint32)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    N = int(offs[-1])
    dev = torch.device("cuda:0")
    print(f"[large] batch of {count} structures, {N} keys", flush=True)
    keys_dev = W.keys_device(N, 4, dev)
    vals_dev = (W.splitmix64_device(1004, 0, N, dev) & 0xFF).to(torch.uint8)
    params = burr.Params(ranges=1 << 16)
    b = burr.build_batch(keys_dev, vals_dev, offs, rs, params)
    order = np.argsort(sizes, kind="stable")
    picks = sorted({int(order[0]), int(order[-1]), int(order[count // 2]),
                    *np.random.default_rng(44).integers(0, count, 29).tolist(),
                    *order[-8:].tolist()})
    for i in picks:
        lo, hi, r = int(offs[i]), int(offs[i + 1]), int(rs[i])
        mk = W.keys(hi - lo, 4, lo)
        mv = (W.splitmix64(1004, lo, hi - lo) & np.uint64((1 << r) - 1)).astype(np.uint8)
        ref = oracle.build(mk, mv, r, oracle.Params(ranges=1 << 16))
        hm = b.member(i)
        assert hm.export() == ref.export(), f"member {i} ({hi - lo} keys, r={r})"
        assert torch.equal(hm.query(keys_dev[lo:hi]), vals_dev[lo:hi] & ((1 << r) - 1))
    b.free()
