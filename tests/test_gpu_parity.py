"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bit-exact comparison of the whole exported structure (per-layer sizes,
2-bit codes, solution words, final layer), of the per-layer key sets, and of
query results for members and non-members.
"""
import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W
from tests.gpu_compare import check_handle, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


_dev = to_dev


def _burr():
    import paper_2411_12365_amd as burr
    return burr


def _compare(keys, vals, r, kw, label=""):
    burr = _burr()
    filt = kw.get("filter_mode", 0)
    print(f"[parity] {label} n={len(keys)} r={r} {kw}", flush=True)
    ref = oracle.build(keys, None if filt else vals, r, oracle.Params(**kw))
    h = burr.build(_dev(keys), None if filt else _dev(vals), r,
                   burr.Params(flags=burr.BURR_FLAG_KEEP_LAYER_KEYS, **kw))
    check_handle(h, ref, keys, filt=bool(filt))
    return h, ref


CASES = [
    (1, 8, dict(ranges=4)),
    (64, 2, dict(ranges=1)),
    (200, 8, dict(ranges=1)),
    (1000, 8, dict(ranges=4, minbpt=2)),
    (5000, 1, dict(ranges=8, minbpt=2, seed=77)),
    (20000, 8, dict(ranges=64)),
    (30000, 16, dict(ranges=16)),
    (30000, 32, dict(ranges=8, seed=5)),
    (25000, 13, dict(ranges=100, minbpt=2, load_num=90, load_den=100, layers=5)),
    (20000, 5, dict(ranges=37, minbpt=3, filter_mode=1, seed=9)),
    # a filter wider than 8 bits through every partition level: its
    # fingerprints are left out of the records and computed at level 3
    (700000, 12, dict(ranges=512, filter_mode=1, seed=21)),
    (8000, 8, dict(layers=0)),
    (20000, 8, dict(ranges=16, t_lo=8, t_hi=40, seed=123)),
    (3000, 4, dict(ranges=6, minbpt=2, load_num=60, load_den=100, layers=4)),
    (200000, 8, dict(ranges=4096, minbpt=4)),
    # the final plain layer is the whole structure: thousands of segments,
    # log2 merge levels, boundary propagation across all of them
    (200000, 8, dict(layers=0)),
    (150000, 32, dict(layers=0, seed=11)),
    (100000, 3, dict(layers=1, ranges=64)),
    # a tight final layer (1.0 slots per key) fails its first attempts,
    # some of them only when segments are merged
    (60000, 8, dict(layers=0, final_num=100, final_den=100, seed=4)),
    (60000, 8, dict(layers=0, final_num=100, final_den=100, seed=5)),
    # 1+-bit thresholds: exact thresholds found by bisection in the ring
    (20000, 8, dict(ranges=64, threshold_mode=1)),
    (200000, 8, dict(ranges=4096, minbpt=4, threshold_mode=1)),
    (100000, 16, dict(ranges=16, threshold_mode=1, filter_mode=1, seed=3)),
    (40000, 8, dict(ranges=64, load_num=80, load_den=100, threshold_mode=1, seed=4)),
    (30000, 1, dict(ranges=8, load_num=70, load_den=100, threshold_mode=1, seed=14)),
    (20000, 32, dict(ranges=1, threshold_mode=1, layers=5, seed=15)),
    # searched cut points: every strategy, search ranges wider and narrower
    # than half a range, with both threshold modes
    (200000, 8, dict(ranges=1000, minbpt=8, cut_strategy=1, cut_search=50)),
    (200000, 8, dict(ranges=1000, minbpt=8, cut_strategy=2, cut_search=50, seed=6)),
    (200000, 4, dict(ranges=1000, minbpt=8, cut_strategy=3, cut_search=50, seed=7)),
    (100000, 8, dict(ranges=300, minbpt=2, cut_strategy=2, cut_search=6, seed=8)),
    (150000, 8, dict(ranges=2000, minbpt=4, cut_strategy=3, cut_search=50,
                     threshold_mode=1, seed=9)),
    (50000, 3, dict(ranges=100, cut_strategy=1, cut_search=1, seed=10)),
]


@pytest.mark.parametrize("n,r,kw", CASES)
def test_structure_matches_oracle(n, r, kw):
    keys = W.keys(n, 1000 + n)
    vals = W.values(n, r, 2000 + n)
    _compare(keys, vals, r, kw, "case")


def test_empty_build():
    burr = _burr()
    h = burr.build(_dev(np.zeros(0, np.uint64)), _dev(np.zeros(0, np.uint8)), 8, burr.Params())
    ref = oracle.build(np.zeros(0, np.uint64), np.zeros(0, np.uint8), 8, oracle.Params())
    assert h.export() == ref.export()
    q = W.keys(100, 5)
    assert (h.query(_dev(q)).cpu().numpy() == 0).all()


def test_equal_duplicates_and_conflicts():
    burr = _burr()
    keys = W.keys(5000, 8)
    vals = W.values(5000, 8, 9)
    dk = np.concatenate([keys, keys[::11]])
    dv = np.concatenate([vals, vals[::11]])
    _compare(dk, dv, 8, dict(ranges=8, minbpt=2), "dups")
    bad = dv.copy()
    bad[-1] ^= 1
    with pytest.raises(burr.BurrError) as e:
        burr.build(_dev(dk), _dev(bad), 8, burr.Params(ranges=8, minbpt=2))
    assert e.value.code == burr.BURR_E_UNSOLVABLE


def test_import_roundtrip():
    burr = _burr()
    keys = W.keys(30000, 3)
    vals = W.values(30000, 8, 4)
    h, ref = _compare(keys, vals, 8, dict(ranges=32), "import")
    h2 = burr.import_(h.export())
    assert h2.export() == ref.export()
    assert np.array_equal(h2.query(_dev(keys)).cpu().numpy(), vals)


def test_one_million_keys_one_range():
    # 1M keys, r = 8, one range (no boundary bumping)
    keys = W.keys(1_000_000, 1)
    vals = W.values(1_000_000, 8, 1001)
    _compare(keys, vals, 8, dict(ranges=1), "1M")


def test_ten_million_keys_many_ranges():
    keys = W.keys(10_000_000, 2)
    vals = W.values(10_000_000, 8, 1002)
    _compare(keys, vals, 8, dict(ranges=1 << 16), "10M")


def _low_word_pair(m, seed, tries=1 << 24, chunk=1 << 22):
    """Two keys that both start at slot 0 of a layer-0 table of m slots and
    whose coefficient rows agree in their low 32 bits but not in their high
    ones. Candidates are screened with a numpy copy of the hash; the oracle's
    hash confirms the pair."""
    def mix(x):
        x = x ^ (x >> np.uint64(33))
        x = x * np.uint64(0xFF51AFD7ED558CCD)
        x = x ^ (x >> np.uint64(33))
        x = x * np.uint64(0xC4CEB9FE1A85EC53)
        return x ^ (x >> np.uint64(33))

    salt_s = np.uint64(oracle.fmix64(seed ^ 1))
    salt_c = np.uint64(oracle.fmix64(seed ^ 2))
    span = m - 63
    first = (2**64 - 1) // span  # start 0 <=> hash * span < 2^64
    rng = np.random.default_rng(2411)
    cand = []
    with np.errstate(over="ignore"):
        for _ in range(tries // chunk):
            k = rng.integers(0, 2**64 - 1, size=chunk, dtype=np.uint64, endpoint=True)
            k = k[mix(k ^ salt_s) <= np.uint64(first)]
            cand.append(k)
        k = np.concatenate(cand)
        low = (mix(k ^ salt_c) | np.uint64(1)) & np.uint64(0xFFFFFFFF)
    order = np.argsort(low, kind="stable")
    ls, ks = low[order], k[order]
    for i in np.nonzero(ls[1:] == ls[:-1])[0]:
        a, b = int(ks[i]), int(ks[i + 1])
        (sa, ra), (sb, rb) = oracle.hash_key(a, 0, m, seed), oracle.hash_key(b, 0, m, seed)
        if sa == sb == 0 and (ra ^ rb) & 0xFFFFFFFF == 0 and ra != rb:
            return a, b
    raise AssertionError("no colliding pair among the candidates")


def test_low_word_collision_takes_the_exact_pass():
    # Two keys start at slot 0 of bucket 0 (of 2) with rows equal in their
    # low 32 bits: one claims slot 0, the other's XOR with it has a zero low
    # word and a nonzero high word, which stops the fast pass; the exact pass
    # must then give the oracle's structure. The other 98 keys start later,
    # so slot 0 is empty when the pair arrives.
    n = 100
    m = 128  # 64 * ceil(0.97 * 100 / 64): two buckets, one range
    a, b = _low_word_pair(m, 0)
    rng = np.random.default_rng(7)
    others = []
    while len(others) < n - 2:
        k = int(rng.integers(0, 2**63))
        if oracle.hash_key(k, 0, m, 0)[0] != 0 and k not in (a, b):
            others.append(k)
    keys = np.array([a, b] + others, dtype=np.uint64)
    vals = W.values(n, 8, 31)
    _compare(keys, vals, 8, dict(ranges=1), "low-word pair")


@pytest.mark.parametrize("n,r,kw", [
    (120_000, 8, dict(ranges=16, load_num=50, load_den=100, seed=31)),
    (150_000, 16, dict(ranges=1, load_num=60, load_den=100, seed=32)),
    (120_000, 8, dict(ranges=16, load_num=50, load_den=100, seed=33, threshold_mode=1)),
])
def test_overfull_buckets_and_sub_bins(n, r, kw):
    """Two rarely taken kernel paths, reached on purpose: at 0.5-0.6 slots per
    key, layer-0 buckets hold 100-128 keys on average, so the insertion
    kernel must read records past its 127-record LDS stage from the item
    stream, and 64-bucket sub-bins hold more than the 4,608 records the
    level-3 sort stages in LDS, so it takes its two-pass global path."""
    keys = W.keys(n, 3000 + n)
    vals = W.values(n, r, 4000 + n)
    op = oracle.Params(**kw)
    m, B, R = oracle.layer_geometry(op, n)
    per_bucket = np.bincount(oracle.start_buckets(keys, 0, m, op), minlength=B)
    assert per_bucket.max() >= 128, "no bucket exceeds the insertion stage"
    per_sub = np.add.reduceat(per_bucket, np.arange(0, B, 64)) + \
        np.minimum(64, B - np.arange(0, B, 64))  # records + one header per bucket
    assert per_sub.max() > 4608, "no sub-bin exceeds the level-3 LDS block"
    _compare(keys, vals, r, kw, "overfull")


@pytest.mark.parametrize("kw", [
    dict(ranges=64, threshold_mode=1, seed=2),
    dict(ranges=64, minbpt=8, cut_strategy=2, cut_search=50, seed=3),
    dict(ranges=64, minbpt=8, threshold_mode=1, cut_strategy=1, cut_search=10, seed=4),
])
def test_import_roundtrip_of_new_sections(kw):
    # the oracle's export (1+-bit bit words, threshold bytes, cut points)
    # imported by the library answers like the oracle and exports the same bytes
    burr = _burr()
    keys, vals = W.keys(50_000, 61), W.values(50_000, 8, 62)
    ref = oracle.build(keys, vals, 8, oracle.Params(**kw))
    print(f"[parity] import {kw}", flush=True)
    h = burr.import_(ref.export())
    assert h.export() == ref.export()
    q = np.concatenate([keys[:20_000], W.non_members(50_000, 20_000, 63)])
    assert np.array_equal(h.query(_dev(q)).cpu().numpy(), ref.query(q))
    h.free()
