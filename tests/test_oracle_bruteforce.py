"""Brute-force pins of the oracle's construction on tiny inputs.

For every layer the thresholds are recomputed from their definition - the
smallest of the four 2-bit threshold values (at least the one forced by the
range end) for which the kept equations so far plus the bucket's keys at or
above it form a consistent GF(2) system - with dense Gaussian elimination on
the whole layer (no ranges, no band, no chunks). The solution is the dense
solution of the kept equations with free columns zero, the bump set is the set
of keys below their bucket's threshold, and the final layer's attempt is the
first table size whose dense system is consistent.
"""
import bisect
import random

import numpy as np
import pytest

import oracle
from paper_2411_12365_amd import workload as W
from tests import gf2

WIDTH = 64


def _ceil_div(a, b):
    return -(-a // b)


def layer_geometry(p: oracle.Params, n: int):
    m = p.bucket * max(1, _ceil_div(n * p.load_num, p.load_den * p.bucket))
    B = m // p.bucket
    R = max(1, min(p.ranges, B // max(p.minbpt, 2)))
    first = [rho * B // R for rho in range(R + 1)]
    return m, B, R, first


def thresholds(p: oracle.Params):
    """Allowed threshold values: four with 2-bit thresholds (Sec. 2), every
    offset 0..b with 1+-bit thresholds (an exact value per bumped bucket)."""
    if p.threshold_mode == 1:
        return list(range(p.bucket + 1))
    return [0, p.t_lo, p.t_hi, p.bucket]


def forced_threshold(p, starts, beta):
    """Smallest allowed threshold above every offset of a key of bucket beta
    whose row would cross the end of a range ending with beta (0 if none)."""
    end = (beta + 1) * p.bucket
    forced = [s - beta * p.bucket for s in starts if s > end - WIDTH]
    if not forced:
        return 0
    return min(t for t in thresholds(p) if t > max(forced))


def brute_cuts(p, starts_by_bucket, B, R):
    """First bucket of every range (and B): the equal split, or, with a cut
    strategy, each cut moved within its window to the bucket that the
    strategy's score prefers (Sec. 3 "Selecting Cut Points"), computed here
    from the start slots directly."""
    first = [rho * B // R for rho in range(R + 1)]
    if p.cut_strategy == 0 or p.cut_search < 2 or R < 2:
        return first
    h = min(p.cut_search // 2, max(0, (B // R - 2) // 2))
    if h == 0:
        return first
    all_starts = sorted(s for bk in starts_by_bucket for s in bk)
    out = [0]

    def keys_in(lo, hi):  # keys with start slot in [lo, hi)
        return bisect.bisect_left(all_starts, hi) - bisect.bisect_left(all_starts, lo)

    for rho in range(R - 1):
        b0 = first[rho + 1] - 1
        best = None
        for beta in range(b0 - h, b0 + h + 1):
            T = forced_threshold(p, starts_by_bucket[beta], beta)
            bumped = sum(1 for s in starts_by_bucket[beta] if s - beta * p.bucket < T)
            prev = keys_in(beta * p.bucket - (WIDTH - 1), beta * p.bucket)
            score = {1: bumped, 2: -prev, 3: bumped - prev}[p.cut_strategy]
            key = (score, abs(beta - b0), beta)
            if best is None or key < best[0]:
                best = (key, beta)
        out.append(best[1] + 1)
    out.append(B)
    return out


def final_slots(p: oracle.Params, n: int, a: int) -> int:
    num = n * (p.final_num * 10 + a * p.final_den)
    return WIDTH * max(1, _ceil_div(num, p.final_den * 10 * WIDTH))


def brute_layer(keys, vals, layer, p: oracle.Params):
    n = len(keys)
    m, B, R, _ = layer_geometry(p, n)
    theta = thresholds(p)
    eq = []
    for k, v in zip(keys, vals):
        s, c = oracle.hash_key(int(k), layer, m, p.seed)
        eq.append((s, c << s, int(v), int(k)))
    by_bucket = [[] for _ in range(B)]
    for e in eq:
        by_bucket[e[0] // p.bucket].append(e)
    first = brute_cuts(p, [[e[0] for e in bk] for bk in by_bucket], B, R)
    range_of = np.searchsorted(first, np.arange(B), side="right") - 1
    kept_rows, kept_rhs = [], []
    codes, bumped = [], []
    for beta in range(B):
        members = by_bucket[beta]
        rho = int(range_of[beta])
        tf = 0
        if rho < R - 1 and beta == first[rho + 1] - 1:
            tf = forced_threshold(p, [e[0] for e in members], beta)
        T = None
        for t in theta:
            if t < tf:
                continue
            sel = [e for e in members if e[0] - beta * p.bucket >= t]
            if gf2.consistent(kept_rows + [e[1] for e in sel], kept_rhs + [e[2] for e in sel]):
                T = t
                break
        assert T is not None
        codes.append(T if p.threshold_mode == 1 else theta.index(T))
        for e in members:
            if e[0] - beta * p.bucket >= T:
                kept_rows.append(e[1])
                kept_rhs.append(e[2])
            else:
                bumped.append(e[3])
    Z = gf2.solve(kept_rows, kept_rhs, m)
    assert Z is not None and gf2.check(kept_rows, kept_rhs, Z)
    return dict(m=m, B=B, R=R, codes=codes, Z=Z, bumped=bumped,
                cut_last=[f - 1 for f in first[1:]])


def brute_final(keys, vals, p: oracle.Params):
    n = len(keys)
    if n == 0:
        return dict(m=0, attempt=0, Z=[])
    for a in range(p.final_attempts):
        m = final_slots(p, n, a)
        rows, rhs = [], []
        for k, v in zip(keys, vals):
            s, c = oracle.hash_key(int(k), p.layers, m, p.seed)
            rows.append(c << s)
            rhs.append(int(v))
        Z = gf2.solve(rows, rhs, m)
        if Z is not None:
            return dict(m=m, attempt=a, Z=Z)
    return None


CASES = [
    # n, r, params
    (200, 8, dict(ranges=1)),
    (300, 3, dict(ranges=3, minbpt=2)),
    (1000, 8, dict(ranges=4, minbpt=2)),
    (600, 1, dict(ranges=8, minbpt=2, seed=77)),
    (800, 6, dict(bucket=128, t_lo=32, t_hi=64, ranges=3, minbpt=2)),
    (700, 5, dict(ranges=5, minbpt=2, filter_mode=1, seed=5)),
    (900, 4, dict(ranges=6, minbpt=2, load_num=80, load_den=100, layers=4)),
    (500, 8, dict(layers=0, ranges=1)),
    (1200, 12, dict(ranges=3, minbpt=3, t_lo=8, t_hi=40, seed=123)),
    (64, 2, dict(ranges=1)),
    (1, 8, dict(ranges=4)),
    # heavily overloaded with r = 1: half of the eliminated rows are redundant
    (800, 1, dict(load_num=60, load_den=100, ranges=2, minbpt=2, seed=3)),
    # 1+-bit thresholds (any offset 0..b): one range, several, bucket 128, overloaded
    (1000, 8, dict(ranges=1, threshold_mode=1)),
    (1200, 5, dict(ranges=4, minbpt=2, threshold_mode=1, seed=21)),
    (900, 3, dict(bucket=128, t_lo=32, t_hi=64, ranges=3, minbpt=2, threshold_mode=1)),
    (800, 1, dict(load_num=70, load_den=100, ranges=3, minbpt=2, threshold_mode=1, seed=8)),
    # searched cut points, each strategy, with both threshold modes
    (1500, 8, dict(ranges=3, minbpt=2, cut_strategy=1, cut_search=50, seed=31)),
    (1500, 8, dict(ranges=3, minbpt=2, cut_strategy=2, cut_search=50, seed=32)),
    (1500, 6, dict(ranges=3, minbpt=2, cut_strategy=3, cut_search=4, seed=33)),
    (1500, 4, dict(ranges=4, minbpt=2, cut_strategy=2, cut_search=50, threshold_mode=1,
                   load_num=90, load_den=100, seed=34)),
    (1400, 7, dict(ranges=3, minbpt=2, cut_strategy=3, cut_search=50, threshold_mode=1,
                   seed=35)),
    (2000, 8, dict(ranges=2, minbpt=2, threshold_mode=1, load_num=90, load_den=100, seed=41)),
]


@pytest.mark.parametrize("n,r,kw", CASES)
def test_layers_match_dense_definition(n, r, kw):
    p = oracle.Params(**kw)
    keys = W.keys(n, 1000 + n)
    vals = W.values(n, r, 2000 + n)
    ref = oracle.build(keys, None if p.filter_mode else vals, r, p)
    cur_k = [int(k) for k in keys]
    if p.filter_mode:
        cur_v = [oracle.fingerprint(k, r, p.seed) for k in cur_k]
    else:
        cur_v = [int(v) for v in vals]
    for layer in range(ref.layers_built):
        got_keys = sorted(int(k) for k in ref.layer_keys(layer))
        assert got_keys == sorted(cur_k)
        bl = brute_layer(cur_k, cur_v, layer, p)
        info = ref.layer_info(layer)
        assert (info["m"], info["nbuckets"], info["nranges"]) == (bl["m"], bl["B"], bl["R"])
        assert list(ref.layer_codes(layer)) == bl["codes"]
        assert [int(c) for c in ref.layer_cuts(layer)] == bl["cut_last"]
        assert [int(z) for z in ref.layer_solution(layer)] == bl["Z"]
        assert info["bumped"] == len(bl["bumped"])
        vmap = dict(zip(cur_k, cur_v))
        cur_k = bl["bumped"]
        cur_v = [vmap[k] for k in cur_k]
    if ref.layers_built < p.layers:
        assert cur_k == []
    fin = ref.final_info()
    assert sorted(int(k) for k in ref.layer_keys(ref.layers_built)) == sorted(cur_k)
    bf = brute_final(cur_k, cur_v, p)
    assert (fin["m"], fin["attempt"]) == (bf["m"], bf["attempt"])
    assert [int(z) for z in ref.layer_solution(ref.layers_built)] == bf["Z"]


def boundary_edge_keys(seed: int = 0):
    """320 keys for a 640-slot layer 0 (twice as many slots as keys, so no
    bucket conflicts) of 10 buckets in 2 ranges, whose keys in range 0's last
    bucket (slots 256..319, range end 320) start only at slot 256 (offset 0:
    the row ends exactly at the range end) or 257 (offset 1: it would cross)."""
    out, at256, at257 = [], 0, 0
    start = 0
    while len(out) < 320:
        for k in W.keys(4096, 4242, start=start):
            if len(out) == 320:
                break
            s, _ = oracle.hash_key(int(k), 0, 640, seed)
            if 256 <= s < 320:
                if s == 256 and at256 < 3:
                    at256 += 1
                elif s == 257 and at257 < 2:
                    at257 += 1
                else:
                    continue
            elif len(out) >= 320 - (2 - at257) - (3 - at256):
                continue
            out.append(int(k))
        start += 4096
    assert at256 == 3 and at257 == 2
    return np.array(out, dtype=np.uint64)


def test_boundary_edge_case():
    keys = boundary_edge_keys()
    vals = W.values(len(keys), 8, 5)
    p = oracle.Params(ranges=2, minbpt=2, load_num=200, load_den=100)
    ref = oracle.build(keys, vals, 8, p)
    bl = brute_layer([int(k) for k in keys], [int(v) for v in vals], 0, p)
    assert (bl["m"], bl["R"]) == (640, 2)
    # the offset-1 keys force threshold t_lo on bucket 4, bumping offsets 0 and
    # 1; no other bucket bumps anything at this load
    assert bl["codes"] == [0, 0, 0, 0, 1, 0, 0, 0, 0, 0]
    assert list(ref.layer_codes(0)) == bl["codes"]
    assert sorted(int(k) for k in ref.layer_keys(1)) == sorted(bl["bumped"])
    assert [int(z) for z in ref.layer_solution(0)] == bl["Z"]


def test_equal_duplicates_are_redundant_equations():
    # a repeated key with the same value reduces to 0 = 0: it is kept and
    # consumes no slot, exactly like in the dense system
    keys = W.keys(900, 71)
    vals = W.values(900, 8, 72)
    dk = np.concatenate([keys, keys[::7]])
    dv = np.concatenate([vals, vals[::7]])
    p = oracle.Params(ranges=3, minbpt=2, layers=2)
    ref = oracle.build(dk, dv, 8, p)
    bl = brute_layer([int(k) for k in dk], [int(v) for v in dv], 0, p)
    assert list(ref.layer_codes(0)) == bl["codes"]
    assert [int(z) for z in ref.layer_solution(0)] == bl["Z"]
    assert ref.layer_info(0)["redundant"] > 0
    assert (ref.query(dk) == dv).all()


def test_final_layer_scale_up_attempts():
    # a final layer at 1.0 slots per key almost always fails first; the
    # attempt index must be the first size whose dense system is consistent
    p = oracle.Params(layers=0, final_num=100, final_den=100)
    seen = set()
    for seed in range(6):
        keys = W.keys(640, 50 + seed)
        vals = W.values(640, 8, 60 + seed)
        ref = oracle.build(keys, vals, 8, p)
        bf = brute_final([int(k) for k in keys], [int(v) for v in vals], p)
        fin = ref.final_info()
        assert (fin["m"], fin["attempt"]) == (bf["m"], bf["attempt"])
        seen.add(fin["attempt"])
    assert max(seen) >= 1


def test_load_two_reduces_to_plain_ribbon():
    # with twice as many slots as keys nothing is bumped (w.h.p.) and the
    # layer is the dense solution of all equations
    p = oracle.Params(load_num=200, load_den=100, ranges=1)
    keys = W.keys(1500, 31)
    vals = W.values(1500, 8, 32)
    ref = oracle.build(keys, vals, 8, p)
    assert ref.layers_built == 1
    assert (ref.layer_codes(0) == 0).all()
    m = ref.layer_info(0)["m"]
    rows, rhs = [], []
    for k, v in zip(keys, vals):
        s, c = oracle.hash_key(int(k), 0, m, p.seed)
        rows.append(c << s)
        rhs.append(int(v))
    assert [int(z) for z in ref.layer_solution(0)] == gf2.solve(rows, rhs, m)


def test_gf2_helper_catches_planted_errors():
    # the dense helper itself: random consistent systems are solved, a
    # flipped right-hand side of a dependent row is reported inconsistent
    rng = random.Random(1)
    for _ in range(50):
        m = 40
        Zt = [rng.getrandbits(4) for _ in range(m)]
        rows = [rng.getrandbits(m) | 1 for _ in range(30)]

        def rhs_of(row):
            acc = 0
            for j in range(m):
                if (row >> j) & 1:
                    acc ^= Zt[j]
            return acc
        rhs = [rhs_of(rw) for rw in rows]
        Z = gf2.solve(rows, rhs, m)
        assert Z is not None and gf2.check(rows, rhs, Z)
        dep = rows[0] ^ rows[1]
        assert gf2.consistent(rows + [dep], rhs + [rhs[0] ^ rhs[1]])
        assert not gf2.consistent(rows + [dep], rhs + [rhs[0] ^ rhs[1] ^ 1])


CUT_CASES = [
    (200_000, dict(ranges=2000, minbpt=8, cut_strategy=1, cut_search=50)),
    (200_000, dict(ranges=2000, minbpt=8, cut_strategy=2, cut_search=50)),
    (200_000, dict(ranges=1000, minbpt=8, cut_strategy=3, cut_search=50, threshold_mode=1)),
    (150_000, dict(ranges=500, minbpt=8, cut_strategy=2, cut_search=6, seed=9)),
    (100_000, dict(ranges=60, minbpt=2, cut_strategy=3, cut_search=50, bucket=128, t_lo=32,
                   t_hi=64)),
]


@pytest.mark.parametrize("n,kw", CUT_CASES)
def test_cut_points_match_definition(n, kw):
    """The cut points alone (they depend only on start slots and forced
    thresholds), at sizes too large for the dense check: every layer-0 cut
    of the oracle equals the one the strategy's definition picks."""
    p = oracle.Params(**kw)
    keys = W.keys(n, 77 + n % 13)
    ref = oracle.build(keys, W.values(n, 4, 5), 4, p)
    m, B, R, first = layer_geometry(p, n)
    starts = [[] for _ in range(B)]
    for k in keys.tolist():
        s, _ = oracle.hash_key(k, 0, m, p.seed)
        starts[s // p.bucket].append(s)
    want = [f - 1 for f in brute_cuts(p, starts, B, R)[1:]]
    got = [int(c) for c in ref.layer_cuts(0)]
    assert got == want
    assert sum(a != b for a, b in zip(got, [f - 1 for f in first[1:]])) > R // 4
