"""Pins of the composed hash of the oracle: start slot, coefficient row and
fingerprint (a reading of ours: the paper's ribbon hashing in Sec. 2 names no
function, so parity against the paper stays unpinned for the choice of mixer).

The composition is
  salt_s = fmix64(seed ^ (2*layer+1)), salt_c = fmix64(seed ^ (2*layer+2)),
  s  = floor(fmix64(key ^ salt_s) * (m - 63) / 2^64)   (start in [0, m-64]),
  c  = fmix64(key ^ salt_c) | 1,
  fp = top r bits of fmix64(key ^ fmix64(~seed)).

Two kinds of pins:
  - special cases that reduce the composition to the published finalizer
    alone: fmix64(0) = 0, so a seed equal to 2*layer+1 (2*layer+2, ~0) zeroes
    the start (row, fingerprint) salt, and keys chosen through the exact
    inverse of the finalizer then land on values fixed by arithmetic (the
    largest start m-64, the middle, row 1, fingerprint 2^r-1);
  - an independent recomputation with Python integers, over 10^4 random
    tuples and the checked-in vectors of tests/golden/hash_vectors.txt.
"""
import os
import random

import pytest

import oracle

MASK = (1 << 64) - 1
C1 = 0xFF51AFD7ED558CCD
C2 = 0xC4CEB9FE1A85EC53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hash_vectors.txt")


def _fmix(x: int) -> int:
    # MurmurHash3 fmix64, published steps
    x ^= x >> 33
    x = (x * C1) & MASK
    x ^= x >> 33
    x = (x * C2) & MASK
    return x ^ (x >> 33)


def _unxorshift(y: int, k: int) -> int:
    x = y
    for _ in range(64 // k + 1):
        x = y ^ (x >> k)
    return x & MASK


def _fmix_inv(y: int) -> int:
    y = _unxorshift(y, 33)
    y = (y * pow(C2, -1, 1 << 64)) & MASK
    y = _unxorshift(y, 33)
    y = (y * pow(C1, -1, 1 << 64)) & MASK
    return _unxorshift(y, 33)


def _compose(key, layer, m, seed):
    salt_s = _fmix(seed ^ (2 * layer + 1))
    salt_c = _fmix(seed ^ (2 * layer + 2))
    s = (_fmix(key ^ salt_s) * (m - 63)) >> 64
    c = _fmix(key ^ salt_c) | 1
    return s, c


def _fp(key, r, seed):
    return _fmix(key ^ _fmix(~seed & MASK)) >> (64 - r)


MS = [64, 65, 128, 1000, 970_048, 97_000_000, 970_000_000, (1 << 40) - 5, (1 << 40) + 64]


def test_inverse_is_exact():
    rng = random.Random(1)
    for _ in range(500):
        y = rng.getrandbits(64)
        assert _fmix(_fmix_inv(y)) == y
    assert _fmix(0) == 0 and oracle.fmix64(0) == 0


@pytest.mark.parametrize("layer", [0, 1, 2, 3, 7])
def test_start_salt_zero_reduces_to_the_finalizer(layer):
    seed = 2 * layer + 1  # seed ^ (2*layer+1) = 0, salt_s = fmix64(0) = 0
    top = _fmix_inv(MASK)          # fmix64 = 2^64-1: the largest start
    mid = _fmix_inv(1 << 63)       # fmix64 = 2^63: the middle of the span
    for m in MS:
        assert oracle.hash_key(0, layer, m, seed)[0] == 0
        assert oracle.hash_key(top, layer, m, seed)[0] == m - 64
        assert oracle.hash_key(mid, layer, m, seed)[0] == (m - 63) // 2


@pytest.mark.parametrize("layer", [0, 1, 3])
def test_row_salt_zero_reduces_to_the_finalizer(layer):
    seed = 2 * layer + 2  # salt_c = 0
    assert oracle.hash_key(0, layer, 1 << 20, seed)[1] == 1
    for y in (0xAAAAAAAAAAAAAAAA, 0x8000000000000000, 0x123456789ABCDEF0, MASK):
        key = _fmix_inv(y)
        assert oracle.hash_key(key, layer, 1 << 20, seed)[1] == (y | 1)


def test_fingerprint_salt_zero_reduces_to_the_finalizer():
    seed = MASK  # fmix64(~seed) = fmix64(0) = 0
    for r in (1, 5, 8, 16, 32):
        assert oracle.fingerprint(_fmix_inv(MASK), r, seed) == (1 << r) - 1
        assert oracle.fingerprint(0, r, seed) == 0
        v = 5 % (1 << r)
        assert oracle.fingerprint(_fmix_inv(v << (64 - r)), r, seed) == v


def test_largest_start_at_any_seed():
    rng = random.Random(2)
    for _ in range(300):
        seed, layer = rng.getrandbits(64), rng.randrange(8)
        m = rng.choice(MS)
        key = _fmix_inv(MASK) ^ _fmix(seed ^ (2 * layer + 1))
        assert oracle.hash_key(key, layer, m, seed)[0] == m - 64


def test_independent_recomputation_of_random_tuples():
    rng = random.Random(3)
    for i in range(10_000):
        key = rng.getrandbits(64)
        layer = rng.randrange(0, 33)
        m = MS[i % len(MS)] if i % 2 else rng.randrange(64, 1 << 41)
        seed = rng.getrandbits(64)
        assert oracle.hash_key(key, layer, m, seed) == _compose(key, layer, m, seed)
        if i % 10 == 0:
            for r in (1, 8, 16, 32):
                assert oracle.fingerprint(key, r, seed) == _fp(key, r, seed)


def test_golden_vectors():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        f = line.split()
        key, layer, m, seed = int(f[0], 16), int(f[1]), int(f[2]), int(f[3], 16)
        s, c = int(f[4]), int(f[5], 16)
        fps = [int(x) for x in f[6:10]]
        assert _compose(key, layer, m, seed) == (s, c)
        assert oracle.hash_key(key, layer, m, seed) == (s, c)
        for r, want in zip((1, 8, 16, 32), fps):
            assert _fp(key, r, seed) == want
            assert oracle.fingerprint(key, r, seed) == want
        n += 1
    assert n >= 400
