"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the
oracle's tests.

This module holds none of the retrieval method's arithmetic: it only draws
keys, values, query mixes and batch/serving size schedules.

Keys are the SplitMix64 output stream (Steele, Lea, Flood, OOPSLA 2014) of a
seeded counter: output i = mix(seed + (i+1) * golden_gamma). The mix is a
bijection of the counter, so keys drawn from distinct counters of one stream
are distinct; members use counters [0, n), non-members counters >= n.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream seeded with seed."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _signed(x: int) -> int:
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >> 63 else x


def splitmix64_device(seed: int, start: int, count: int, device, chunk: int = 1 << 27):
    """The same stream as splitmix64(), computed with torch int64 arithmetic
    on `device` (products wrap modulo 2^64; right shifts are made logical by
    masking). Returns an int64 tensor holding the u64 bit patterns."""
    import torch
    out = torch.empty(count, dtype=torch.int64, device=device)

    def lsr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    for lo in range(0, count, chunk):
        c = min(chunk, count - lo)
        z = torch.arange(start + lo + 1, start + lo + c + 1, dtype=torch.int64, device=device)
        z = z * _signed(int(_GAMMA)) + _signed(seed)
        z = (z ^ lsr(z, 30)) * _signed(int(_M1))
        z = (z ^ lsr(z, 27)) * _signed(int(_M2))
        out[lo:lo + c] = z ^ lsr(z, 31)
    return out


def keys_device(n: int, seed: int, device, start: int = 0):
    """keys(n, seed, start) generated on `device` (int64 tensor)."""
    return splitmix64_device(seed, start, n, device)


def value_dtype(r: int):
    return np.uint8 if r <= 8 else (np.uint16 if r <= 16 else np.uint32)


def keys(n: int, seed: int, start: int = 0) -> np.ndarray:
    """n distinct uniform 64-bit keys (members use start=0)."""
    return splitmix64(seed, start, n)


def values(n: int, r: int, seed: int) -> np.ndarray:
    """n uniform r-bit values, stored in the narrowest of u8/u16/u32."""
    v = splitmix64(seed, 0, n)
    mask = np.uint64((1 << r) - 1)
    return (v & mask).astype(value_dtype(r))


def non_members(n_members: int, q: int, seed: int) -> np.ndarray:
    """q keys of the same stream that are not among the first n_members."""
    return splitmix64(seed, n_members, q)


def query_mix(n_members: int, q: int, seed: int, key_seed: int,
              member_frac: float = 0.5) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """q queries, each a member (uniform index, with replacement) with
    probability member_frac, else a non-member. Returns (keys, is_member,
    member index or -1)."""
    rng = np.random.default_rng(seed)
    is_mem = rng.random(q) < member_frac
    idx = rng.integers(0, max(n_members, 1), size=q, dtype=np.int64)
    out = np.empty(q, dtype=np.uint64)
    if n_members > 0 and is_mem.any():
        out[is_mem] = _gather_stream(key_seed, idx[is_mem])
    else:
        is_mem[:] = False
    nm = int((~is_mem).sum())
    out[~is_mem] = splitmix64(key_seed, n_members, nm)
    idx[~is_mem] = -1
    return out, is_mem, idx


def _gather_stream(seed: int, idx: np.ndarray) -> np.ndarray:
    """Stream outputs at arbitrary indices without materialising the stream."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def batch_sizes(count: int, seed: int, median: float = 2000.0, lo: int = 100,
                hi: int = 200_000) -> np.ndarray:
    """Log-normal structure sizes (median `median`, sigma sqrt(2 ln 2)),
    clipped to [lo, hi] - the shape of many small perfect-hash buckets."""
    rng = np.random.default_rng(seed)
    s = rng.lognormal(mean=np.log(median), sigma=np.sqrt(2 * np.log(2)), size=count)
    return np.clip(np.rint(s), lo, hi).astype(np.int64)


def serving_sizes(count: int, seed: int, kind: str) -> np.ndarray:
    """Request sizes of the serving workload: builds log-normal with median
    1e5 keys clipped to [1e3, 1e7]; query batches log-normal with median 1e5
    clipped to [1e4, 1e6] (the clip bounds taken as +-3 sigma)."""
    rng = np.random.default_rng(seed)
    if kind == "build":
        s = rng.lognormal(np.log(1e5), np.log(1e4) / 6, size=count)
        return np.clip(np.rint(s), 1_000, 10_000_000).astype(np.int64)
    s = rng.lognormal(np.log(1e5), np.log(100) / 6, size=count)
    return np.clip(np.rint(s), 10_000, 1_000_000).astype(np.int64)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
