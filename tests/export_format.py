"""Independent reader of the canonical export layout (version 2), shared by
the oracle's layout tests and the GPU tests that compare sections of
exports (e.g. the deeper layers of a large structure against the oracle
built from that layer on).

Layout (little endian):
  u64 magic "BuRRexp1"; u32 x 20: version, w, b, r, load_num, load_den,
  final_num, final_den, layers, t_lo, t_hi, ranges, minbpt, final_attempts,
  filter_mode, layers_built, threshold_mode, cut_strategy, cut_search,
  first_layer; u64 seed; u64 n
  per BuRR layer first_layer .. layers_built-1: u64 n, m, R; thresholds
  (2-bit: ceil(B/32) words of 2-bit codes; 1+-bit: ceil(B/64) bit words,
  u64 K, ceil(K/8) words of K threshold-minus-1 bytes); (m/64)*r solution
  words; with a cut strategy ceil((R-1)/2) words of u32 last buckets
  final: u64 n, m, attempt; (m/64)*r solution words
"""
import struct

import numpy as np

HEADER_FIELDS = ("version", "w", "b", "r", "load_num", "load_den", "final_num", "final_den",
                 "layers", "t_lo", "t_hi", "ranges", "minbpt", "final_attempts",
                 "filter_mode", "built", "threshold_mode", "cut_strategy", "cut_search",
                 "first_layer")


def parse(buf: bytes) -> dict:
    """Sections as numpy views of buf (no copies: exports of a billion keys
    are gigabytes): per layer codes or thresholds (uint8 per bucket), words
    (uint64), cuts (uint32, with a cut strategy) and `bytes`, a memoryview of
    the layer's whole section; the final layer likewise."""
    mv = memoryview(buf)
    off = 0

    def take(fmt):
        nonlocal off
        v = struct.unpack_from("<" + fmt, buf, off)
        off += struct.calcsize("<" + fmt)
        return v

    def words(count):
        nonlocal off
        a = np.frombuffer(buf, dtype="<u8", count=count, offset=off)
        off += 8 * count
        return a

    (magic,) = take("Q")
    hdr = dict(zip(HEADER_FIELDS, take("20I")))
    hdr["seed"], hdr["n"] = take("2Q")
    r, b = hdr["r"], hdr["b"]
    layers = []
    for li in range(hdr["first_layer"], hdr["built"]):
        start = off
        n, m, R = take("3Q")
        B = m // b
        idx = np.arange(B, dtype=np.uint64)
        L = dict(layer=li, n=n, m=m, R=R)
        if hdr["threshold_mode"] == 1:
            bits = words((B + 63) // 64)
            (K,) = take("Q")
            thr = np.frombuffer(buf, dtype=np.uint8, count=K, offset=off)
            off += (K + 7) // 8 * 8
            set_ = ((bits[idx >> np.uint64(6)] >> (idx & np.uint64(63))) & np.uint64(1)).astype(bool)
            assert int(set_.sum()) == K
            T = np.zeros(B, dtype=np.uint16)
            T[set_] = thr.astype(np.uint16) + 1
            L["thresholds"] = T
            L["K"] = K
        else:
            cw = words((B + 31) // 32)
            L["codes"] = ((cw[idx >> np.uint64(5)] >> ((idx & np.uint64(31)) * np.uint64(2)))
                          & np.uint64(3)).astype(np.uint8)
        L["words"] = words((m // 64) * r)
        if hdr["cut_strategy"]:
            cw = R // 2  # ceil((R - 1) / 2) words of u32
            L["cuts"] = np.frombuffer(buf, dtype="<u4", count=2 * cw, offset=off)[:R - 1]
            off += 8 * cw
        L["bytes"] = mv[start:off]
        layers.append(L)
    start = off
    fn, fm, fa = take("3Q")
    fwords = words((fm // 64) * r)
    fin = dict(n=fn, m=fm, attempt=fa, words=fwords, bytes=mv[start:off])
    assert off == len(buf), (off, len(buf))
    return dict(magic=magic, header=hdr, layers=layers, final=fin)


def structure_bytes(buf: bytes) -> int:
    """Bytes a query needs: header and every layer's thresholds and solution
    words (the cut points of a searched split are build metadata)."""
    e = parse(buf)
    total = len(buf)
    for L in e["layers"]:
        if "cuts" in L:
            total -= (len(L["cuts"]) + 1) // 2 * 8
    return total
