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

HEADER_FIELDS = ("version", "w", "b", "r", "load_num", "load_den", "final_num", "final_den",
                 "layers", "t_lo", "t_hi", "ranges", "minbpt", "final_attempts",
                 "filter_mode", "built", "threshold_mode", "cut_strategy", "cut_search",
                 "first_layer")


def parse(buf: bytes) -> dict:
    off = 0

    def take(fmt):
        nonlocal off
        v = struct.unpack_from("<" + fmt, buf, off)
        off += struct.calcsize("<" + fmt)
        return v

    (magic,) = take("Q")
    hdr = dict(zip(HEADER_FIELDS, take("20I")))
    hdr["seed"], hdr["n"] = take("2Q")
    r, b = hdr["r"], hdr["b"]
    layers = []
    for li in range(hdr["first_layer"], hdr["built"]):
        start = off
        n, m, R = take("3Q")
        B = m // b
        L = dict(layer=li, n=n, m=m, R=R)
        if hdr["threshold_mode"] == 1:
            bits = take(f"{(B + 63) // 64}Q")
            (K,) = take("Q")
            thr = buf[off:off + K]
            off += (K + 7) // 8 * 8
            T = []
            k = 0
            for beta in range(B):
                if (bits[beta // 64] >> (beta % 64)) & 1:
                    T.append(thr[k] + 1)
                    k += 1
                else:
                    T.append(0)
            assert k == K
            L["thresholds"] = T
            L["K"] = K
        else:
            codes = take(f"{(B + 31) // 32}Q")
            L["codes"] = [(codes[beta // 32] >> (2 * (beta % 32))) & 3 for beta in range(B)]
        L["words"] = take(f"{(m // 64) * r}Q")
        if hdr["cut_strategy"]:
            cw = (R - 1 + 1) // 2
            cuts = take(f"{2 * cw}I")
            L["cuts"] = list(cuts[:R - 1])
        L["bytes"] = buf[start:off]
        layers.append(L)
    start = off
    fn, fm, fa = take("3Q")
    fwords = take(f"{(fm // 64) * r}Q")
    fin = dict(n=fn, m=fm, attempt=fa, words=fwords, bytes=buf[start:off])
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
