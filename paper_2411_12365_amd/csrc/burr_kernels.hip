// burr_kernels.hip - HIP kernels of the BuRR library for gfx950 (CDNA4).
//
// Per layer (Sec. 2 and Sec. 3 of the paper):
//   sort      : partition of the keys by (bucket, chunk) in up to three
//               levels (bins, 64-bucket sub-bins, then (bucket, chunk) inside
//               a sub-bin), each writing contiguous runs ordered in LDS; the
//               output is the item stream (a header per bucket + 16-byte
//               records: key, value, offset, chunk)
//   solve     : one wave per range; the lanes insert a bucket's records
//               together (banded GF(2) elimination against a 128-row ring in
//               LDS, claims by compare-and-swap), bucket by bucket, thresholds
//               from chunk prefixes (2-bit) or by bisection (1+-bit), forced
//               bumps at range ends
//   backsub   : a group of lanes per range, one lane per value column,
//               column-interleaved output words
//   gather    : bumped keys (a suffix of every bucket) -> next layer input
//   query     : one lane per key, layer walk, two-word window, popcount parity
#include "burr_kernels.h"

namespace burr {

// ---------------------------------------------------------------------------
// Block-wide exclusive scan (DPP wave scan + LDS totals)
// ---------------------------------------------------------------------------
// Inclusive sum over a wave's 64 lanes with DPP moves, which read a
// neighbour lane's register within the VALU instruction (no LDS crossbar
// round trip as with __shfl_up): a Hillis-Steele scan inside each row of 16
// lanes (row_shr 1, 2, 4, 8; lanes shifted past their row's start add 0),
// then row 0's total into row 1 and row 2's into row 3 (row_bcast:15), and
// rows 0-1's total into rows 2-3 (row_bcast:31). Every lane must be active.
__device__ inline uint32_t wave_inclusive_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* wsum, uint32_t* total) {
  constexpr int NW = NT / 64;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_sum(x);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    const uint32_t w = lane < (uint32_t)NW ? wsum[lane] : 0u;
    const uint32_t wi = wave_inclusive_sum(w);
    if (lane < (uint32_t)NW) wsum[lane] = wi - w;
    if (lane == (uint32_t)NW - 1 && total) *total = wi;
  }
  __syncthreads();
  uint32_t res = wsum[wid] + inc - x;
  __syncthreads();
  return res;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of u32 (tiles of 2048, recursive on tile sums)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr size_t kScanTile = (size_t)kScanThreads * kScanPer;

// VEC: data is 16-byte aligned, so a thread's 8 words move as two 16-byte
// accesses (one per 4 words) wherever all 8 lie inside [0, n)
template <bool VEC>
__global__ __launch_bounds__(kScanThreads) void k_scan_tile(uint32_t* data, size_t n,
                                                             uint32_t* sums) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t total;
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanPer;
  const bool whole = VEC && base + kScanPer <= n;
  uint32_t v[kScanPer];
  uint32_t tot = 0;
  if (whole) {
    const uint4 a = *reinterpret_cast<const uint4*>(data + base);
    const uint4 b = *reinterpret_cast<const uint4*>(data + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = (base + k < n) ? data[base + k] : 0u;
  }
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) tot += v[k];
  uint32_t run = block_exclusive_scan<kScanThreads>(tot, wsum, &total);
  uint32_t o[kScanPer];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    o[k] = run;
    run += v[k];
  }
  if (whole) {
    *reinterpret_cast<uint4*>(data + base) = make_uint4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<uint4*>(data + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
      if (base + k < n) data[base + k] = o[k];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t* data, size_t n,
                                                            const uint32_t* sums) {
  const uint32_t add = sums[blockIdx.x];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  for (size_t k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (base + k < n) data[base + k] += add;
}

// The same with the tile sums not yet scanned: each workgroup adds up the
// sums of the tiles before it (at most kScanAddTiles of them, read from L2),
// which saves the launch of a scan of the sums
constexpr size_t kScanAddTiles = 2048;
__global__ __launch_bounds__(kScanThreads) void k_scan_add_raw(uint32_t* data, size_t n,
                                                                const uint32_t* sums) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  uint32_t part = 0;
  for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) part += sums[t];
  for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
  if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = part;
  __syncthreads();
  uint32_t add = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) add += wsum[w];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  for (size_t k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (base + k < n) data[base + k] += add;
}

// One workgroup scans up to kScanOneMax words (one launch instead of two
// or three for the small scans): the words move between HBM and LDS
// coalesced, and each thread scans kScanOnePer consecutive words in LDS
// (word i at i + i/32, so that the threads' strided reads hit distinct banks)
// around one block-wide scan of the thread totals.
constexpr int kScanOneThreads = 1024;
constexpr int kScanOnePer = 32;
constexpr size_t kScanOneMax = (size_t)kScanOneThreads * kScanOnePer;
constexpr size_t kScanOneLds = (kScanOneMax + kScanOneMax / 32) * 4;
__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(uint32_t* data, size_t n) {
  __shared__ uint32_t wsum[kScanOneThreads / 64];
  __shared__ uint32_t total;
  extern __shared__ uint32_t buf[];
  const uint32_t nn = (uint32_t)n;
#pragma unroll 8
  for (uint32_t k = 0; k < (uint32_t)kScanOnePer; ++k) {
    const uint32_t i = k * kScanOneThreads + threadIdx.x;
    buf[i + i / 32] = i < nn ? data[i] : 0u;
  }
  __syncthreads();
  const uint32_t base = threadIdx.x * kScanOnePer;
  uint32_t tot = 0;
#pragma unroll 8
  for (uint32_t k = 0; k < (uint32_t)kScanOnePer; ++k) tot += buf[base + k + (base + k) / 32];
  uint32_t run = block_exclusive_scan<kScanOneThreads>(tot, wsum, &total);
#pragma unroll 8
  for (uint32_t k = 0; k < (uint32_t)kScanOnePer; ++k) {
    const uint32_t i = base + k, x = buf[i + i / 32];
    buf[i + i / 32] = run;
    run += x;
  }
  __syncthreads();
#pragma unroll 8
  for (uint32_t k = 0; k < (uint32_t)kScanOnePer; ++k) {
    const uint32_t i = k * kScanOneThreads + threadIdx.x;
    if (i < nn) data[i] = buf[i + i / 32];
  }
}

size_t scan_tmp_words(size_t n) {
  size_t w = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    w += n;
  }
  return w + 1;
}

hipError_t scan_exclusive(uint32_t* data, size_t n, uint32_t* tmp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t tiles = (n + kScanTile - 1) / kScanTile;
  const bool vec = reinterpret_cast<uintptr_t>(data) % 16 == 0;
  if (tiles > 1 && n <= kScanOneMax) {
    (void)hipFuncSetAttribute((const void*)k_scan_one, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kScanOneLds);
    k_scan_one<<<1, kScanOneThreads, kScanOneLds, s>>>(data, n);
    return hipGetLastError();
  }
  if (tiles == 1) {
    if (vec)
      k_scan_tile<true><<<1, kScanThreads, 0, s>>>(data, n, nullptr);
    else
      k_scan_tile<false><<<1, kScanThreads, 0, s>>>(data, n, nullptr);
    return hipGetLastError();
  }
  if (vec)
    k_scan_tile<true><<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
  else
    k_scan_tile<false><<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tiles <= kScanAddTiles) {  // the tile sums are added up where they are used
    k_scan_add_raw<<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
    return hipGetLastError();
  }
  e = scan_exclusive(tmp, tiles, tmp + tiles, s);
  if (e != hipSuccess) return e;
  k_scan_add<<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sorting: three levels, each writing contiguous runs
// ---------------------------------------------------------------------------
// level 1: hash every key (start slot, value), partition into nb1 bins of S
//          sub-bins; each tile of kTile keys is ordered by bin in LDS first,
//          so the writes to a bin are runs of consecutive records
// level 2: per bin, partition into its S sub-bins the same way
// level 3: one workgroup per sub-bin (64 buckets) orders its records by
//          (bucket, chunk) in LDS and writes headers and records as one block
// Intermediate records (16 B): key, value | slot within the bin << 32.
// 4 records per thread: level 1 takes 46 VGPRs for a single structure and
// 66-68 for a batch (8 and 7 waves per SIMD), level 2 takes 38 (8 waves per
// SIMD). A level
// with more than kBigTileDigits digits has tiles of twice as many records,
// so that a tile still gives each digit a run of about 16 or more: level 1
// with twice the threads (at 8 records per thread it would take over 128
// VGPRs; held to 64 VGPRs for two workgroups per CU, it spills and is
// slower), level 2 with 8 records per thread (one 16-wave workgroup per CU)
constexpr int kPartPer = 4;                         // records per thread of a tile
constexpr int kPartPerBig = 8;                      // level 2 with many sub-bins
constexpr int kPart1BigThreads = 1024;              // level 1 with many bins
constexpr uint32_t kBigTileDigits = 128;
constexpr int kPartThreads = 2048 / kPartPer;       // level 1: 2048-key tiles
constexpr int kPart2Threads = 4096 / kPartPer;      // level 2: 4096-key tiles
constexpr uint32_t kTile = kPartThreads * kPartPer;  // level-1 keys per tile
constexpr int kHistPer = 8;  // keys (records) per thread and step of the counting passes
constexpr uint32_t kSubSlots = kSubBuckets * 64;     // slots per sub-bin
constexpr uint32_t kChunk2 = 16384;                  // level-2 keys per workgroup
constexpr int kL3Threads = 512;  // 8 waves: with the 73 KB block, 4 waves per SIMD
constexpr int kL3Per = 9;                            // records per thread held in registers
constexpr uint32_t kL3Cap = kL3Threads * kL3Per;     // items of a sub-bin staged in LDS

// Up to this many sub-bins, level 1 partitions into the sub-bins directly
// (a 2048-key tile still writes runs of 16 or more records per sub-bin) and
// level 2 is skipped.
constexpr uint32_t kSingleLevelSubs = 128;

// Fused counting (plan.H > 0): counting workgroup c covers the keys of the
// cc level-1 workgroups [cc c, cc (c+1)) and counts them per (bin, level-1
// workgroup), which level 1 scatters by, and per (bin, sub-bin) into row c.
// The records level-1 workgroups [cs h, cs (h+1)) write into bin d are
// contiguous; they form level 2's chunk (d, h), whose output position for
// sub-bin s is the number of records of all sub-bins before (d, s) plus
// those of (d, s) in the rows before the chunk's first row c = h cs/cc - a
// prefix over the rows. That replaces level 2's own counting pass over the
// level-1 records. cs is chosen so that a chunk holds about kChunkFused
// records (most of one level-2 tile; twice that with the larger tiles), cc
// so that the counting workgroups fill the device (kCountWgs).
constexpr uint32_t kCountThreads = 1024;
constexpr uint32_t kCountSlicesMax = 32;
constexpr uint32_t kChunkFused = 3800;
constexpr uint32_t kCountWgs = 256;  // one per CU: its counters fill most of a CU's LDS
constexpr uint32_t kCountLdsMax = 112 * 1024;  // one counting workgroup per CU
constexpr uint32_t kColBlock = 32;             // h per block of the prefix over h
__host__ __device__ constexpr uint64_t count_lds_bytes(uint32_t nb1, uint32_t S, uint32_t cs) {
  return ((uint64_t)nb1 * S + (uint64_t)nb1 * cs) * 4;
}

SortPlan plan_sort(uint64_t nkeys, uint64_t nbuckets, uint32_t nstructs) {
  SortPlan p{};
  const uint64_t J = nstructs ? nstructs : 1;
  p.nsub = (uint32_t)((nbuckets + kSubBuckets - 1) / kSubBuckets);
  uint32_t nb = 1;
  if (p.nsub <= kSingleLevelSubs)
    nb = p.nsub;  // one sub-bin per bin
  else
    while ((uint64_t)nb * nb < p.nsub) ++nb;  // about sqrt(nsub) bins of about sqrt(nsub) sub-bins
  if (nb < 1) nb = 1;
  if (nb > kMaxDigits) nb = kMaxDigits;
  p.S = (p.nsub + nb - 1) / nb;
  p.nb1 = (p.nsub + p.S - 1) / p.S;
  uint64_t g = (nkeys + kTile - 1) / kTile;  // up to one workgroup per tile
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  p.G1 = (uint32_t)g;
  p.per_group = (nkeys + p.G1 - 1) / p.G1;
  p.U2 = (uint32_t)(nkeys / kChunk2 + p.nb1 + 1);
  p.invS = 1.0f / (float)p.S;
  // Larger tiles pay only where a tile's records spread over many digits:
  // over every bin (sub-bin) of a large structure, but in a batch of small
  // structures a tile holds few structures and each spans few digits, so
  // its runs are long already and larger tiles cost occupancy (measured).
  // The digits a structure spans, on average:
  const uint64_t span1 = p.nb1 / J, span2 = p.nsub / J < p.S ? p.nsub / J : p.S;
  p.big1 = span1 > kBigTileDigits;
  p.big2 = span2 > kBigTileDigits;
  p.H = 0;
  const uint64_t chunk = (uint64_t)kChunkFused * (p.big2 ? kPartPerBig / kPartPer : 1);
  uint64_t cs = (chunk * p.nb1 + p.per_group / 2) / p.per_group;
  cs = cs < 1 ? 1 : (cs > kCountSlicesMax ? kCountSlicesMax : cs);
  uint32_t cc = (p.G1 + kCountWgs - 1) / kCountWgs;  // counting rows: about kCountWgs
  if (cc > cs) cc = (uint32_t)cs;
  p.cs = (uint32_t)((cs + cc - 1) / cc * cc);  // a multiple of cc
  p.cc = cc;
  if (p.S > 1 && count_lds_bytes(p.nb1, p.S, p.cc) <= kCountLdsMax) {
    p.H = (p.G1 + p.cs - 1) / p.cs;
    p.Hc = (p.G1 + p.cc - 1) / p.cc;
    p.U2 = p.nb1 * p.H;
  }
  return p;
}

uint64_t sort_counts2_words(const SortPlan& sp) {
  if (!sp.H) return (uint64_t)sp.U2 * sp.S + 1;
  const uint64_t nds = (uint64_t)sp.nb1 * sp.S;
  const uint64_t hb = (sp.Hc + kColBlock - 1) / kColBlock;
  return nds * sp.Hc + nds * hb + nds + 1;  // counts per (row, sub-bin), block prefixes, sub-bin starts
}

// LDS counter a[d] += 1 for every calling lane; returns the value before
// this lane's increment (lanes in lane order). When all calling lanes of the
// wave count the same digit - consecutive keys of one small structure of a
// batch fall into one bin or sub-bin - one atomic adds for the whole wave:
// 64 atomics on one address would be applied one after another.
__device__ inline uint32_t lds_count(uint32_t* a, uint32_t d) {
  const uint64_t m = __builtin_amdgcn_ballot_w64(true);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if (__builtin_amdgcn_ballot_w64(d == d0) == m) {
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    uint32_t old = 0;
    if (rank == 0) old = atomicAdd(&a[d0], (uint32_t)__popcll(m));
    return __builtin_amdgcn_readfirstlane(old) + rank;
  }
  return atomicAdd(&a[d], 1u);
}
// lds_count for the keys of a layer of several structures (BATCH), the
// plain atomic for one structure, whose keys spread over every digit
template <bool BATCH>
__device__ inline uint32_t key_count(uint32_t* a, uint32_t d) {
  if constexpr (BATCH)
    return lds_count(a, d);
  else
    return atomicAdd(&a[d], 1u);
}

// Threads walk their keys in increasing index order: the structure of the
// first key is found by binary search, later ones by stepping forward.
struct KeyWalk {
  uint32_t j;
  uint64_t end;   // first key of the next structure
  uint64_t span;  // start positions of structure j
  uint64_t bb;    // first global bucket of structure j
  uint32_t r;     // value bits of structure j
  __device__ KeyWalk(const LayerGeom& g, uint64_t i) {
    j = i < g.nkeys ? find_struct(g.key_off, g.J, i) : 0;
    load(g);
  }
  __device__ void load(const LayerGeom& g) {
    end = g.key_off[j + 1];
    span = g.span[j];
    bb = g.bucket_base[j];
    r = g.rbits[j];
  }
  __device__ void advance(const LayerGeom& g, uint64_t i) {
    while (i >= end) {
      ++j;
      load(g);
    }
  }
};

// The same for a layer of one structure: its geometry is the same for every
// key, held in scalar registers, and there is nothing to walk.
struct OneWalk {
  uint64_t span;
  uint64_t bb = 0;
  uint32_t r;
  __device__ explicit OneWalk(const LayerGeom& g) {
    const uint64_t sp = g.span[0];
    span = (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)sp) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sp >> 32)) << 32;
    r = __builtin_amdgcn_readfirstlane(g.rbits[0]);
  }
  __device__ void advance(const LayerGeom&, uint64_t) {}
};
template <bool ONE>
struct WalkOf {
  using T = KeyWalk;
  __device__ static KeyWalk make(const LayerGeom& g, uint64_t i) { return KeyWalk(g, i); }
};
template <>
struct WalkOf<true> {
  using T = OneWalk;
  __device__ static OneWalk make(const LayerGeom& g, uint64_t) { return OneWalk(g); }
};

// The geometry of the structures a workgroup's keys [lo, hi) belong to,
// staged in LDS when there are at most kWalkCache of them: in a batch of
// small structures a thread crosses a structure every few keys, and a
// crossing then costs LDS reads instead of a round trip to HBM.
constexpr uint32_t kWalkCache = 512;
__host__ __device__ constexpr size_t walk_cache_bytes() { return (size_t)kWalkCache * 28 + 16; }
struct WalkCache {
  uint64_t *end, *span, *bb;  // per cached structure: first key of the next, span, first bucket
  uint32_t *r, *jr;           // value bits; jr[0..1]: first structure, count
};
// mem: 16-byte aligned LDS block of walk_cache_bytes(). Called by every
// thread; false (the same for all) if the structures do not fit.
template <int NT>
__device__ inline bool fill_walk_cache(WalkCache& c, uint32_t* mem, const LayerGeom& g,
                                       uint64_t lo, uint64_t hi) {
  c.end = reinterpret_cast<uint64_t*>(mem);
  c.span = c.end + kWalkCache;
  c.bb = c.span + kWalkCache;
  c.r = reinterpret_cast<uint32_t*>(c.bb + kWalkCache);
  c.jr = c.r + kWalkCache;
  if (threadIdx.x == 0) {
    const uint32_t j0 = find_struct(g.key_off, g.J, lo);
    c.jr[0] = j0;
    c.jr[1] = find_struct(g.key_off, g.J, hi - 1) - j0 + 1;
  }
  __syncthreads();
  const uint32_t j0 = c.jr[0], n = c.jr[1];
  if (n > kWalkCache) return false;
  for (uint32_t t = threadIdx.x; t < n; t += NT) {
    c.end[t] = g.key_off[j0 + t + 1];
    c.span[t] = g.span[j0 + t];
    c.bb[t] = g.bucket_base[j0 + t];
    c.r[t] = g.rbits[j0 + t];
  }
  __syncthreads();
  return true;
}
struct CachedWalk {
  const WalkCache& c;
  uint32_t k;  // cached structure of the current key
  uint64_t end, span, bb;
  uint32_t r;
  // i: the thread's first key, in [lo, hi) of the cache or past hi
  __device__ CachedWalk(const WalkCache& cache, uint64_t i) : c(cache) {
    uint32_t a = 0, b = c.jr[1] - 1;  // first k with end[k] > i (the last if none)
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (c.end[mid] > i) b = mid; else a = mid + 1;
    }
    k = a;
    load();
  }
  __device__ void load() {
    end = c.end[k];
    span = c.span[k];
    bb = c.bb[k];
    r = c.r[k];
  }
  __device__ void advance(const LayerGeom&, uint64_t i) {
    while (i >= end) {
      ++k;
      load();
    }
  }
};

// Level-1 bin of a global slot and the slot's offset within the bin. A bin
// is S sub-bins of kSubSlots slots, so the bin is the global sub-bin index
// (below 2^24, checked when the layer is sorted) divided by S, computed in
// single precision from 1/S rounded on the host: the index and S are exact,
// the rounded product is off by less than one and one integer step corrects
// it (a 64-bit integer division took most of the level-1 kernels' issue).
struct BinSplit {
  uint32_t S;
  float inv;  // 1/S
  __device__ explicit BinSplit(const SortPlan& sp) : S(sp.S), inv(sp.invS) {}
  __device__ uint32_t bin(uint64_t slot, uint32_t& in_bin) const {
    const uint32_t gsb = (uint32_t)(slot / kSubSlots);
    uint32_t d = (uint32_t)((float)gsb * inv);
    if (d * S > gsb)
      --d;
    else if ((d + 1) * S <= gsb)
      ++d;
    in_bin = (gsb - d * S) * kSubSlots + (uint32_t)(slot % kSubSlots);
    return d;
  }
};

// Block-wide exclusive scan of n <= kMaxDigits counters in LDS (in place);
// a[n] receives the total.
template <int NT = kPartThreads>
__device__ inline void lds_scan(uint32_t* a, uint32_t n, uint32_t* wsum) {
  constexpr uint32_t per = (kMaxDigits + NT - 1) / NT;
  uint32_t loc[per];
  uint32_t tot = 0;
  const uint32_t base = threadIdx.x * per;
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    loc[k] = base + k < n ? a[base + k] : 0u;
    tot += loc[k];
  }
  __syncthreads();
  uint32_t total;
  uint32_t run = block_exclusive_scan<NT>(tot, wsum, wsum + NT / 64);
  total = wsum[NT / 64];
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    if (base + k < n) a[base + k] = run;
    run += loc[k];
  }
  if (threadIdx.x == 0) a[n] = total;
  __syncthreads();
}

// Level 1, pass 1: per workgroup, keys per bin.
template <bool ONE>
__global__ __launch_bounds__(kPartThreads) void k_p1_hist(const uint64_t* __restrict__ keys,
                                                          LayerGeom g, SortPlan sp,
                                                          uint32_t* __restrict__ counts) {
  extern __shared__ __align__(16) uint32_t hist[];  // nb1 counters, then (batches) the walk cache
  for (uint32_t i = threadIdx.x; i < sp.nb1; i += kPartThreads) hist[i] = 0;
  __syncthreads();
  const uint64_t lo = (uint64_t)blockIdx.x * sp.per_group;
  const uint64_t hi = lo + sp.per_group < g.nkeys ? lo + sp.per_group : g.nkeys;
  const BinSplit bs(sp);
  auto run = [&](auto& w) {
  for (uint64_t t0 = lo; t0 < hi; t0 += kHistPer * kPartThreads) {
    // all of a thread's loads are issued before the first is used (past
    // the end, the last key is read again and not counted)
    uint64_t kk[kHistPer];
#pragma unroll
    for (int k = 0; k < kHistPer; ++k) {
      const uint64_t i = t0 + threadIdx.x + (uint64_t)k * kPartThreads;
      kk[k] = keys[i < hi ? i : hi - 1];
    }
#pragma unroll
    for (int k = 0; k < kHistPer; ++k) {
      const uint64_t i = t0 + threadIdx.x + (uint64_t)k * kPartThreads;
      if (i < hi) {
        w.advance(g, i);
        const uint64_t slot = 64 * w.bb + start_of(kk[k], g.salt_s, w.span);
        uint32_t in_bin;
        key_count<!ONE>(hist, bs.bin(slot, in_bin));
      }
    }
  }
  };
  if constexpr (ONE) {
    OneWalk w(g);
    run(w);
  } else {
    WalkCache wc;
    if (lo < hi && fill_walk_cache<kPartThreads>(wc, hist + ((sp.nb1 + 3) & ~3u), g, lo, hi)) {
      CachedWalk w(wc, lo + threadIdx.x);
      run(w);
    } else {
      KeyWalk w(g, lo + threadIdx.x);
      run(w);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < sp.nb1; i += kPartThreads)
    counts[(size_t)i * sp.G1 + blockIdx.x] = hist[i];
}

// Fused counting pass: per (bin, level-1 workgroup) into counts1 ([bin][w]
// layout, as k_p1_hist) and per (bin, sub-bin) into counts2t[h][d*S+s].
template <bool ONE>
__global__ __launch_bounds__(kCountThreads) void k_p1_count(const uint64_t* __restrict__ keys,
                                                            LayerGeom g, SortPlan sp,
                                                            uint32_t* __restrict__ counts1,
                                                            uint32_t* __restrict__ counts2t) {
  extern __shared__ __align__(16) uint32_t sm[];
  const uint32_t nds = sp.nb1 * sp.S;
  uint32_t* h2 = sm;        // per (bin, sub-bin)
  uint32_t* h1 = sm + nds;  // per (bin, slice); then (batches) the walk cache
  for (uint32_t i = threadIdx.x; i < nds + sp.nb1 * sp.cc; i += kCountThreads) sm[i] = 0;
  __syncthreads();
  const BinSplit bs(sp);
  for (uint32_t wl = 0; wl < sp.cc; ++wl) {
    const uint64_t w = (uint64_t)blockIdx.x * sp.cc + wl;
    if (w >= sp.G1) break;
    const uint64_t lo = w * sp.per_group;
    const uint64_t hi = lo + sp.per_group < g.nkeys ? lo + sp.per_group : g.nkeys;
    if (lo >= hi) break;
    auto run = [&](auto& kw) {
    for (uint64_t t0 = lo; t0 < hi; t0 += kHistPer * kCountThreads) {
      uint64_t kk[kHistPer];  // all loads issued before the first is used
#pragma unroll
      for (int k = 0; k < kHistPer; ++k) {
        const uint64_t i = t0 + threadIdx.x + (uint64_t)k * kCountThreads;
        kk[k] = keys[i < hi ? i : hi - 1];
      }
#pragma unroll
      for (int k = 0; k < kHistPer; ++k) {
        const uint64_t i = t0 + threadIdx.x + (uint64_t)k * kCountThreads;
        if (i < hi) {
          kw.advance(g, i);
          const uint64_t slot = 64 * kw.bb + start_of(kk[k], g.salt_s, kw.span);
          uint32_t in_bin;
          const uint32_t d = bs.bin(slot, in_bin);
          const uint32_t sb = in_bin / kSubSlots;
          key_count<!ONE>(h2, d * sp.S + sb);
          key_count<!ONE>(h1, d * sp.cc + wl);
        }
      }
    }
    };
    if constexpr (ONE) {
      OneWalk kw(g);
      run(kw);
    } else {
      __syncthreads();  // the previous slice's walk is done with the cache
      WalkCache wc;
      if (fill_walk_cache<kCountThreads>(wc, sm + ((nds + sp.nb1 * sp.cc + 3) & ~3u), g, lo, hi)) {
        CachedWalk kw(wc, lo + threadIdx.x);
        run(kw);
      } else {
        KeyWalk kw(g, lo + threadIdx.x);
        run(kw);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < sp.nb1 * sp.cc; i += kCountThreads) {
    const uint32_t d = i / sp.cc;
    const uint64_t w = (uint64_t)blockIdx.x * sp.cc + (i - d * sp.cc);
    if (w < sp.G1) counts1[(size_t)d * sp.G1 + w] = h1[i];
  }
  uint32_t* out = counts2t + (size_t)blockIdx.x * nds;
  for (uint32_t i = threadIdx.x; i < nds; i += kCountThreads) out[i] = h2[i];
}

// Prefix over h of counts2t[h][x] (x = d*S+s), in three steps around a scan
// of the sub-bin totals: block sums over kColBlock consecutive h ...
__global__ __launch_bounds__(256) void k_col_blocksum(const uint32_t* __restrict__ c2t,
                                                      uint32_t nds, uint32_t H,
                                                      uint32_t* __restrict__ psum) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  const uint32_t hb = blockIdx.y;
  if (x >= nds) return;
  const uint32_t h0 = hb * kColBlock;
  const uint32_t h1 = h0 + kColBlock < H ? h0 + kColBlock : H;
  uint32_t v[kColBlock];
#pragma unroll
  for (uint32_t k = 0; k < kColBlock; ++k)
    v[k] = h0 + k < h1 ? c2t[(size_t)(h0 + k) * nds + x] : 0u;
  uint32_t t = 0;
#pragma unroll
  for (uint32_t k = 0; k < kColBlock; ++k) t += v[k];
  psum[(size_t)hb * nds + x] = t;
}
// ... block sums to exclusive block prefixes, sub-bin totals to tot[x] ...
__global__ __launch_bounds__(256) void k_col_blockbase(uint32_t* __restrict__ psum, uint32_t nds,
                                                       uint32_t HB, uint32_t* __restrict__ tot) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  if (x >= nds) return;
  uint32_t run = 0;
  for (uint32_t hb = 0; hb < HB; ++hb) {
    const uint32_t t = psum[(size_t)hb * nds + x];
    psum[(size_t)hb * nds + x] = run;
    run += t;
  }
  tot[x] = run;
}
// ... and, once tot holds each sub-bin's start, every count to the output
// position of chunk (d, h) in sub-bin (d, s); tot[nds] = nkeys.
__global__ __launch_bounds__(256) void k_col_apply(uint32_t* __restrict__ c2t, uint32_t nds,
                                                   uint32_t H, const uint32_t* __restrict__ psum,
                                                   uint32_t* __restrict__ tot, uint32_t nkeys) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  const uint32_t hb = blockIdx.y;
  if (x == 0 && hb == 0) tot[nds] = nkeys;
  if (x >= nds) return;
  const uint32_t h0 = hb * kColBlock;
  const uint32_t h1 = h0 + kColBlock < H ? h0 + kColBlock : H;
  uint32_t v[kColBlock];
#pragma unroll
  for (uint32_t k = 0; k < kColBlock; ++k)
    v[k] = h0 + k < h1 ? c2t[(size_t)(h0 + k) * nds + x] : 0u;
  uint32_t run = tot[x] + psum[(size_t)hb * nds + x];
#pragma unroll
  for (uint32_t k = 0; k < kColBlock; ++k) {
    if (h0 + k < h1) c2t[(size_t)(h0 + k) * nds + x] = run;
    run += v[k];
  }
}

// Intermediate records of the partition levels. PACKED (every value fits
// 8 bits, every slot within a level-1 bin fits 24): 12 bytes {key low, key
// high, slot | value << 24}, one dwordx3 access; else 16 bytes {key low, key
// high, value, slot}.
template <bool PACKED>
struct PRec {
  using T = uint4;
  __device__ static T make(uint64_t key, uint32_t slot, uint32_t v) {
    return make_uint4((uint32_t)key, (uint32_t)(key >> 32), v, slot);
  }
  __device__ static uint32_t slot(const T& r) { return r.w; }
  __device__ static uint4 unpack(const T& r) { return r; }  // {key lo, key hi, value, slot}
};
template <>
struct PRec<true> {
  using T = uint3;
  __device__ static T make(uint64_t key, uint32_t slot, uint32_t v) {
    return make_uint3((uint32_t)key, (uint32_t)(key >> 32), slot | (v << 24));
  }
  __device__ static uint32_t slot(const T& r) { return r.z & 0xffffffu; }
  __device__ static uint4 unpack(const T& r) {
    return make_uint4(r.x, r.y, r.z >> 24, r.z & 0xffffffu);
  }
};

// Orders one tile of records by digit in LDS and writes every digit's part
// as a run at that digit's cursor (cur[d] advances by the tile's count).
// rec/dr: each thread's PER records and their digit << kRankBits | rank
// within the digit (kNoDigit: none).
constexpr uint32_t kNoDigit = 0xffffffffu;
constexpr uint32_t kRankBits = 13;  // ranks within a tile of at most 8192 records
static_assert(kPart2Threads * kPartPerBig <= (1u << kRankBits), "tile rank bits");
static_assert(kMaxDigits <= (1u << (32 - kRankBits)), "tile digit bits");
template <int NT, int PER, class R>
__device__ inline void tile_write(const R (&rec)[PER], const uint32_t (&dr)[PER], uint32_t D,
                                  uint32_t* cur, uint32_t* toff, R* stage, uint16_t* sdig,
                                  uint32_t* wsum, uint32_t ntile, R* __restrict__ out) {
  lds_scan<NT>(toff, D, wsum);  // tile counts -> tile offsets
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (dr[k] != kNoDigit) {
      const uint32_t d = dr[k] >> kRankBits;
      const uint32_t pos = toff[d] + (dr[k] & ((1u << kRankBits) - 1u));
      stage[pos] = rec[k];
      sdig[pos] = (uint16_t)d;
    }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < ntile; j += NT) {
    const uint32_t d = sdig[j];
    out[cur[d] + (j - toff[d])] = stage[j];
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < D; d += NT) cur[d] += toff[d + 1] - toff[d];
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < D; d += NT) toff[d] = 0;
  __syncthreads();
}

// LDS layout of the partition kernels: cur[D], toff[D+1], wsum, stage, sdig
// (RB: bytes of a record)
template <int NT, int PER>
__host__ __device__ constexpr size_t part_lds_bytes(uint32_t D, size_t RB) {
  return (size_t)(2 * D + 2 + NT / 64 + 2) * 4 + 15 + (size_t)NT * PER * (RB + 2);
}
template <int NT, int PER, class R>
struct PartLds {
  uint32_t *cur, *toff, *wsum;
  R* stage;
  uint16_t* sdig;
  __device__ PartLds(uint32_t* sm, uint32_t D) {
    cur = sm;
    toff = sm + D;
    wsum = toff + D + 2;
    // the stage at the next 16-byte boundary of the (16-byte aligned) block,
    // by pointer arithmetic alone: a pointer that passes through an integer
    // loses its LDS address space, and the stage's accesses then become flat
    // instructions, which wait on the global stores of the tile's write
    const uint32_t w = (2 * D + 2 + NT / 64 + 2 + 3) & ~3u;
    stage = reinterpret_cast<R*>(sm + w);
    sdig = reinterpret_cast<uint16_t*>(stage + NT * PER);
  }
};

// Level 1, pass 2: hash, mask or fingerprint the value, write tile runs per bin.
// Level 1, pass 2, the tiles of a workgroup's keys [lo, hi) (W: how a
// thread finds the structure of its keys)
template <typename VT, bool PACKED, int NT, bool ONE, class W,
          class R = typename PRec<PACKED>::T>
__device__ __forceinline__ void p1_tiles(const uint64_t* __restrict__ keys,
                                         const VT* __restrict__ vals, const LayerGeom& g,
                                         const SortPlan& sp, PartLds<NT, kPartPer, R>& L,
                                         uint64_t lo, uint64_t hi, uint32_t mask_values,
                                         uint32_t filter, uint64_t fp_salt, uint32_t fp_late,
                                         R* __restrict__ out, W& w) {
  constexpr int PER = kPartPer;
  constexpr uint32_t T1 = NT * PER;
  const bool no_vals = filter && (mask_values || fp_late);  // values not read
  const BinSplit bs(sp);
  for (uint64_t t0 = lo; t0 < hi; t0 += T1) {
    R rec[PER];
    uint32_t dr[PER];
    // all of a thread's loads are issued before the first is used (past
    // the end, the last key is read again and not used)
    uint64_t kk[PER];
    uint32_t vv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint64_t i = t0 + threadIdx.x + (uint64_t)k * NT;
      const uint64_t ic = i < hi ? i : hi - 1;
      kk[k] = keys[ic];
      vv[k] = no_vals ? 0u : (uint32_t)vals[ic];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint64_t i = t0 + threadIdx.x + (uint64_t)k * NT;
      dr[k] = kNoDigit;
      if (i < hi) {
        w.advance(g, i);
        const uint64_t key = kk[k];
        uint32_t v;
        if (fp_late)  // fingerprint computed at level 3
          v = 0;
        else if (filter && mask_values)
          v = (uint32_t)(mix64(key ^ fp_salt) >> (64 - w.r));
        else if (mask_values)
          v = vv[k] & (w.r >= 32 ? 0xffffffffu : ((1u << w.r) - 1u));
        else
          v = vv[k];
        const uint64_t slot = 64 * w.bb + start_of(key, g.salt_s, w.span);
        uint32_t in_bin;
        const uint32_t d = bs.bin(slot, in_bin);
        rec[k] = PRec<PACKED>::make(key, in_bin, v);
        dr[k] = d << kRankBits | key_count<!ONE>(L.toff, d);
      }
    }
    const uint32_t ntile = (uint32_t)(hi - t0 < T1 ? hi - t0 : T1);
    __syncthreads();
    tile_write<NT, PER, R>(rec, dr, sp.nb1, L.cur, L.toff, L.stage, L.sdig, L.wsum, ntile, out);
  }
}

template <typename VT, bool PACKED, int NT, bool ONE>
__global__ __launch_bounds__(NT) void k_p1_scatter(
    const uint64_t* __restrict__ keys, const VT* __restrict__ vals, LayerGeom g, SortPlan sp,
    const uint32_t* __restrict__ offs, uint32_t mask_values, uint32_t filter, uint64_t fp_salt,
    uint32_t fp_late, void* __restrict__ out_raw) {
  using R = typename PRec<PACKED>::T;
  extern __shared__ __align__(16) uint32_t sm[];
  constexpr int PER = kPartPer;
  PartLds<NT, PER, R> L(sm, sp.nb1);
  R* out = reinterpret_cast<R*>(out_raw);
  for (uint32_t d = threadIdx.x; d < sp.nb1; d += NT) {
    L.cur[d] = offs[(size_t)d * sp.G1 + blockIdx.x];
    L.toff[d] = 0;
  }
  __syncthreads();
  const uint64_t lo = (uint64_t)blockIdx.x * sp.per_group;
  const uint64_t hi = lo + sp.per_group < g.nkeys ? lo + sp.per_group : g.nkeys;
  if constexpr (ONE) {
    OneWalk w(g);
    p1_tiles<VT, PACKED, NT, ONE>(keys, vals, g, sp, L, lo, hi, mask_values, filter, fp_salt,
                                  fp_late, out, w);
  } else {  // the walk cache after the tile's LDS
    WalkCache wc;
    uint32_t* cmem = sm + (uint32_t)((part_lds_bytes<NT, PER>(sp.nb1, sizeof(R)) + 15) / 16 * 4);
    if (lo < hi && fill_walk_cache<NT>(wc, cmem, g, lo, hi)) {
      CachedWalk w(wc, lo + threadIdx.x);
      p1_tiles<VT, PACKED, NT, ONE>(keys, vals, g, sp, L, lo, hi, mask_values, filter, fp_salt,
                                    fp_late, out, w);
    } else {
      KeyWalk w(g, lo + threadIdx.x);
      p1_tiles<VT, PACKED, NT, ONE>(keys, vals, g, sp, L, lo, hi, mask_values, filter, fp_salt,
                                    fp_late, out, w);
    }
  }
}

// Level 2 plan (one workgroup): bin ranges and level-2 workgroups per bin.
__global__ __launch_bounds__(kPartThreads) void k_p2_plan(const uint32_t* __restrict__ offs1,
                                                          SortPlan sp, uint64_t nkeys,
                                                          uint32_t* __restrict__ binlo,
                                                          uint32_t* __restrict__ nch,
                                                          uint32_t* __restrict__ cbase) {
  __shared__ uint32_t a[kMaxDigits + 1];
  __shared__ uint32_t wsum[kPartThreads / 64 + 2];
  for (uint32_t b = threadIdx.x; b < sp.nb1; b += kPartThreads) {
    const uint32_t lo = offs1[(size_t)b * sp.G1];
    const uint32_t hi = b + 1 < sp.nb1 ? offs1[(size_t)(b + 1) * sp.G1] : (uint32_t)nkeys;
    binlo[b] = lo;
    const uint32_t c = (hi - lo + kChunk2 - 1) / kChunk2;
    nch[b] = c;
    a[b] = c;
  }
  if (threadIdx.x == 0) binlo[sp.nb1] = (uint32_t)nkeys;
  __syncthreads();
  lds_scan(a, sp.nb1, wsum);
  for (uint32_t b = threadIdx.x; b <= sp.nb1; b += kPartThreads) cbase[b] = a[b];
}

// level-2 workgroup -> (bin, chunk, key range); false if unused.
// Called by every thread of the workgroup. The bin is the last b with
// cbase[b] <= wg (cbase is non-decreasing); each wave finds it with 64-way
// rounds, a ballot over 64 evenly spaced entries per round (two rounds for
// up to 4096 bins), so a workgroup waits on three dependent loads before
// its records rather than on one per halving of a binary search.
struct Chunk2 {
  uint32_t b, c, lo, hi, base;  // base: first counts2 entry of the bin
};
__device__ inline bool chunk2_of(uint32_t wg, const SortPlan& sp, const uint32_t* binlo,
                                 const uint32_t* nch, const uint32_t* cbase, Chunk2& ch) {
  const uint32_t used = cbase[sp.nb1];
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t lo = 0, len = sp.nb1;  // the bin is in [lo, lo + len), and cbase[lo] <= wg
  while (len > 1) {
    const uint32_t step = (len + 63) >> 6;
    const uint32_t idx = lo + lane * step;
    const uint64_t ok = __ballot(idx < lo + len && cbase[idx] <= wg);
    const uint32_t k = 63u - (uint32_t)__clzll((long long)ok);  // lane 0 is set
    lo += k * step;
    const uint32_t rest = len - k * step;
    len = step < rest ? step : rest;
  }
  if (wg >= used) return false;
  ch.b = lo;
  ch.c = wg - cbase[lo];
  ch.lo = binlo[lo] + ch.c * kChunk2;
  ch.hi = ch.lo + kChunk2 < binlo[lo + 1] ? ch.lo + kChunk2 : binlo[lo + 1];
  ch.base = cbase[lo] * sp.S;
  (void)nch;
  return true;
}

// Level 2, pass 1: keys per sub-bin of each chunk; counts2 is laid out per
// bin as [sub-bin][chunk] so that one scan gives every run's position.
template <bool PACKED>
__global__ __launch_bounds__(kPart2Threads) void k_p2_hist(const void* __restrict__ in_raw,
                                                          SortPlan sp,
                                                          const uint32_t* __restrict__ binlo,
                                                          const uint32_t* __restrict__ nch,
                                                          const uint32_t* __restrict__ cbase,
                                                          uint32_t* __restrict__ counts) {
  using R = typename PRec<PACKED>::T;
  const R* in = reinterpret_cast<const R*>(in_raw);
  extern __shared__ uint32_t hist[];
  Chunk2 ch;
  if (!chunk2_of(blockIdx.x, sp, binlo, nch, cbase, ch)) return;
  for (uint32_t i = threadIdx.x; i < sp.S; i += kPart2Threads) hist[i] = 0;
  __syncthreads();
  constexpr uint32_t T2 = kPart2Threads * kHistPer;
  for (uint32_t t0 = ch.lo; t0 < ch.hi; t0 += T2) {
    // loads first (unconditional: past the end the last record is read
    // again and not counted), then the counting atomics
    uint32_t sl[kHistPer];
#pragma unroll
    for (int k = 0; k < kHistPer; ++k) {
      const uint32_t i = t0 + threadIdx.x + k * kPart2Threads;
      const uint32_t ic = i < ch.hi ? i : ch.hi - 1;
      sl[k] = PACKED ? in[ic].z : reinterpret_cast<const uint4*>(in)[ic].w;
    }
#pragma unroll
    for (int k = 0; k < kHistPer; ++k)
      if (PACKED) sl[k] &= 0xffffffu;
#pragma unroll
    for (int k = 0; k < kHistPer; ++k)
      if (t0 + threadIdx.x + k * kPart2Threads < ch.hi) lds_count(hist, sl[k] / kSubSlots);
  }
  __syncthreads();
  const uint32_t nc = nch[ch.b];
  for (uint32_t i = threadIdx.x; i < sp.S; i += kPart2Threads)
    counts[ch.base + i * nc + ch.c] = hist[i];
}

// Level 2, pass 2: tile runs per sub-bin. FUSED (plan.H > 0): workgroup
// d*H + h takes chunk (d, h), the run level-1 workgroups [cs h, cs (h+1))
// wrote into bin d (offs1: the scanned level-1 counts), and its sub-bin
// positions from the prefixed fused counts (offs).
template <bool PACKED, bool FUSED, int PER>
__global__ __launch_bounds__(kPart2Threads) void k_p2_scatter(
    const void* __restrict__ in_raw, SortPlan sp, const uint32_t* __restrict__ binlo,
    const uint32_t* __restrict__ nch, const uint32_t* __restrict__ cbase,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ offs1, uint64_t nkeys,
    void* __restrict__ out_raw) {
  using R = typename PRec<PACKED>::T;
  const R* in = reinterpret_cast<const R*>(in_raw);
  R* out = reinterpret_cast<R*>(out_raw);
  extern __shared__ __align__(16) uint32_t sm[];
  Chunk2 ch;
  PartLds<kPart2Threads, PER, R> L(sm, sp.S);
  if constexpr (FUSED) {
    const uint32_t d = blockIdx.x / sp.H, h = blockIdx.x - d * sp.H;
    const uint32_t w0 = h * sp.cs;
    const uint32_t w1 = w0 + sp.cs < sp.G1 ? w0 + sp.cs : sp.G1;
    ch.lo = offs1[(size_t)d * sp.G1 + w0];
    ch.hi = w1 < sp.G1 ? offs1[(size_t)d * sp.G1 + w1]
          : (d + 1 < sp.nb1 ? offs1[(size_t)(d + 1) * sp.G1] : (uint32_t)nkeys);
    const uint32_t* o = offs + (size_t)h * (sp.cs / sp.cc) * sp.nb1 * sp.S + (size_t)d * sp.S;
    for (uint32_t x = threadIdx.x; x < sp.S; x += kPart2Threads) {
      L.cur[x] = o[x];
      L.toff[x] = 0;
    }
  } else {
    (void)offs1;
    (void)nkeys;
    if (!chunk2_of(blockIdx.x, sp, binlo, nch, cbase, ch)) return;
    const uint32_t nc = nch[ch.b];
    for (uint32_t d = threadIdx.x; d < sp.S; d += kPart2Threads) {
      L.cur[d] = offs[ch.base + d * nc + ch.c];
      L.toff[d] = 0;
    }
  }
  __syncthreads();
  constexpr uint32_t T2 = kPart2Threads * PER;
  for (uint32_t t0 = ch.lo; t0 < ch.hi; t0 += T2) {
    R rec[PER];
    uint32_t dr[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {  // loads first, then the counting atomics
      const uint32_t i = t0 + threadIdx.x + k * kPart2Threads;
      rec[k] = R{};
      if (i < ch.hi) rec[k] = in[i];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t i = t0 + threadIdx.x + k * kPart2Threads;
      dr[k] = kNoDigit;
      if (i < ch.hi) {
        const uint32_t d = PRec<PACKED>::slot(rec[k]) / kSubSlots;
        dr[k] = d << kRankBits | lds_count(L.toff, d);
      }
    }
    const uint32_t ntile = ch.hi - t0 < T2 ? ch.hi - t0 : T2;
    __syncthreads();
    tile_write<kPart2Threads, PER, R>(rec, dr, sp.S, L.cur, L.toff, L.stage, L.sdig, L.wsum,
                                      ntile, out);
  }
}

// First record of every sub-bin (and sstart[nsub] = nkeys).
__global__ void k_p2_starts(SortPlan sp, uint64_t nkeys, const uint32_t* __restrict__ binlo,
                            const uint32_t* __restrict__ nch, const uint32_t* __restrict__ cbase,
                            const uint32_t* __restrict__ offs, uint32_t* __restrict__ sstart) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > sp.nsub) return;
  if (t == sp.nsub) {
    sstart[t] = (uint32_t)nkeys;
    return;
  }
  const uint32_t b = t / sp.S, s = t - b * sp.S;
  sstart[t] = nch[b] ? offs[cbase[b] * sp.S + s * nch[b]] : binlo[b];
}

// Level 3: one workgroup per sub-bin. The item stream holds, per bucket, a
// header and its records ordered by digit - the chunk (2-bit thresholds,
// final layer) or the offset, highest first (1+-bit thresholds); the
// sub-bin's items form one contiguous block starting at item sstart[g] + 64 g.
// The header carries the bucket's record count, its largest offset and its
// number of records at offset 0: the insertion kernel derives the threshold
// forced on a range's last bucket from them, and the cut-point search its
// scores.
// Dynamic LDS: the staged block (kL3Cap items), then the digit counters.
__host__ __device__ constexpr size_t l3_lds_bytes(uint32_t D) {
  return (size_t)kL3Cap * sizeof(uint4) + ((size_t)kSubBuckets * D + 1) * 4;
}
// a level-2 record as {key low, key high, value, slot within the level-1 bin}
template <bool PACKED>
__device__ inline uint4 part_rec(const void* in, uint32_t i) {
  return PRec<PACKED>::unpack(reinterpret_cast<const typename PRec<PACKED>::T*>(in)[i]);
}
template <bool PACKED, uint32_t D>
__global__ __launch_bounds__(kL3Threads) void k_p3_sort(const void* __restrict__ in,
                                                        LayerGeom g, SortPlan sp,
                                                        const uint32_t* __restrict__ sstart,
                                                        Rec* __restrict__ items,
                                                        uint32_t* __restrict__ bstart,
                                                        uint64_t fp_salt, uint32_t fp_bits,
                                                        SortClear cl) {
  __shared__ uint32_t maxoff[kSubBuckets];
  __shared__ uint32_t nzero[kSubBuckets];
  __shared__ uint32_t wsum[kL3Threads / 64 + 2];
  extern __shared__ uint4 stage[];  // kL3Cap items, then the digit counters
  uint32_t* dcur = reinterpret_cast<uint32_t*>(stage + kL3Cap);
  const uint32_t nd = kSubBuckets * D;
  const uint32_t sb = blockIdx.x;
  const uint32_t lo = sstart[sb], hi = sstart[sb + 1], n = hi - lo;
  const uint64_t beta0 = (uint64_t)sb * kSubBuckets;
  const uint32_t nbk = (uint32_t)(g.nbuckets - beta0 < kSubBuckets ? g.nbuckets - beta0 : kSubBuckets);
  const uint32_t sub_in_bin = sb % sp.S;
  const uint32_t slot0 = sub_in_bin * kSubSlots;
  auto digit = [&](uint32_t o) { return D == 3 ? rank_of(o, g) : 63u - o; };
  // the value of an item: from the record, or (fp_bits > 0) the key's
  // fingerprint, which level 1 left out of the record
  auto value = [&](uint32_t klo, uint32_t khi, uint32_t v) {
    const uint64_t key = (uint64_t)klo | (uint64_t)khi << 32;
    return fp_bits ? (uint32_t)(mix64(key ^ fp_salt) >> (64 - fp_bits)) : v;
  };
  for (uint32_t i = threadIdx.x; i < nd; i += kL3Threads) dcur[i] = 0;
  for (uint32_t i = threadIdx.x; i < kSubBuckets; i += kL3Threads) {
    maxoff[i] = 0;
    nzero[i] = 0;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
    for (uint64_t i = (uint64_t)sb * kL3Threads + threadIdx.x; i < cl.n[c];
         i += (uint64_t)gridDim.x * kL3Threads)
      cl.p[c][i] = 0;
  __syncthreads();
  // the block is assembled in LDS when it fits; then every record is read
  // once, into registers, and its rank inside its digit comes from the
  // counting atomic
  const bool fits = n + nbk <= kL3Cap;
  uint4 rec[kL3Per];
  uint32_t dr[kL3Per];  // digit | rank << 12
  if (fits) {
    // loads first, then the counting atomics. The loads are unconditional
    // (past the end the last record is read again and not used): a load
    // under a branch whose record is unpacked inside it waits there for its
    // data, and the loads then run one after another
    using PT = typename PRec<PACKED>::T;
    PT raw[kL3Per];
    if (n) {
#pragma unroll
      for (int k = 0; k < kL3Per; ++k) {
        const uint32_t i = lo + threadIdx.x + k * kL3Threads;
        raw[k] = reinterpret_cast<const PT*>(in)[i < hi ? i : hi - 1];
      }
    }
#pragma unroll
    for (int k = 0; k < kL3Per; ++k) {
      const uint32_t i = lo + threadIdx.x + k * kL3Threads;
      dr[k] = 0xffffffffu;
      if (i < hi) {
        rec[k] = PRec<PACKED>::unpack(raw[k]);
        const uint32_t sl = rec[k].w - slot0;
        const uint32_t bl = sl >> 6, o = sl & 63u;
        const uint32_t d = bl * D + digit(o);
        dr[k] = d | (atomicAdd(&dcur[d], 1u) << 12);
        atomicMax(&maxoff[bl], o);
        if (o == 0) atomicAdd(&nzero[bl], 1u);
      }
    }
  } else {
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kL3Threads) {
      const uint32_t sl = part_rec<PACKED>(in, i).w - slot0;
      const uint32_t bl = sl >> 6, o = sl & 63u;
      atomicAdd(&dcur[bl * D + digit(o)], 1u);
      atomicMax(&maxoff[bl], o);
      if (o == 0) atomicAdd(&nzero[bl], 1u);
    }
  }
  __syncthreads();
  {  // exclusive scan of the digit counts (a thread owns up to 8 consecutive ones)
    constexpr uint32_t kMaxPer = (kSubBuckets * 64 + kL3Threads - 1) / kL3Threads;
    const uint32_t per = (nd + kL3Threads - 1) / kL3Threads;
    const uint32_t base = threadIdx.x * per;
    uint32_t loc[kMaxPer];
    uint32_t tot = 0;
#pragma unroll
    for (uint32_t k = 0; k < kMaxPer; ++k) {
      loc[k] = (k < per && base + k < nd) ? dcur[base + k] : 0u;
      tot += loc[k];
    }
    __syncthreads();
    uint32_t run = block_exclusive_scan<kL3Threads>(tot, wsum, nullptr);
#pragma unroll
    for (uint32_t k = 0; k < kMaxPer; ++k) {
      if (k < per && base + k < nd) dcur[base + k] = run;
      run += loc[k];
    }
    if (threadIdx.x == 0) dcur[nd] = n;
    __syncthreads();
  }
  Rec* gout = items + lo + beta0;
  // headers and bucket starts
  for (uint32_t bl = threadIdx.x; bl < nbk; bl += kL3Threads) {
    const uint32_t first = dcur[D * bl];
    const uint32_t count = dcur[D * bl + D] - first;
    uint32_t c0 = 0, c1 = 0;
    if (D == 3) {
      c0 = dcur[3 * bl + 1] - first;
      c1 = dcur[3 * bl + 2] - dcur[3 * bl + 1];
    }
    bstart[beta0 + bl] = lo + first;
    const uint4 hd = make_uint4(count, maxoff[bl] | (nzero[bl] << 8), c0, c1);
    if (fits)
      stage[first + bl] = hd;
    else
      reinterpret_cast<uint4*>(gout)[first + bl] = hd;
  }
  if (sb + 1 == sp.nsub && threadIdx.x == 0) bstart[g.nbuckets] = (uint32_t)g.nkeys;
  // records: key, value | offset << 32 | rank << 40
  if (fits) {
#pragma unroll
    for (int k = 0; k < kL3Per; ++k) {
      if (dr[k] == 0xffffffffu) continue;
      const uint32_t d = dr[k] & 0xfffu;
      const uint32_t bl = d / D, rk = D == 3 ? d - bl * 3 : 0u;
      const uint32_t o = (rec[k].w - slot0) & 63u;
      stage[dcur[d] + (dr[k] >> 12) + bl + 1] =
          make_uint4(rec[k].x, rec[k].y, value(rec[k].x, rec[k].y, rec[k].z), o | (rk << 8));
    }
    __syncthreads();
    uint4* go = reinterpret_cast<uint4*>(gout);
    for (uint32_t j = threadIdx.x; j < n + nbk; j += kL3Threads) go[j] = stage[j];
    return;
  }
  __syncthreads();
  for (uint32_t i = lo + threadIdx.x; i < hi; i += kL3Threads) {
    const uint4 r = part_rec<PACKED>(in, i);
    const uint32_t sl = r.w - slot0;
    const uint32_t bl = sl >> 6, o = sl & 63u;
    const uint32_t dg = digit(o);
    const uint32_t rk = D == 3 ? dg : 0u;
    const uint32_t pos = atomicAdd(&dcur[bl * D + dg], 1u) + bl + 1;
    reinterpret_cast<uint4*>(gout)[pos] = make_uint4(r.x, r.y, value(r.x, r.y, r.z), o | (rk << 8));
  }
}

template <int V>
struct IntTag {
  static constexpr int value = V;
};
template <bool V>
struct BoolTag {
  static constexpr bool value = V;
};
template <class T>
struct TypeTag {
  using type = T;
};

template <bool PACKED>
hipError_t sort_layer_t(const SortArgs& a, bool fp_late, hipStream_t s) {
  const SortPlan& sp = a.plan;
  const uint64_t n = a.g.nkeys;
  hipError_t e;
  const size_t nds = (size_t)sp.nb1 * sp.S;
  if (sp.H) {  // one counting pass for both partition levels
    const size_t lds = count_lds_bytes(sp.nb1, sp.S, sp.cc);
    if (a.g.J == 1) {
      (void)hipFuncSetAttribute((const void*)k_p1_count<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      k_p1_count<true><<<sp.Hc, kCountThreads, lds, s>>>(a.keys, a.g, sp, a.counts1, a.counts2);
    } else {  // + the walk cache
      const size_t ldsw = (lds + 15) / 16 * 16 + walk_cache_bytes();
      (void)hipFuncSetAttribute((const void*)k_p1_count<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsw);
      k_p1_count<false><<<sp.Hc, kCountThreads, ldsw, s>>>(a.keys, a.g, sp, a.counts1,
                                                           a.counts2);
    }
  } else if (a.g.J == 1) {
    k_p1_hist<true><<<sp.G1, kPartThreads, (size_t)sp.nb1 * 4, s>>>(a.keys, a.g, sp, a.counts1);
  } else {  // + the walk cache
    const size_t lds = (size_t)((sp.nb1 + 3) & ~3u) * 4 + walk_cache_bytes();
    (void)hipFuncSetAttribute((const void*)k_p1_hist<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_p1_hist<false><<<sp.G1, kPartThreads, lds, s>>>(a.keys, a.g, sp, a.counts1);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_exclusive(a.counts1, (size_t)sp.nb1 * sp.G1, a.scan_tmp, s)) != hipSuccess) return e;
  using R = typename PRec<PACKED>::T;
  // level 1: threads per workgroup by the bin count
  auto scatter1 = [&](auto nt, auto vt) {
    constexpr int NT = decltype(nt)::value;
    using VT = typename decltype(vt)::type;
    const size_t lds = part_lds_bytes<NT, kPartPer>(sp.nb1, sizeof(R));
    const size_t lds_walk = (lds + 15) / 16 * 16 + walk_cache_bytes();  // batches: + walk cache
    if (a.g.J == 1) {
      (void)hipFuncSetAttribute((const void*)k_p1_scatter<VT, PACKED, NT, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      k_p1_scatter<VT, PACKED, NT, true><<<sp.G1, NT, lds, s>>>(
          a.keys, (const VT*)a.vals, a.g, sp, a.counts1, a.mask_values, a.filter, a.fp_salt,
          fp_late ? 1u : 0u, a.r1);
    } else {
      (void)hipFuncSetAttribute((const void*)k_p1_scatter<VT, PACKED, NT, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_walk);
      k_p1_scatter<VT, PACKED, NT, false><<<sp.G1, NT, lds_walk, s>>>(
          a.keys, (const VT*)a.vals, a.g, sp, a.counts1, a.mask_values, a.filter, a.fp_salt,
          fp_late ? 1u : 0u, a.r1);
    }
  };
  auto scatter1_v = [&](auto nt) {
    switch (a.vbytes) {
      case 1: scatter1(nt, TypeTag<uint8_t>{}); break;
      case 2: scatter1(nt, TypeTag<uint16_t>{}); break;
      default: scatter1(nt, TypeTag<uint32_t>{}); break;
    }
  };
  if (sp.big1)
    scatter1_v(IntTag<kPart1BigThreads>{});
  else
    scatter1_v(IntTag<kPartThreads>{});
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // level 2: records per thread by the sub-bin count
  auto scatter2 = [&](auto per, auto fused, const uint32_t* offs, const uint32_t* offs1) {
    constexpr int PER = decltype(per)::value;
    constexpr bool FU = decltype(fused)::value;
    const size_t lds = part_lds_bytes<kPart2Threads, PER>(sp.S, sizeof(R));
    (void)hipFuncSetAttribute((const void*)k_p2_scatter<PACKED, FU, PER>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_p2_scatter<PACKED, FU, PER><<<sp.U2, kPart2Threads, lds, s>>>(
        a.r1, sp, a.binlo, a.nch, a.cbase, offs, offs1, n, a.r2);
  };
  auto scatter2_p = [&](auto fused, const uint32_t* offs, const uint32_t* offs1) {
    if (sp.big2)
      scatter2(IntTag<kPartPerBig>{}, fused, offs, offs1);
    else
      scatter2(IntTag<kPartPer>{}, fused, offs, offs1);
  };
  if (!sp.H) {
    k_p2_plan<<<1, kPartThreads, 0, s>>>(a.counts1, sp, n, a.binlo, a.nch, a.cbase);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // level 3 with the digits per bucket of the layer (one per chunk or per offset)
  const bool by_offset = digits_per_bucket(a.g) == 64;
  auto level3 = [&](const void* in, const uint32_t* starts) {
    if (by_offset) {
      (void)hipFuncSetAttribute((const void*)k_p3_sort<PACKED, 64>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3_lds_bytes(64));
      k_p3_sort<PACKED, 64><<<sp.nsub, kL3Threads, l3_lds_bytes(64), s>>>(
          in, a.g, sp, starts, a.out_rec, a.bstart, a.fp_salt, fp_late ? a.g.r : 0u, a.clear);
    } else {
      (void)hipFuncSetAttribute((const void*)k_p3_sort<PACKED, 3>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3_lds_bytes(3));
      k_p3_sort<PACKED, 3><<<sp.nsub, kL3Threads, l3_lds_bytes(3), s>>>(
          in, a.g, sp, starts, a.out_rec, a.bstart, a.fp_salt, fp_late ? a.g.r : 0u, a.clear);
    }
    return hipGetLastError();
  };
  if (sp.S == 1)  // the bins are the sub-bins: level 3 reads level 1's output
    return level3(a.r1, a.binlo);
  if (sp.H) {  // positions of the fused counts: prefix over the rows, sub-bin starts
    const uint32_t HB = (sp.Hc + kColBlock - 1) / kColBlock;
    uint32_t* psum = a.counts2 + nds * sp.Hc;
    uint32_t* tot = psum + nds * HB;  // nds + 1: the sub-bin starts
    const dim3 gb((unsigned)((nds + 255) / 256), HB);
    k_col_blocksum<<<gb, 256, 0, s>>>(a.counts2, (uint32_t)nds, sp.Hc, psum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_col_blockbase<<<(unsigned)((nds + 255) / 256), 256, 0, s>>>(psum, (uint32_t)nds, HB, tot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(tot, nds, a.scan_tmp, s)) != hipSuccess) return e;
    k_col_apply<<<gb, 256, 0, s>>>(a.counts2, (uint32_t)nds, sp.Hc, psum, tot, (uint32_t)n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    scatter2_p(BoolTag<true>{}, a.counts2, a.counts1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return level3(a.r2, tot);
  }
  const size_t n2 = (size_t)sp.U2 * sp.S;
  if ((e = hipMemsetAsync(a.counts2, 0, (n2 + 1) * 4, s)) != hipSuccess) return e;
  k_p2_hist<PACKED><<<sp.U2, kPart2Threads, (size_t)sp.S * 4, s>>>(a.r1, sp, a.binlo, a.nch,
                                                                   a.cbase, a.counts2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_exclusive(a.counts2, n2, a.scan_tmp, s)) != hipSuccess) return e;
  scatter2_p(BoolTag<false>{}, a.counts2, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_p2_starts<<<(sp.nsub + 256) / 256, 256, 0, s>>>(sp, n, a.binlo, a.nch, a.cbase, a.counts2,
                                                     a.sstart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return level3(a.r2, a.sstart);
}

// Records are packed when every slot within a level-1 bin fits the low 24
// bits of the meta word and every value fits its top byte - or is left out:
// the fingerprints of a single filter structure wider than 8 bits are
// computed again from the keys at level 3 (one hash per key there against 4
// bytes more per record through both partition levels).
hipError_t sort_layer(const SortArgs& a, hipStream_t s) {
  if (a.g.nkeys == 0) return hipErrorInvalidValue;
  if (a.plan.nsub >= (1u << 24)) return hipErrorInvalidValue;  // level-1 bin arithmetic
  const uint64_t bin_slots = (uint64_t)a.plan.S * kSubSlots;
  if (bin_slots <= (1ull << 24)) {
    if (a.g.r <= 8) return sort_layer_t<true>(a, false, s);
    if (a.filter && a.g.J == 1) return sort_layer_t<true>(a, true, s);
  }
  return sort_layer_t<false>(a, false, s);
}

// ---------------------------------------------------------------------------
// Cut points (Sec. 3 "Selecting Cut Points")
// ---------------------------------------------------------------------------
// One thread per global range rho: rfirst[rho] = its first global bucket,
// rfirst[nranges] = nbuckets. A structure's first range starts at its first
// bucket; the range before every other range ends at a bucket chosen within
// h of the equal split's last bucket b0, h = min(cut_search / 2,
// (floor(B/R) - 2) / 2) (every range keeps two buckets, so each cut is chosen
// on its own). Scores of a candidate last bucket beta, from the bucket
// headers: bumped = its records if any lies past offset 0 (the threshold
// forced on a range's last bucket then bumps all of them, b = w = 64), prev
// = the records of bucket beta-1 past offset 0 (starts in the w-1 slots
// before beta). minbump: fewest bumped; maxprev: most prev; diff: smallest
// bumped - prev; ties to the nearest candidate, then the lower one.
__global__ void k_cuts(LayerGeom g, const uint4* __restrict__ rec,
                       const uint32_t* __restrict__ bstart, uint32_t* __restrict__ rfirst) {
  const uint64_t rho = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rho > g.nranges) return;
  if (rho == g.nranges) {
    rfirst[rho] = (uint32_t)g.nbuckets;
    return;
  }
  const uint32_t j = find_struct(g.range_base, g.J, rho);
  const uint64_t bb = g.bucket_base[j];
  const uint64_t B = g.bucket_base[j + 1] - bb;
  const uint64_t R = g.range_base[j + 1] - g.range_base[j];
  const uint64_t lr = rho - g.range_base[j];
  uint64_t first = bb + lr * B / R;
  const uint64_t L = B / R;
  uint64_t h = g.cut_search / 2;
  const uint64_t hmax = L >= 2 ? (L - 2) / 2 : 0;
  if (h > hmax) h = hmax;
  if (lr > 0 && g.cut_strategy != 0 && g.cut_search >= 2 && h > 0) {
    const uint64_t b0 = first - 1;
    int64_t best = 0;
    uint64_t best_beta = b0, best_dist = 0;
    bool have = false;
    for (uint64_t beta = b0 - h; beta <= b0 + h; ++beta) {
      const uint4 hd = rec[bstart[beta] + beta];
      const uint4 hp = rec[bstart[beta - 1] + beta - 1];
      const int64_t bumped = (hd.y & 63u) ? (int64_t)hd.x : 0;
      const int64_t prev = (int64_t)hp.x - (int64_t)(hp.y >> 8);
      const int64_t score = g.cut_strategy == 1 ? bumped : (g.cut_strategy == 2 ? -prev : bumped - prev);
      const uint64_t dist = beta > b0 ? beta - b0 : b0 - beta;
      if (!have || score < best || (score == best && dist < best_dist)) {
        have = true;
        best = score;
        best_beta = beta;
        best_dist = dist;
      }
    }
    first = best_beta + 1;
  }
  rfirst[rho] = (uint32_t)first;
}

hipError_t choose_cuts(const Rec* rec, const uint32_t* bstart, const LayerGeom& g, uint32_t* rfirst,
                       hipStream_t s) {
  const uint64_t n = g.nranges + 1;
  k_cuts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, reinterpret_cast<const uint4*>(rec), bstart,
                                                     rfirst);
  return hipGetLastError();
}

// Records the state of the first wave that stops with an internal error.
__device__ inline void solve_diag(uint64_t* d, uint32_t code, uint64_t rho, uint32_t js,
                                  uint32_t hq, uint32_t count, uint32_t q, uint32_t nq,
                                  uint32_t cand, bool unused0, uint32_t kept, uint32_t thr,
                                  uint32_t kf, uint32_t unused1, uint32_t unused2, uint64_t fb) {
  if (!d || atomicCAS((unsigned long long*)d, 0ull, 1ull) != 0ull) return;
  d[1] = code;
  d[2] = rho;
  d[3] = js;
  d[4] = hq;
  d[5] = count;
  d[6] = q;
  d[7] = nq;
  d[8] = cand;
  d[9] = unused0;
  d[10] = kept;
  d[11] = thr;
  d[12] = kf;
  d[13] = unused1;
  d[14] = unused2;
  d[15] = fb;
}

// ---------------------------------------------------------------------------
// Solve: one wave per range, the lanes insert a bucket's records together
// ---------------------------------------------------------------------------
// The range's rows live in a window of 128 slots in LDS shared by the wave:
// bucket q's slots [64q, 64q+126] sit at window slots [0, 126], and after
// the bucket its first 64 slots are published and the upper half moves
// down (it is bucket q+1's first half). A pass inserts a set of records of
// the current bucket: lanes take records from the staged bucket, and every
// lane repeats one elimination step against the ring - XOR with the row at
// its leading slot and shift - until its row reduces to zero or reaches an
// empty slot, which it claims with an LDS compare-and-swap. Claims serialize,
// so a pass equals sequential insertion in claim order; the pivot set and the
// solution with free slots 0 do not depend on that order (they are
// invariants of the row space), nor does the consistency of the inserted set.
//
// Per bucket, the first pass inserts every record that is not forced out.
// If it meets an inconsistency (a row reducing to 0 with a nonzero value),
// its rows are removed and the shorter chunk prefixes are tried, largest
// first; the first consistent prefix is kept and the failing chunk sets the
// bucket's threshold - the outcome of inserting the chunks one after the
// other in decreasing offset order (Sec. 2, 2-bit thresholds), since a
// prefix of a consistent set is consistent.
// Lane groups: LANES lanes insert one range, so a wave holds 64 / LANES
// ranges, each with its own ring and stage in LDS. A bucket takes as long as
// its longest elimination chain while its ~66 keys need far fewer lane-steps
// than 64 lanes offer, so with 32 lanes per range two ranges share the lanes
// one range would leave idle.
//
// The staged bucket: header + records, a staged record holding its
// coefficient row instead of its key: {row low, row high, value,
// offset|rank}; records past the stage are read from the item stream.
template <int LANES>
struct Stage {
  static constexpr uint32_t items = LANES == 64 ? 128 : 96;
  static constexpr uint32_t per_lane = items / LANES;
};

// The ring of one range: rows in an array of 8-byte slots and values in an
// array of 4-byte slots, addressed by the row's byte offset (the value's is
// half of it). Lanes read random slots, so the narrow value array spreads
// their value reads over twice as many LDS banks as an 8-byte stride would
// (measured: 16-byte {row, value} slots and 8-byte value slots both had
// more bank conflicts). An empty slot has row 0 and value 0; a row has bit 0
// set.
template <int LANES>
struct WaveRing {
  uint64_t c[kRing];
  uint32_t v[kRing + 64];  // + one spare word per lane (claims that lose write there)
  uint4 stage[Stage<LANES>::items];
  uint32_t bs[LANES];      // bucket starts of a window of LANES buckets
};
// row and value of the slot at byte offset off = 8 * slot
template <class Ring>
__device__ inline void ring_read_b(const Ring& R, uint32_t off, uint64_t& row, uint32_t& val) {
  row = *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(R.c) + off);
  val = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(R.v) + (off >> 1));
}
// claims the empty slot at byte offset off for row c and value v; false if
// another lane took it first
template <class Ring>
__device__ inline bool ring_claim(Ring& R, uint32_t off, uint64_t c, uint32_t v) {
  const uint64_t old = atomicCAS(
      reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(R.c) + off), 0ull,
      (unsigned long long)c);
  const bool won = old == 0;
  // the value goes to the slot if the row did, else to this lane's spare word
  // (a select instead of a branch inside the claim)
  const uint32_t voff = won ? (off >> 1) : (uint32_t)((kRing + (threadIdx.x & 63u)) * 4u);
  *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(R.v) + voff) = v;
  return won;
}
template <class Ring>
__device__ inline void ring_read(const Ring& R, uint32_t i, uint64_t& row, uint32_t& val) {
  row = R.c[i];
  val = R.v[i];
}
template <class Ring>
__device__ inline void ring_clear(Ring& R, uint32_t p) {
  R.c[p] = 0;
  R.v[p] = 0;
}

__device__ inline uint64_t slot_row(const uint4& s) {
  return (uint64_t)s.x | ((uint64_t)s.y << 32);
}

// a record of the item stream as staged: its key replaced by its row
__device__ inline uint4 staged(const uint4& r, const LayerGeom& g) {
  const uint64_t c = row_of((uint64_t)r.x | ((uint64_t)r.y << 32), g);
  return make_uint4((uint32_t)c, (uint32_t)(c >> 32), r.z, r.w);
}

// This lane's group: ballots, "any" and ranks restricted to the group's
// lanes. Within one wave, LDS operations complete in order, so a fence that
// waits for them orders the group's LDS traffic (no barrier is needed, and
// none is used inside code where the groups diverge).
template <int LANES>
struct Grp {
  uint32_t id;    // group within the wave
  uint32_t lane;  // lane within the group
  __device__ Grp() : id(LANES == 64 ? 0u : threadIdx.x / LANES), lane(threadIdx.x % LANES) {}
  __device__ uint64_t ballot(bool p) const {
    const uint64_t m = __builtin_amdgcn_ballot_w64(p);
    if constexpr (LANES == 64)
      return m;
    else
      return (m >> (id * LANES)) & ((1ull << LANES) - 1);
  }
  __device__ bool any(bool p) const { return ballot(p) != 0; }
  // set bits of a group mask below this lane
  __device__ uint32_t rank(uint64_t m) const {
    if constexpr (LANES == 64)
      return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    else
      return (uint32_t)__popcll(m & ((1ull << lane) - 1));
  }
  __device__ void sync() const {
    if constexpr (LANES == 64) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
  }
};

#ifndef BURR_SOLVE_K
#define BURR_SOLVE_K 4
#endif
constexpr int kSolveK = BURR_SOLVE_K;  // elimination steps per loop trip

// Optional counters (-DBURR_SOLVE_STATS): elimination steps, and loop trips,
// passes and active lanes per trip in the three words after the step count.
#ifdef BURR_SOLVE_STATS
struct SolveStats {
  uint64_t trips = 0, passes = 0, lanes = 0;
};
#define BURR_STAT(x) x
#else
struct SolveStats {};
#define BURR_STAT(x)
#endif

// Inserts records [r0, r1) of the staged bucket q. Returns 0 if the set was
// consistent, 1 if an inconsistency was met (its rows are removed again), 2
// on an internal error, or 3 (FAST only) if the pass has to be run exactly.
// Each loop trip: lanes without a row take the next records, every lane
// makes kSolveK XOR-and-shift steps against the ring, then the lanes at an
// empty slot claim it. The steps need no per-lane masking: at an empty slot
// (row 0, value 0) a step leaves the lane's row, value and position
// unchanged (its row keeps bit 0, so the shift is 0), and the state of lanes
// that finished is not used again.
// A lane's position is kept as the byte offset of its slot within the
// window (8 (i - 64 q) for slot i), which addresses the slot's row and
// value; a step advances it with one shift-add (with a wrapping ring it also
// took a mask, one more instruction on every step's dependent chain). A row
// ending in the window's upper half has crossed into bucket q+1: when q is
// the range's last bucket and there is no spill buffer (last_half set),
// claiming it would be an error.
// With 64 lanes per range, r0, r1 and next are wave-uniform (scalar), so the
// record hand-out costs no vector instructions once the records are taken.
//
// FAST: a step finds the shift from the row's low word alone. Rows are hash
// words with bit 0 set, so after an XOR with an occupied slot's row the low
// word is nonzero unless the row reduced to zero (redundant or inconsistent)
// or, with probability 2^-31, its lowest set bit is in the high word. If an
// active lane met a zero low word in a trip, the pass stops before that
// trip's claims, is undone and returns 3, and the caller runs it again
// exactly (not FAST), which gives the outcome of sequential insertion in
// every case. Without such an event, lanes only leave the active state by
// claiming, so the steps track nothing else. FAST passes are not used with
// last_half (they do not check claims against the range end).
template <int LANES, bool FAST>
__device__ inline uint32_t wave_pass(WaveRing<LANES>& R, const Grp<LANES>& G,
                                     const SolveArgs& a, const uint4* rec4, uint32_t hq,
                                     uint32_t q, uint32_t r0, uint32_t r1, bool last_half,
                                     uint64_t& steps, SolveStats& st) {
  (void)st;
  (void)steps;
  BURR_STAT(++st.passes; uint64_t pass_steps = 0;)
  // occupied slots before the pass: an undo clears the slots claimed since
  uint64_t before[kRing / 64];
#pragma unroll
  for (uint32_t h = 0; h < kRing / 64; ++h) {
    uint64_t m = 0;
#pragma unroll
    for (uint32_t k = 0; k < 64 / LANES; ++k)
      m |= G.ballot(R.c[h * 64 + k * LANES + G.lane] != 0) << (k * LANES);
    before[h] = m;
  }
  // Bucket q's first slot is the ring's first (after each bucket the ring's
  // upper half moves down), so a kept row's slot is at most 126 and a step
  // needs no wrap-around. Lanes whose state is no longer used (finished, or
  // a FAST pass about to stop) may walk past the ring: they only read, and
  // LDS reads past the workgroup's allocation return 0.
  constexpr uint32_t kHalf = 64u * 8u;  // byte size of a ring half (rows)
  bool active = false, conflict = false, err = false, hung = false, special = false;
  uint64_t c = 0;
  uint32_t v = 0, ib = 0;  // ib: byte offset of the lane's slot
  uint32_t next = r0;
  uint32_t guard = (r1 - r0) * 256u + 1024u;  // a lane advances or stops every other step
  while (true) {
    if (next < r1) {
      // lanes without a row take the next records
      const uint64_t freem = G.ballot(!active);
      const uint32_t rank = G.rank(freem);
      if (!active && rank < r1 - next) {
        const uint32_t t = next + rank;
        constexpr uint32_t last = Stage<LANES>::items - 1;
        uint4 r = R.stage[t < last ? t + 1 : last];
        c = slot_row(r);
        if (t >= last) {  // bucket larger than the stage (rare; a load that cannot merge with the LDS read)
          typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
          const u32x4 g4 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rec4 + hq + 1 + t));
          r = make_uint4(g4.x, g4.y, g4.z, g4.w);
          c = row_of((uint64_t)r.x | ((uint64_t)r.y << 32), a.g);
        }
        v = r.z;
        ib = (r.w & 63u) << 3;
        active = true;
      }
      const uint32_t nfree = (uint32_t)__popcll(freem);
      next = (r1 - next < nfree) ? r1 : next + nfree;
      if constexpr (LANES == 64) next = __builtin_amdgcn_readfirstlane(next);  // uniform
      // a record was taken, or every lane already had one: some lane is active
    } else if (!G.any(active)) {
      break;
    }
    BURR_STAT(++st.trips; st.lanes += __popcll(G.ballot(active));)
    if (guard-- == 0) {
      hung = true;
      break;
    }
    uint64_t row = 0;
    uint32_t off = ib;
    bool low_ok = true;  // FAST: every step's low word was nonzero
#pragma unroll
    for (int u = 0; u < kSolveK; ++u) {
      off = ib;
      uint32_t rv;
      ring_read_b(R, off, row, rv);
      const uint64_t cx = c ^ row;
      const uint32_t vx = v ^ rv;
      BURR_STAT(pass_steps += (active && row != 0) ? 1u : 0u;)
      uint32_t j;
      if constexpr (FAST) {
        const uint32_t lo = (uint32_t)cx;
        low_ok = low_ok && lo != 0;
        // lowest set bit of the low word (all ones for 0: the pass stops)
        asm("v_ffbl_b32 %0, %1" : "=v"(j) : "v"(lo));
      } else {
        const bool nz = cx != 0;  // else reduced to 0 = vx: redundant or inconsistent
        conflict = conflict || (active && !nz && vx != 0);
        active = active && nz;
        j = (uint32_t)__builtin_ctzg(cx, 64);
      }
      c = cx >> (j & 63u);
      v = vx;
      ib += j << 3;
      // opaque to the compiler, which would otherwise sum the steps' shifts
      // first and add them to the start (two dependent adds per step)
      asm("" : "+v"(ib));
    }
    // the last step read an empty slot: the lane stayed on it (at byte offset off)
    const bool at_empty = active && row == 0;
    if constexpr (FAST) {
      if (G.any(active && !low_ok)) {
        special = true;
        break;
      }
    }
    if (at_empty) {
      if (!FAST && last_half && off >= kHalf) {
        active = false;  // unreachable: a kept row crossing the range end
        err = true;
      } else {
        if (ring_claim(R, off, c, v)) active = false;
        // otherwise another lane took the slot: step against its row next time
      }
    }
    if constexpr (!FAST) {
      if (G.any(conflict || err)) break;
    }
  }
  G.sync();
  uint32_t result;
  if constexpr (FAST)
    result = hung ? 2u : (special ? 3u : 0u);
  else
    result = (hung || G.any(err)) ? 2u : (G.any(conflict) ? 1u : 0u);
  BURR_STAT(if (result != 3) steps += pass_steps;)  // a stopped FAST pass is run again
  if (result != 0) {
#pragma unroll
    for (uint32_t k = 0; k < kRing / LANES; ++k) {
      const uint32_t t = k * LANES + G.lane;
      if (R.c[t] != 0 && !((before[t >> 6] >> (t & 63)) & 1ull)) ring_clear(R, t);
    }
  }
  G.sync();
  return result;
}

// Publishes a released ring half: its 64 rows, values and occupancy word go
// to the layer's row arrays (or, past the range end, to the segment's spill
// buffer) as one coalesced block, and clears it.
template <int LANES>
__device__ inline void release_half(WaveRing<LANES>& R, const Grp<LANES>& G, uint32_t hb,
                                    uint64_t* rowsC, uint32_t* rowsV, uint64_t* occw) {
  uint64_t word = 0;
#pragma unroll
  for (uint32_t k = 0; k < 64 / LANES; ++k) {
    const uint32_t t = k * LANES + G.lane;
    uint64_t row;
    uint32_t val;
    ring_read(R, hb + t, row, val);
    word |= G.ballot(row != 0) << (k * LANES);
    rowsC[t] = row;
    rowsV[t] = val;
  }
  if (G.lane == 0) *occw = word;
}

// Moves the ring's upper half to its lower half (after the lower half was
// published) and clears the upper half. Within one wave LDS operations
// complete in order, so the moves read the upper half before it is cleared
// and write the lower half after release_half read it.
template <int LANES>
__device__ inline void shift_down(WaveRing<LANES>& R, const Grp<LANES>& G) {
#pragma unroll
  for (uint32_t k = 0; k < 64 / LANES; ++k) {
    const uint32_t t = k * LANES + G.lane;
    uint64_t row;
    uint32_t val;
    ring_read(R, 64 + t, row, val);
    R.c[t] = row;
    R.v[t] = val;
    ring_clear(R, 64 + t);
  }
}

// 8 waves per SIMD: the kernel then fits 64 VGPRs (no spills), and the
// ring, stage and bucket starts of 32 waves (4 KB each) fit a CU's LDS. ONE_PLUS: the
// instantiation for 1+-bit thresholds of BuRR layers (the 2-bit one carries
// no code of the threshold bisection).
template <int LANES, bool ONE_PLUS>
__global__ __launch_bounds__(64, 8) void k_solve_wave(SolveArgs a) {
  constexpr uint32_t NG = 64 / LANES;
  constexpr uint32_t SP = Stage<LANES>::per_lane;
  __shared__ WaveRing<LANES> RR[NG];
  const Grp<LANES> G;
  WaveRing<LANES>& R = RR[G.id];
  const LayerGeom g = a.g;
  const uint64_t rho = (uint64_t)blockIdx.x * NG + G.id;
  // this group's range: buckets [fb, fb + nq) of structure js (none past the
  // last range); the structure's last range bumps nothing for its end
  uint32_t js = 0, nq = 0;
  uint64_t fb = 0;
  bool last_range = true;
  if (rho < g.nranges) {
    js = find_struct(g.range_base, g.J, rho);
    uint64_t f0, f1;
    range_buckets(g, js, rho, f0, f1);
    fb = f0;
    nq = (uint32_t)(f1 - f0);
    last_range = rho + 1 == g.range_base[js + 1];
  }
  const uint32_t last_item = a.nrec - 1;
  const uint4* rec4 = reinterpret_cast<const uint4*>(a.rec);
#pragma unroll
  for (uint32_t k = 0; k < kRing / LANES; ++k) ring_clear(R, k * LANES + G.lane);
  uint64_t steps = 0;
  SolveStats sst;
  bool failed = false;
  // Item index of bucket q's header, from the starts of a window of LANES
  // buckets that the group keeps in LDS (loaded once per window), so that a
  // bucket's items are loaded without first waiting for its start.
  auto load_window = [&](uint32_t w) {
    const uint64_t b = fb + w + G.lane;
    R.bs[G.lane] = a.bstart[b < g.nbuckets ? b : g.nbuckets];
  };
  auto item_of = [&](uint32_t q) -> uint32_t {
    uint32_t st = R.bs[q % LANES];
    if constexpr (LANES == 64) st = __builtin_amdgcn_readfirstlane(st);
    return st + (uint32_t)(fb + q);
  };
  // A bucket's items are staged through registers: loaded (unconditionally:
  // past the range, the next buckets' items, not used) before the previous
  // bucket is inserted and written to the stage after it. The loads are
  // then not waited for before that insertion; a conditional load, or
  // registers that carry a value from one loop trip into the next, make the
  // compiler copy the loaded values, and wait for them, right away.
  uint4 nx[SP];
  auto load_items = [&](uint32_t h) {
#pragma unroll
    for (uint32_t k = 0; k < SP; ++k) {
      const uint32_t t = h + k * LANES + G.lane;
      nx[k] = rec4[t < last_item ? t : last_item];
    }
  };
  auto stage_items = [&]() {
#pragma unroll
    for (uint32_t k = 0; k < SP; ++k)  // entry 0 is the bucket header
      R.stage[k * LANES + G.lane] = (k == 0 && G.lane == 0) ? nx[0] : staged(nx[k], g);
  };
  if (nq) {
    load_window(0);
    G.sync();
    load_items(item_of(0));
    stage_items();
  }
  for (uint32_t q = 0; q < nq && !failed; ++q) {
    const uint64_t beta = fb + q;
    const uint32_t hq = item_of(q);
    if ((q + 1) % LANES == 0) {
      G.sync();  // every lane has read its start of this window
      load_window(q + 1);
    }
    G.sync();
    load_items(item_of(q + 1));  // while bucket q is inserted
    uint4 hd = R.stage[0];
    if constexpr (LANES == 64) {  // the same for every lane: keep it scalar
      hd.x = __builtin_amdgcn_readfirstlane(hd.x);
      hd.y = __builtin_amdgcn_readfirstlane(hd.y);
      hd.z = __builtin_amdgcn_readfirstlane(hd.z);
      hd.w = __builtin_amdgcn_readfirstlane(hd.w);
    }
    const uint32_t count = hd.x, maxo = hd.y & 63u;
    // the last bucket of a range that is not its structure's last: every key
    // past the bucket's first slot would cross the range end (b = w = 64), so
    // the threshold is forced above the largest offset (Sec. 3 "Bumping"):
    // the smallest 2-bit value above it, or with 1+-bit thresholds the
    // offset + 1 (kf: 2-bit code index, or 1+-bit threshold value)
    const bool at_end = !g.plain && !last_range && q + 1 == nq && maxo > 0;
    const uint32_t kf = !at_end ? 0u
                      : ONE_PLUS ? maxo + 1u
                      : (maxo >= g.t_hi ? 3u : (maxo >= g.t_lo ? 2u : 1u));
    const uint32_t e1 = hd.z, e2 = hd.z + hd.w;  // ends of ranks 0 and 1
    // claims past the range end: only from its last bucket, without a spill buffer
    const bool last_half = q + 1 == nq && !a.spillC;
    // records [r0, r1) of the bucket on top of the ring: fast pass, exact
    // pass if it stopped (exact only in a range's last bucket without a
    // spill buffer)
    auto pass = [&](uint32_t r0, uint32_t r1) {
      const uint32_t res =
          last_half ? 3u : wave_pass<LANES, true>(R, G, a, rec4, hq, q, r0, r1, false, steps, sst);
      return res == 3 ? wave_pass<LANES, false>(R, G, a, rec4, hq, q, r0, r1, last_half, steps, sst)
                      : res;
    };
    constexpr bool one_plus = ONE_PLUS;
    // 1+-bit: kf > 0 lies above every offset, so then nothing is a candidate
    const uint32_t keep_ranks = g.plain ? 3u : 3u - kf;
    const uint32_t cand = one_plus ? (kf == 0 ? count : 0u)
                        : keep_ranks == 3 ? count : (keep_ranks == 2 ? e2 : (keep_ranks == 1 ? e1 : 0u));
    uint32_t kept = cand, code = kf;
    if constexpr (ONE_PLUS) {
     if (cand > 0) {
      // records ordered by offset, highest first: the records with offset
      // >= theta are a prefix of the bucket; its length from ballots over
      // the staged offsets (records past the stage from the item stream)
      auto prefix_len = [&](uint32_t theta) {
        constexpr uint32_t last = Stage<LANES>::items - 1;
        const uint32_t ns = count < last ? count : last;  // staged records
        uint32_t c = 0;
        for (uint32_t t0 = 0; t0 < ns; t0 += LANES) {
          const uint32_t t = t0 + G.lane;
          const uint32_t o = t < ns ? R.stage[t + 1].w & 63u : 0u;
          c += (uint32_t)__popcll(G.ballot(t < ns && o >= theta));
        }
        // records past the stage (a bucket of more than `last` records,
        // rare) in a loop of their own: a global load beside the stage
        // reads would make them wait for every memory operation in flight
        for (uint32_t t0 = last; t0 < count; t0 += LANES) {
          const uint32_t t = t0 + G.lane;
          const uint32_t o = t < count ? rec4[hq + 1 + (t < count ? t : last)].w & 63u : 0u;
          c += (uint32_t)__popcll(G.ballot(t < count && o >= theta));
        }
        return c;
      };
      uint32_t res = pass(0, cand);
      if (res == 1) {
        // the smallest threshold whose kept set is consistent, by bisection
        // over offsets: the ring keeps the rows of the largest prefix known
        // to be consistent (threshold `good`), a trial inserts the next
        // records on top of it and is undone if it fails (a prefix of a
        // consistent set is consistent, so the outcome equals inserting the
        // keys one by one in decreasing offset order)
        uint32_t good = 64, n_good = 0, bad = kf, n_bad = cand;
        res = 0;
        while (good - bad > 1 && res != 2) {
          const uint32_t mid = (good + bad) >> 1;
          const uint32_t n_mid = prefix_len(mid);
          if (n_mid == n_good) {
            good = mid;
          } else if (n_mid == n_bad) {
            bad = mid;
          } else {
            res = pass(n_good, n_mid);
            if (res == 0) {
              good = mid;
              n_good = n_mid;
            } else if (res == 1) {
              bad = mid;
              n_bad = n_mid;
              res = 0;
            }
          }
        }
        kept = n_good;
        code = good;
      }
      if (res == 2) {
        if (G.lane == 0) {
          a.fail[js] = 2u;
          solve_diag(a.diag, 2, rho, js, hq, count, q, nq, cand, 0, kept, code, kf, 0, 0, fb);
        }
        failed = true;
      }
     }
    } else if (cand > 0) {
      uint32_t res = pass(0, cand);
      if (res == 1 && g.plain) {
        if (G.lane == 0) a.fail[js] = 1u;
        failed = true;
      } else if (res == 1) {
        kept = 0;
        code = 3;
        uint32_t failed_size = cand;  // smallest prefix known to be inconsistent
        for (uint32_t rr = keep_ranks - 1; rr >= 1 && res != 2; --rr) {
          const uint32_t e = rr == 2 ? e2 : e1;
          if (e == failed_size) continue;  // the same set again
          res = e ? pass(0, e) : 0u;
          if (res == 0) {
            kept = e;
            code = 3 - rr;
            break;
          }
          failed_size = e;
        }
      }
      if (res == 2) {
        if (G.lane == 0) {
          a.fail[js] = 2u;
          solve_diag(a.diag, 2, rho, js, hq, count, q, nq, cand, 0, kept, code, kf, 0, 0, fb);
        }
        failed = true;
      }
    }
    G.sync();
    // bucket q+1's items to the stage first: their loads are the oldest
    // memory operations in flight, so waiting for them does not wait for
    // the stores below. Unconditionally (after the last bucket the stage is
    // not read again): with a path on which the loads stay unused, the
    // compiler waits for all memory operations, stores included, before it
    // reuses their registers.
    stage_items();
    if (!g.plain && G.lane == 0) {
      a.code8[beta] = (uint8_t)code;
      a.bump[beta] = count - kept;
    }
    if (q + 1 < nq && !failed) {
      // bucket q's first 64 slots, which no later bucket changes: publish
      // their rows; bucket q+1 starts at the ring's base
      release_half(R, G, 0, a.rowsC + beta * 64, a.rowsV + beta * 64, a.occ + beta);
      shift_down(R, G);
    }
  }
  if (nq && !failed) {
    const uint64_t beta = fb + nq - 1;
    release_half(R, G, 0, a.rowsC + beta * 64, a.rowsV + beta * 64, a.occ + beta);
    if (a.spill_occ) {  // rows past the segment end (final layer)
      release_half(R, G, 64, a.spillC + rho * 64, a.spillV + rho * 64, a.spill_occ + rho);
    }
  }
  if (a.steps) {
    for (int d = 32; d >= 1; d >>= 1) steps += __shfl_xor(steps, d, 64);
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)a.steps, (unsigned long long)steps);
#ifdef BURR_SOLVE_STATS
    uint64_t t3[3] = {sst.trips, sst.passes, sst.lanes};
    for (int k = 0; k < 3; ++k) {
      uint64_t x = G.lane == 0 ? t3[k] : 0;  // one count per group
      for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
      if (threadIdx.x == 0) atomicAdd((unsigned long long*)a.steps + 1 + k, (unsigned long long)x);
    }
#endif
  }
}

// Lanes per range. 64: one range per wave (default). 32 (-DBURR_SOLVE_LANES=32):
// two ranges per wave; same results, measured slower at 100M keys (3.30
// against 2.60 ms: the per-group control moves from scalar to vector
// registers and occupancy drops from 8 to 5 waves per SIMD) and on small
// layers.
#ifndef BURR_SOLVE_LANES
#define BURR_SOLVE_LANES 64
#endif

hipError_t solve_layer(const SolveArgs& a, hipStream_t s) {
  if (a.g.nranges == 0) return hipSuccess;
  constexpr int NG = 64 / BURR_SOLVE_LANES;
  const unsigned grid = (unsigned)((a.g.nranges + NG - 1) / NG);
  if (a.g.thr_mode == 1 && !a.g.plain)
    k_solve_wave<BURR_SOLVE_LANES, true><<<grid, 64, 0, s>>>(a);
  else
    k_solve_wave<BURR_SOLVE_LANES, false><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Back-substitution: a group of RG lanes per range, one lane per value column
// ---------------------------------------------------------------------------
// From the range end down, per 64-slot block: the group loads the block's
// rows and values into LDS (the next block's loads are in flight meanwhile),
// then every lane runs the block's 64 slots for its column:
// Z[i] = V[i] xor parity(C[i] >> 1 AND the next 63 values), kept as a 64-bit
// window per column. Free slots are 0 without a test: every released block
// holds row 0 and value 0 in its free slots (the ring's empty slots are
// zero, and merges write occupied slots only), which gives Z = 0 there. After
// a block's 64 slots the window holds exactly the block's values.
template <int RG>
__global__ __launch_bounds__(64) void k_backsub(const uint64_t* __restrict__ rowsC,
                                                const uint32_t* __restrict__ rowsV, LayerGeom g,
                                                uint64_t* __restrict__ W,
                                                const uint32_t* __restrict__ bnd) {
  constexpr int NG = 64 / RG;   // ranges per wave
  constexpr int PER = 64 / RG;  // slots each lane loads per block
  // one padding slot per range: the groups read slot tt of their own block
  // at the same time, which would otherwise fall into one LDS bank
  __shared__ uint64_t sc[2][NG][65];  // rows shifted right by 1 (bit 0 is the pivot)
  __shared__ uint32_t sv[2][NG][65];
  const uint32_t lane = threadIdx.x, grp = lane / RG, col = lane % RG;
  // a wave takes NG ranges at a time, the grid's waves in turn (the grid may
  // be narrower than the ranges: a back-substitution beside other layers'
  // work is given a bounded share of the device)
  for (uint64_t rho0 = (uint64_t)blockIdx.x * NG; rho0 < g.nranges; rho0 += (uint64_t)gridDim.x * NG) {
  const uint64_t rho = rho0 + grp;
  const bool valid = rho < g.nranges;
  uint32_t r = 0;
  uint64_t fb = 0, lb = 0, wb = 0, bb = 0;
  if (valid) {
    const uint32_t j = find_struct(g.range_base, g.J, rho);
    bb = g.bucket_base[j];
    range_buckets(g, j, rho, fb, lb);
    r = g.rbits[j];
    wb = g.word_base[j];  // block k of the structure at wb + (k - bb) * r
  }
  const uint32_t nblk = (uint32_t)(lb - fb);
  uint32_t maxblk = nblk;
  for (int d = 32; d >= 1; d >>= 1) maxblk = max(maxblk, (uint32_t)__shfl_xor((int)maxblk, d, 64));
  uint64_t win = 0;  // bit t = value of this column at slot i+1+t
  if (bnd && valid) {
    // the 63 slots after the range hold known values (final-layer segments)
    for (uint32_t t = 0; t < 63; ++t) win |= (uint64_t)((bnd[rho * 64 + t] >> col) & 1u) << t;
  }
  uint64_t pc[PER];
  uint32_t pv[PER];
#define BURR_BS_LOAD(t)                                                  \
  if ((t) < nblk) {                                                      \
    const uint64_t base = (lb - 1 - (t)) * 64;                           \
    _Pragma("unroll") for (int e = 0; e < PER; ++e) {                    \
      pc[e] = rowsC[base + col + e * RG];                                \
      pv[e] = rowsV[base + col + e * RG];                                \
    }                                                                    \
  }
  BURR_BS_LOAD(0u)
  for (uint32_t t = 0; t < maxblk; ++t) {
    const uint32_t buf = t & 1u;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      sc[buf][grp][col + e * RG] = pc[e] >> 1;
      sv[buf][grp][col + e * RG] = pv[e];
    }
    __syncthreads();
    BURR_BS_LOAD(t + 1)
    if (t < nblk) {
#pragma unroll 8
      for (int tt = 63; tt >= 0; --tt) {
        const uint64_t C = sc[buf][grp][tt];
        const uint32_t V = sv[buf][grp][tt];
        // parity of C AND win plus this column's value bit: the two words'
        // ANDs folded by XOR, counted on top of V >> col, then bit 0
        const uint32_t x = ((uint32_t)C & (uint32_t)win) ^ ((uint32_t)(C >> 32) & (uint32_t)(win >> 32));
        const uint32_t z = ((uint32_t)__popc(x) + (V >> col)) & 1u;
        win = (win << 1) | z;
      }
      const uint64_t k = lb - 1 - t;
      if (col < r) W[wb + (k - bb) * r + col] = win;
    }
  }
  __syncthreads();  // the next ranges reuse the LDS blocks
  }
#undef BURR_BS_LOAD
}

hipError_t back_substitute(const uint64_t* rowsC, const uint32_t* rowsV, const LayerGeom& g,
                           uint64_t* W, hipStream_t s, const uint32_t* bnd, uint32_t max_waves) {
  if (g.nranges == 0) return hipSuccess;
  auto grid = [&](uint64_t per_wave) {  // at least a quarter of the full grid
    const uint64_t w = (g.nranges + per_wave - 1) / per_wave;
    const uint64_t cap = max_waves > w / 4 ? max_waves : w / 4;
    return (unsigned)(max_waves && w > cap ? cap : w);
  };
  if (g.r <= 8)
    k_backsub<8><<<grid(8), 64, 0, s>>>(rowsC, rowsV, g, W, bnd);
  else if (g.r <= 16)
    k_backsub<16><<<grid(4), 64, 0, s>>>(rowsC, rowsV, g, W, bnd);
  else
    k_backsub<32><<<grid(2), 64, 0, s>>>(rowsC, rowsV, g, W, bnd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final plain layer across segments
// ---------------------------------------------------------------------------
// The final layer cannot bump, so its segments are not independent: a row may
// end past its segment's end. After the per-segment solve those rows wait in
// the segment's spill buffer. Merging inserts a left group's spill rows into
// the right group (the usual elimination, starting at the right group's first
// slots), so after log2(segments) levels the whole layer is one echelon
// system - the same row space, hence the same solution with free slots 0.

// slots [start, end) of global segment p (a "range" of the final layer)
struct SegBounds {
  uint32_t j;       // structure
  uint64_t first;   // first global segment of the structure
  uint64_t count;   // segments of the structure
  uint64_t start, end;
};
__device__ inline SegBounds seg_bounds(uint64_t p, const LayerGeom& g) {
  SegBounds sb;
  sb.j = find_struct(g.range_base, g.J, p);
  const uint64_t B = g.bucket_base[sb.j + 1] - g.bucket_base[sb.j];
  sb.first = g.range_base[sb.j];
  sb.count = g.range_base[sb.j + 1] - sb.first;
  const uint64_t lp = p - sb.first;
  sb.start = 64 * (g.bucket_base[sb.j] + lp * B / sb.count);
  sb.end = 64 * (g.bucket_base[sb.j] + (lp + 1) * B / sb.count);
  return sb;
}

constexpr uint32_t kMergeWin = 1024;  // slots of the right group staged in LDS

// One workgroup per segment p; it merges at level G when p starts a left
// group of G segments inside its structure and a right group follows. The
// left group's spill rows (at most 63) are inserted into the right group in
// parallel, one lane per row, with the same step-and-claim scheme as the
// insertion kernel over an LDS window of the right group (empty slots hold
// 0). Rows whose walk leaves the window are finished one by one in global
// memory afterwards.
__global__ __launch_bounds__(64) void k_merge(FinalArgs a, uint32_t G) {
  // + 64 zero slots after the window: a walk that leaves the window stops at
  // the first of them (a row keeps bit 0, so a step at an empty slot does
  // not move), and the steps need no clamp
  __shared__ uint64_t wc[kMergeWin + 64];
  __shared__ uint32_t wv[kMergeWin + 64];
  __shared__ uint64_t oc_[64];
  __shared__ uint32_t ov_[64], oi_[64];
  const LayerGeom g = a.g;
  const uint64_t p = blockIdx.x;
  const SegBounds sp = seg_bounds(p, g);
  const uint64_t lp = p - sp.first;
  if (lp % (2ull * G) != 0 || lp + G >= sp.count) return;
  // a structure whose segment solve already failed keeps no valid rows in
  // its unfinished buckets: nothing to merge
  if (a.fail[sp.j]) return;
  const uint64_t R0 = p + G;
  const uint64_t lastL = R0 - 1;
  const uint64_t lastR = (lp + 2ull * G < sp.count ? p + 2ull * G : sp.first + sp.count) - 1;
  const uint64_t start = seg_bounds(R0, g).start;
  const uint64_t endR = seg_bounds(lastR, g).end;  // slot after the right group
  // window: slots [start, start + win); slots >= endR are the right group's
  // spill zone, which the window holds either completely or not at all
  // (start, endR and the window are multiples of 64)
  const uint64_t span = endR + 64 - start;
  const uint64_t body = endR - start;
  const uint32_t win = (uint32_t)(span <= kMergeWin ? span : (body < kMergeWin ? body : kMergeWin));
  const uint32_t lane = threadIdx.x;
  // every load of the window is issued before the first LDS store (win >= 64;
  // blocks past the window repeat its last block and are not stored)
  constexpr uint32_t kWinBlocks = kMergeWin / 64;
  const uint32_t nblk = win / 64;
  uint64_t lrow[kWinBlocks], locc[kWinBlocks];
  uint32_t lval[kWinBlocks], lsh[kWinBlocks];
#pragma unroll
  for (uint32_t blk = 0; blk < kWinBlocks; ++blk) {
    const uint64_t slot = start + 64ull * (blk < nblk ? blk : nblk - 1) + lane;
    if (slot < endR) {  // uniform per block: endR is a multiple of 64
      locc[blk] = a.occ[slot / 64];
      lsh[blk] = (uint32_t)(slot % 64);
      lrow[blk] = a.rowsC[slot];
      lval[blk] = a.rowsV[slot];
    } else {
      locc[blk] = a.spill_occ[lastR];
      lsh[blk] = (uint32_t)(slot - endR);
      lrow[blk] = a.spillC[lastR * 64 + (slot - endR)];
      lval[blk] = a.spillV[lastR * 64 + (slot - endR)];
    }
  }
#pragma unroll
  for (uint32_t blk = 0; blk < kWinBlocks; ++blk)
    if (blk < nblk) {
      const bool occd = (locc[blk] >> lsh[blk]) & 1ull;
      wc[64 * blk + lane] = occd ? lrow[blk] : 0ull;
      wv[64 * blk + lane] = occd ? lval[blk] : 0u;  // empty slots: row 0, value 0
    }
  wc[64 * nblk + lane] = 0;  // the 64 slots after the window
  wv[64 * nblk + lane] = 0;
  __syncthreads();
  // parallel phase
  const uint64_t pend = a.spill_occ[lastL];
  bool active = (pend >> lane) & 1ull;
  uint64_t c = active ? a.spillC[lastL * 64 + lane] : 0ull;
  uint32_t v = active ? a.spillV[lastL * 64 + lane] : 0u;
  uint32_t i = lane;  // relative to start: the left group ends where the right one begins
  bool over = false, bad = false, internal = false;
  uint32_t guard = 64u * (win + 64u) + 1024u;
  while (__any(active)) {
    if (guard-- == 0) {
      internal = true;
      break;
    }
    // unmasked steps as in the insertion kernel; a walk that leaves the
    // window stops on the zero slots after it (lanes whose row reduced to
    // zero may walk on past them: they only read, and their state is not
    // used again)
    bool conflict = false;
    uint64_t row = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      row = wc[i];
      const uint32_t rv = wv[i];
      const uint64_t cx = c ^ row;
      const uint32_t vx = v ^ rv;
      const bool nz = cx != 0;  // else redundant (vx = 0) or inconsistent
      conflict = conflict || (active && !nz && vx != 0);
      active = active && nz;
      const uint32_t j = (uint32_t)__builtin_ctzg(cx, 64);
      c = cx >> (j & 63u);
      v = vx;
      i += j;
    }
    if (active && i >= win) {  // left the window: finish later
      over = true;
      active = false;
    } else if (active && row == 0) {
      const uint64_t old = atomicCAS((unsigned long long*)&wc[i], 0ull, (unsigned long long)c);
      if (old == 0) {
        wv[i] = v;
        active = false;
      }
    }
    if (__any(conflict)) {
      bad = true;
      break;
    }
  }
  bad = bad || internal;
  __syncthreads();
  // write the window back with its occupancy
  for (uint32_t blk = 0; blk < win / 64; ++blk) {
    const uint64_t slot = start + 64ull * blk + lane;
    const uint64_t row = wc[64 * blk + lane];
    const uint64_t word = __ballot(row != 0);
    if (slot < endR) {
      if (row) {
        a.rowsC[slot] = row;
        a.rowsV[slot] = wv[64 * blk + lane];
      }
      if (lane == 0) a.occ[slot / 64] = word;
    } else {
      if (row) {
        a.spillC[lastR * 64 + (slot - endR)] = row;
        a.spillV[lastR * 64 + (slot - endR)] = wv[64 * blk + lane];
      }
      if (lane == 0) a.spill_occ[lastR] = word;
    }
  }
  // rows that left the window, one by one in global memory (rare)
  const uint64_t overm = __ballot(over && !bad);
  oc_[lane] = c;
  ov_[lane] = v;
  oi_[lane] = i;
  __syncthreads();
  if (lane == 0) {
    uint64_t rest = overm;
    while (rest && !bad) {
      const uint32_t t0 = (uint32_t)__builtin_ctzll(rest);
      rest &= rest - 1;
      uint64_t cc = oc_[t0];
      uint32_t vv = ov_[t0];
      uint64_t slot = start + oi_[t0];
      while (true) {
        bool occupied;
        uint64_t row;
        uint32_t rv;
        if (slot < endR) {
          occupied = (a.occ[slot / 64] >> (slot % 64)) & 1ull;
          row = a.rowsC[slot];
          rv = a.rowsV[slot];
        } else {
          const uint64_t t = slot - endR;
          if (t >= 64) {  // unreachable: rows end at most 62 slots past the group
            bad = internal = true;
            break;
          }
          occupied = (a.spill_occ[lastR] >> t) & 1ull;
          row = a.spillC[lastR * 64 + t];
          rv = a.spillV[lastR * 64 + t];
        }
        if (!occupied) {
          if (slot < endR) {
            a.rowsC[slot] = cc;
            a.rowsV[slot] = vv;
            a.occ[slot / 64] |= 1ull << (slot % 64);
          } else {
            const uint64_t t = slot - endR;
            a.spillC[lastR * 64 + t] = cc;
            a.spillV[lastR * 64 + t] = vv;
            a.spill_occ[lastR] |= 1ull << t;
          }
          break;
        }
        cc ^= row;
        vv ^= rv;
        if (cc == 0) {
          if (vv != 0) bad = true;  // inconsistent: this table size fails
          break;
        }
        if (cc & 1ull) {  // a stored row always has its leading bit: corrupt state
          bad = internal = true;
          break;
        }
        const uint32_t j = (uint32_t)__builtin_ctzll(cc);
        cc >>= j;
        slot += j;
      }
    }
    if (bad) a.fail[sp.j] = internal ? 2u : 1u;
    a.spill_occ[lastL] = 0;
  }
}

hipError_t final_merge(const FinalArgs& a, uint64_t max_segments, hipStream_t s) {
  for (uint64_t G = 1; G < max_segments; G *= 2) {
    k_merge<<<(unsigned)a.g.nranges, 64, 0, s>>>(a, (uint32_t)G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per segment (one wave), back-substitute with the 63 values after the
// segment unknown: every slot's value is z0 (zero boundary) xor the boundary
// values selected by a 63-bit dependence word X. Lane b < 63 carries bit b
// of X through a 64-bit window (bit k = X[i+1+k] bit b; past the segment end
// X[end+k] is the unit word e_k), lane c < r carries column c of z0; the
// first 63 slots' words are assembled with ballots. Lane t holds row and
// value of slot t of the current block, and every step takes the slot's
// row and value from it with v_readlane (scalar results), so the steps wait
// for no memory round trip (through LDS, each step waited for two).
__global__ __launch_bounds__(64) void k_final_partial(FinalArgs a) {
  const LayerGeom g = a.g;
  const uint32_t lane = threadIdx.x;
  const uint64_t p = blockIdx.x;
  if (p >= g.nranges) return;
  const SegBounds sb = seg_bounds(p, g);
  const uint64_t start = sb.start, end = sb.end;
  const uint32_t r = g.rbits[sb.j];
  const uint64_t zmask = r >= 32 ? 0xffffffffull : ((1ull << r) - 1);
  uint64_t wx = lane < 63 ? (1ull << lane) : 0ull;
  uint64_t wz = 0;
  // free slots hold row 0 and value 0, so they give 0 without a test; the
  // next block's row and value load while this one is processed
  const uint64_t kb = start / 64;
  uint64_t k = end / 64;
  uint64_t pc = 0;
  uint32_t pv = 0;
  if (k > kb) {
    pc = a.rowsC[(k - 1) * 64 + lane];
    pv = a.rowsV[(k - 1) * 64 + lane];
  }
  const uint32_t vsh = lane < 32 ? lane : 31u;  // lanes >= 32 carry no value column
  const uint32_t vmask = lane < 32 ? 1u : 0u;
  // words of the first 63 slots: lane t keeps slot start+t's, stored at the end
  uint64_t myX = 0;
  uint32_t myZ = 0;
  while (k-- > kb) {
    const uint64_t cc = pc >> 1;  // rows without their leading bit
    const uint32_t clo = (uint32_t)cc, chi = (uint32_t)(cc >> 32), cv = pv;
    if (k > kb) {
      pc = a.rowsC[(k - 1) * 64 + lane];
      pv = a.rowsV[(k - 1) * 64 + lane];
    }
    auto step = [&](int tt, uint64_t& xb, uint64_t& zb) {
      const uint32_t Clo = __builtin_amdgcn_readlane(clo, tt);
      const uint32_t Chi = __builtin_amdgcn_readlane(chi, tt);
      const uint32_t vbit = (__builtin_amdgcn_readlane(cv, tt) >> vsh) & vmask;
      const uint32_t x1 = (Clo & (uint32_t)wx) ^ (Chi & (uint32_t)(wx >> 32));
      const uint32_t x2 = (Clo & (uint32_t)wz) ^ (Chi & (uint32_t)(wz >> 32));
      xb = (uint32_t)__popc(x1) & 1u;
      zb = ((uint32_t)__popc(x2) + vbit) & 1u;
      wx = (wx << 1) | xb;
      wz = (wz << 1) | zb;
    };
    if (k > kb) {  // start and end are multiples of 64: only block kb holds the first slots
#pragma unroll 16
      for (int tt = 63; tt >= 0; --tt) {
        uint64_t xb, zb;
        step(tt, xb, zb);
      }
    } else {
#pragma unroll 16
      for (int tt = 63; tt >= 0; --tt) {
        uint64_t xb, zb;
        step(tt, xb, zb);
        const uint64_t X = __ballot(xb != 0) & 0x7fffffffffffffffull;
        const uint32_t Z = (uint32_t)(__ballot(zb != 0) & zmask);
        myX = (uint32_t)tt == lane ? X : myX;
        myZ = (uint32_t)tt == lane ? Z : myZ;
      }
    }
  }
  if (lane < 63) {
    a.xfirst[p * 64 + lane] = myX;
    a.z0first[p * 64 + lane] = myZ;
  }
}

// One wave per structure, from its last segment down: the boundary of
// segment p-1 is the true value of segment p's first 63 slots = z0 xor (X
// applied to segment p's boundary). Lane t holds boundary value t; column c
// of the boundary is gathered into one word with a ballot, so X applied to
// it is one AND and a parity per column. The segments' X and z0 words do not
// depend on the scan, so they are loaded kScanChunk segments at a time into
// LDS (the loads overlap) and the sequential part reads LDS only.
// RC >= r columns, a compile-time count so that the column ballots of one
// segment are independent instructions (columns >= r are zero).
constexpr uint32_t kScanChunk = 32;
template <uint32_t RC>
__global__ __launch_bounds__(64) void k_final_scan(FinalArgs a) {
  __shared__ uint64_t sx[kScanChunk][64];
  __shared__ uint32_t sz[kScanChunk][64];
  const uint32_t t = threadIdx.x;
  const LayerGeom g = a.g;
  const uint32_t j = blockIdx.x;
  const uint64_t first = g.range_base[j], last = g.range_base[j + 1];
  uint32_t b = 0;  // nothing lies past the structure's last segment
  for (uint64_t hi = last; hi > first;) {
    const uint64_t lo = hi - first > kScanChunk ? hi - kScanChunk : first;
    // every load of the chunk is issued before the first LDS store (entries
    // past hi repeat segment hi-1 and are never read)
    uint64_t rx[kScanChunk];
    uint32_t rz[kScanChunk];
#pragma unroll
    for (uint32_t k = 0; k < kScanChunk; ++k) {
      const uint64_t p = lo + k < hi ? lo + k : hi - 1;
      rx[k] = t < 63 ? a.xfirst[p * 64 + t] : 0ull;
      rz[k] = t < 63 ? a.z0first[p * 64 + t] : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < kScanChunk; ++k) {
      sx[k][t] = rx[k];
      sz[k][t] = rz[k];
    }
    __syncthreads();
    for (uint64_t p = hi; p-- > lo;) {
      a.bnd[p * 64 + t] = b;
      const uint64_t X = sx[p - lo][t];
      uint32_t nb = sz[p - lo][t];
#pragma unroll
      for (uint32_t c = 0; c < RC; ++c) {
        const uint64_t col = __ballot(((b >> c) & 1u) != 0) & 0x7fffffffffffffffull;
        const uint32_t x = ((uint32_t)X & (uint32_t)col) ^ ((uint32_t)(X >> 32) & (uint32_t)(col >> 32));
        nb ^= ((uint32_t)__popc(x) & 1u) << c;
      }
      b = t < 63 ? nb : 0u;
    }
    __syncthreads();
    hi = lo;
  }
}

hipError_t final_boundaries(const FinalArgs& a, hipStream_t s) {
  const uint64_t P = a.g.nranges;
  k_final_partial<<<(unsigned)P, 64, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.g.r <= 8)
    k_final_scan<8><<<a.g.J, 64, 0, s>>>(a);
  else if (a.g.r <= 16)
    k_final_scan<16><<<a.g.J, 64, 0, s>>>(a);
  else
    k_final_scan<32><<<a.g.J, 64, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Codes and bumped keys
// ---------------------------------------------------------------------------
__global__ void k_pack_codes(const uint8_t* __restrict__ code8, LayerGeom g,
                             uint64_t ncode_words, uint64_t* __restrict__ words) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ncode_words) return;
  const uint32_t j = find_struct(g.code_base, g.J, w);
  const uint64_t B = g.bucket_base[j + 1] - g.bucket_base[j];
  const uint64_t wl = w - g.code_base[j];
  // the 32 loads are unconditional (past the structure's end its last code
  // is read again and not used), so that they are all in flight together
  const uint8_t* c = code8 + g.bucket_base[j];
  uint32_t cv[32];
#pragma unroll
  for (uint32_t t = 0; t < 32; ++t) {
    const uint64_t b = wl * 32 + t;
    cv[t] = c[b < B ? b : B - 1];
  }
  uint64_t word = 0;
#pragma unroll
  for (uint32_t t = 0; t < 32; ++t)
    if (wl * 32 + t < B) word |= (uint64_t)(cv[t] & 3u) << (2 * t);
  words[w] = word;
}

hipError_t pack_codes(const uint8_t* code8, const LayerGeom& g, uint64_t ncode_words,
                      uint64_t* words, hipStream_t s) {
  if (ncode_words == 0) return hipSuccess;
  k_pack_codes<<<(unsigned)((ncode_words + 255) / 256), 256, 0, s>>>(code8, g, ncode_words,
                                                                     words);
  return hipGetLastError();
}

// 1+-bit thresholds (Sec. 2: one bit per bucket, the exact threshold only
// for buckets that bump). Per structure: bit words (64 buckets each), the
// thresholds minus 1 of the bumping buckets in bucket order (one byte each),
// and a rank directory - the set bits before every block of 8 bit words -
// that finds a bucket's threshold with at most 8 popcounts.
// Pass 1: the bit words and their popcounts (pc, scanned afterwards).
__global__ void k_pack_bits(const uint8_t* __restrict__ code8, LayerGeom g, uint64_t nwords,
                            uint64_t* __restrict__ bits, uint32_t* __restrict__ pc) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const uint32_t j = find_struct(g.code_base, g.J, w);
  const uint64_t bb = g.bucket_base[j];
  const uint64_t B = g.bucket_base[j + 1] - bb;
  const uint64_t wl = w - g.code_base[j];
  uint64_t word = 0;
  for (uint64_t t = 0; t < 64; ++t) {
    const uint64_t b = wl * 64 + t;
    if (b < B && code8[bb + b]) word |= 1ull << t;
  }
  bits[w] = word;
  pc[w] = (uint32_t)__popcll(word);
}

// Pass 2 (pc scanned, pc[nwords] = total): thresholds, rank directory and
// the number of thresholds of every structure.
__global__ void k_pack_thr(const uint8_t* __restrict__ code8, LayerGeom g, uint64_t nwords,
                           const uint64_t* __restrict__ bits, const uint32_t* __restrict__ pc,
                           uint8_t* __restrict__ thr, uint32_t* __restrict__ rank,
                           uint32_t* __restrict__ kcount) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const uint32_t j = find_struct(g.code_base, g.J, w);
  const uint64_t bb = g.bucket_base[j];
  const uint64_t wl = w - g.code_base[j];
  const uint32_t base = pc[g.code_base[j]];
  uint32_t k = pc[w] - base;
  if (wl % 8 == 0) rank[g.rank_base[j] + wl / 8] = k;
  uint64_t word = bits[w];
  while (word) {
    const uint32_t t = (uint32_t)__builtin_ctzll(word);
    thr[g.thr_base[j] + k] = (uint8_t)(code8[bb + wl * 64 + t] - 1u);
    ++k;
    word &= word - 1;
  }
  if (w + 1 == g.code_base[j + 1]) kcount[j] = pc[w + 1] - base;
}

hipError_t pack_thresholds(const uint8_t* code8, const LayerGeom& g, uint64_t nwords,
                           uint64_t* bits, uint32_t* pc, uint32_t* scan_tmp, uint8_t* thr,
                           uint32_t* rank, uint32_t* kcount, hipStream_t s) {
  if (nwords == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nwords + 255) / 256);
  k_pack_bits<<<blocks, 256, 0, s>>>(code8, g, nwords, bits, pc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(pc + nwords, 0, 4, s)) != hipSuccess) return e;
  if ((e = scan_exclusive(pc, nwords + 1, scan_tmp, s)) != hipSuccess) return e;
  k_pack_thr<<<blocks, 256, 0, s>>>(code8, g, nwords, bits, pc, thr, rank, kcount);
  return hipGetLastError();
}

__global__ void k_struct_offsets(const uint32_t* __restrict__ off, LayerGeom g,
                                 uint32_t* __restrict__ out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= g.J) out[j] = off[g.bucket_base[j]];
}

hipError_t struct_offsets(const uint32_t* off, const LayerGeom& g, uint32_t* out, hipStream_t s) {
  k_struct_offsets<<<(g.J + 256) / 256, 256, 0, s>>>(off, g, out);
  return hipGetLastError();
}

// One wave per 64 consecutive buckets: the lanes take the wave's bumped
// records in output order (consecutive outputs, so the writes coalesce and
// a bucket's records are read as a run), each finding its record's bucket by
// a binary search over the 64 buckets' first output positions.
__global__ __launch_bounds__(256) void k_gather(const Rec* __restrict__ rec,
                                                const uint32_t* __restrict__ bstart,
                                                const uint32_t* __restrict__ off, uint64_t B,
                                                uint64_t* __restrict__ nk,
                                                uint32_t* __restrict__ nv) {
  const uint64_t b0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) / 64 * 64;
  if (b0 >= B) return;  // the whole wave
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t beta = b0 + lane;
  const uint64_t bend = b0 + 64 < B ? b0 + 64 : B;
  // this lane's bucket: first output position and the item of its first bumped record
  const uint32_t o = off[beta < B ? beta : B];
  uint32_t first = 0;
  if (beta < B) first = bstart[beta + 1] - (off[beta + 1] - o) + (uint32_t)beta + 1;
  const uint32_t base = off[b0], end = off[bend];
  for (uint32_t k = base + lane; k - lane < end; k += 64) {
    uint32_t l = 0;  // last lane whose bucket starts at or before k
#pragma unroll
    for (uint32_t step = 32; step >= 1; step >>= 1) {
      const uint32_t c = l + step;
      const uint32_t oc = (uint32_t)__shfl((int)o, (int)(c & 63u), 64);
      if (c < 64 && oc <= k) l = c;
    }
    const uint32_t ol = (uint32_t)__shfl((int)o, (int)l, 64);
    const uint32_t fl = (uint32_t)__shfl((int)first, (int)l, 64);
    if (k < end) {
      const Rec r = rec[fl + (k - ol)];
      nk[k] = r.c;
      nv[k] = meta_value(r.meta);
    }
  }
}

hipError_t gather_bumped(const Rec* rec, const uint32_t* bstart, const uint32_t* off, uint64_t B,
                         uint64_t* next_keys, uint32_t* next_vals, hipStream_t s) {
  if (B == 0) return hipSuccess;
  const uint64_t waves = (B + 63) / 64;
  k_gather<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(rec, bstart, off, B, next_keys,
                                                       next_vals);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Input concatenation (requests built together)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_concat(const uint64_t* __restrict__ tab, uint32_t J,
                                                uint64_t n, uint64_t* __restrict__ out_keys,
                                                void* __restrict__ out_vals, uint32_t out_vb) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t* off = tab + 2 * (uint64_t)J;
  const uint32_t j = find_struct(off, J, i);
  const uint64_t k = i - off[j];
  out_keys[i] = reinterpret_cast<const uint64_t*>(tab[j])[k];
  if (!out_vals) return;
  const void* src = reinterpret_cast<const void*>(tab[J + j]);
  const uint32_t vb = (uint32_t)tab[3 * (uint64_t)J + 1 + j];
  uint32_t v = 0;
  if (src) {
    if (vb == 1)
      v = reinterpret_cast<const uint8_t*>(src)[k];
    else if (vb == 2)
      v = reinterpret_cast<const uint16_t*>(src)[k];
    else
      v = reinterpret_cast<const uint32_t*>(src)[k];
  }
  if (out_vb == 1)
    reinterpret_cast<uint8_t*>(out_vals)[i] = (uint8_t)v;
  else if (out_vb == 2)
    reinterpret_cast<uint16_t*>(out_vals)[i] = (uint16_t)v;
  else
    reinterpret_cast<uint32_t*>(out_vals)[i] = v;
}

hipError_t concat_inputs(const uint64_t* tab, uint32_t J, uint64_t n, uint64_t* out_keys,
                         void* out_vals, uint32_t out_vb, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_concat<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tab, J, n, out_keys, out_vals, out_vb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthetic inputs (autotuner): SplitMix64 stream outputs, element i of the
// stream seeded with `seed` is mix(seed + (start + i + 1) * golden gamma)
// (Steele, Lea, Flood, OOPSLA 2014)
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + ctr * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_fill_stream(uint64_t* __restrict__ keys, void* vals,
                                                     uint32_t vb, uint64_t n, uint64_t seed,
                                                     uint64_t vseed, uint64_t vmask) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = splitmix(seed, i + 1);
  if (!vals) return;
  const uint64_t v = splitmix(vseed, i + 1) & vmask;
  if (vb == 1)
    reinterpret_cast<uint8_t*>(vals)[i] = (uint8_t)v;
  else if (vb == 2)
    reinterpret_cast<uint16_t*>(vals)[i] = (uint16_t)v;
  else
    reinterpret_cast<uint32_t*>(vals)[i] = (uint32_t)v;
}

hipError_t fill_stream(uint64_t* keys, void* vals, uint32_t vb, uint64_t n, uint64_t seed,
                       uint64_t vseed, uint64_t vmask, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill_stream<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(keys, vals, vb, n, seed, vseed,
                                                              vmask);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Query: one lane per key
// ---------------------------------------------------------------------------
// r-bit result of one layer: parity of c AND the 64-slot window at s, per
// column, from the column-interleaved words of blocks s/64 and s/64 + 1
// AL: w is 16-byte aligned (R even), so the words load two at a time
template <int R, bool AL>
__device__ inline uint32_t window_parity(const uint64_t* w, uint32_t sh, uint64_t c) {
  uint64_t lo[R], hi[R];
  if constexpr (AL) {
    const uint4* p = reinterpret_cast<const uint4*>(w);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const uint4 a = p[k];
      lo[2 * k] = (uint64_t)a.x | ((uint64_t)a.y << 32);
      lo[2 * k + 1] = (uint64_t)a.z | ((uint64_t)a.w << 32);
    }
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const uint4 a = sh ? p[R / 2 + k] : make_uint4(0, 0, 0, 0);
      hi[2 * k] = (uint64_t)a.x | ((uint64_t)a.y << 32);
      hi[2 * k + 1] = (uint64_t)a.z | ((uint64_t)a.w << 32);
    }
  } else {
#pragma unroll
    for (int col = 0; col < R; ++col) {
      lo[col] = w[col];
      hi[col] = sh ? w[R + col] : 0ull;
    }
  }
  uint32_t res = 0;
#pragma unroll
  for (int col = 0; col < R; ++col) {
    const uint64_t win = sh ? ((lo[col] >> sh) | (hi[col] << (64 - sh))) : lo[col];
    res |= ((uint32_t)__popcll(win & c) & 1u) << col;
  }
  return res;
}
__device__ inline uint32_t window_parity_any(const uint64_t* w, uint32_t r, uint32_t sh,
                                             uint64_t c) {
  uint32_t res = 0;
  for (uint32_t col = 0; col < r; ++col) {
    uint64_t win = w[col] >> sh;
    if (sh) win |= w[r + col] << (64 - sh);
    res |= ((uint32_t)__popcll(win & c) & 1u) << col;
  }
  return res;
}

// Query: one lane per key. Per layer, the bucket's code word and the table
// words of the key's window are independent loads (both follow from the start
// slot), so they are issued together; the threshold then decides whether
// the layer answers.
template <typename OT, int RC, bool AL>
__global__ __launch_bounds__(256) void k_query(QueryPlan plan, const uint64_t* __restrict__ keys,
                                               uint64_t n, OT* __restrict__ out,
                                               uint32_t contains, uint64_t fp_salt) {
  const uint64_t idx = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const uint64_t key = keys[idx];
  const uint32_t r = plan.r;
  uint32_t res = 0;
  for (uint32_t l = 0; l < plan.nlayers; ++l) {
    const QueryLayer& L = plan.layer[l];
    if (L.empty) break;
    const uint64_t s = __umul64hi(mix64(key ^ L.salt_s), L.span);
    const uint64_t c = mix64(key ^ L.salt_c) | 1ull;
    const uint32_t sh = (uint32_t)s & 63u;
    const uint64_t* w = L.W + (s >> 6) * r;
    const uint64_t beta = s >> 6;
    const uint64_t cw = L.plain ? 0ull : L.codes[L.thr_mode ? (beta >> 6) : (beta >> 5)];
    uint32_t val;
    if constexpr (RC > 0)
      val = window_parity<RC, AL>(w, sh, c);
    else
      val = window_parity_any(w, r, sh, c);
    if (!L.plain) {
      uint32_t th;
      if (L.thr_mode) {  // 1+-bit: a set bit sends the lookup to the threshold bytes
        th = 0;
        const uint32_t bit = (uint32_t)(beta & 63);
        if ((cw >> bit) & 1ull) {
          const uint64_t wi = beta >> 6, blk = wi >> 3;
          uint32_t rk = L.rank[blk];
          for (uint64_t x = blk << 3; x < wi; ++x) rk += (uint32_t)__popcll(L.codes[x]);
          rk += (uint32_t)__popcll(cw & ((1ull << bit) - 1ull));
          th = (uint32_t)L.thr[rk] + 1u;
        }
      } else {
        const uint32_t code = (uint32_t)(cw >> (2 * (beta & 31))) & 3u;
        th = code == 0 ? 0u : (code == 1 ? L.t_lo : (code == 2 ? L.t_hi : 64u));
      }
      if (sh < th) continue;
    }
    res = val;
    break;
  }
  if (contains)
    out[idx] = (OT)(res == (uint32_t)(mix64(key ^ fp_salt) >> (64 - r)));
  else
    out[idx] = (OT)res;
}

hipError_t query(const QueryPlan& plan, const uint64_t* keys, uint64_t n, void* out,
                 uint32_t out_bytes, uint32_t contains, uint64_t fp_salt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  const bool al = plan.aligned != 0;
  if (out_bytes == 1 && plan.r == 8 && al)
    k_query<uint8_t, 8, true><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 1 && plan.r == 8)
    k_query<uint8_t, 8, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 1 && plan.r == 1)
    k_query<uint8_t, 1, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 1 && plan.r == 16 && al)  // membership answers of a 16-bit filter
    k_query<uint8_t, 16, true><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 1 && plan.r == 16)
    k_query<uint8_t, 16, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 1)
    k_query<uint8_t, 0, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 2 && plan.r == 16 && al)
    k_query<uint16_t, 16, true><<<blocks, 256, 0, s>>>(plan, keys, n, (uint16_t*)out, contains,
                                                       fp_salt);
  else if (out_bytes == 2 && plan.r == 16)
    k_query<uint16_t, 16, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint16_t*)out, contains,
                                                        fp_salt);
  else if (out_bytes == 2)
    k_query<uint16_t, 0, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint16_t*)out, contains, fp_salt);
  else
    k_query<uint32_t, 0, false><<<blocks, 256, 0, s>>>(plan, keys, n, (uint32_t*)out, contains, fp_salt);
  return hipGetLastError();
}

}  // namespace burr
