// burr_dev.h - device-side definitions shared by the HIP kernels of the
// BuRR library (hash, layer geometry, record layout). Host code of the
// library includes it for the launch structs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace burr {

constexpr uint32_t kWidth = 64;           // ribbon width w (Sec. 2)
constexpr uint32_t kBucket = 64;          // bucket size b handled by the kernels
constexpr uint32_t kRing = 128;           // LDS ring rows per range: bucket q touches slots [64q, 64q+126]
constexpr uint32_t kSubBuckets = 64;      // sort sub-bin: 64 consecutive buckets
constexpr uint32_t kMaxDigits = 2048;     // most bins (sub-bins) of a partition level

// MurmurHash3's 64-bit finalizer (public domain), used as the key mixer.
__host__ __device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Geometry of one layer of one or more structures built together (a single
// build is one structure). Passed by value to kernels; the per-structure
// tables live in device memory. Structure j of the layer owns
//   keys         [key_off[j],     key_off[j+1])      of the layer's key array
//   buckets      [bucket_base[j], bucket_base[j+1])  (global bucket space)
//   ranges       [range_base[j],  range_base[j+1])   (segments in the final layer)
//   table words  [word_base[j],   word_base[j+1])    solution words
//   code words   [code_base[j],   code_base[j+1])
// and hashes its keys into span[j] = m_j - 63 possible start slots.
struct LayerGeom {
  uint64_t salt_s;   // start-position salt of the layer
  uint64_t salt_c;   // coefficient-row salt of the layer
  uint64_t m;        // total slots = 64 * nbuckets
  uint64_t nbuckets; // total buckets
  uint64_t nranges;  // total ranges (final layer: segments)
  uint64_t nkeys;    // total keys
  uint32_t t_lo, t_hi;
  uint32_t plain;    // 1: final plain ribbon (one chunk, conflicts fail)
  uint32_t r;        // largest value width of the structures
  uint32_t J;        // structures in the layer
  uint32_t thr_mode; // 0: 2-bit thresholds, 1: 1+-bit thresholds (Sec. 2)
  uint32_t cut_strategy, cut_search;  // range ends (Sec. 3 "Selecting Cut Points")
  const uint64_t* key_off;
  const uint64_t* span;
  const uint64_t* bucket_base;
  const uint64_t* range_base;
  const uint64_t* word_base;
  const uint64_t* code_base;   // 2-bit: code words; 1+-bit: bit words
  const uint64_t* thr_base;    // 1+-bit: first threshold byte of structure j
  const uint64_t* rank_base;   // 1+-bit: first rank-directory entry of structure j
  const uint32_t* rbits;
  // first global bucket of every global range (nranges + 1 entries; the
  // cut points), or null: the equal split of each structure's buckets
  const uint32_t* rfirst;
};

// buckets [first, end) of global range rho of a BuRR layer: from the cut
// points when the layer has them, else the equal integer split of
// structure js's buckets
__device__ inline void range_buckets(const LayerGeom& g, uint32_t js, uint64_t rho,
                                     uint64_t& first, uint64_t& end) {
  if (g.rfirst) {
    first = g.rfirst[rho];
    end = g.rfirst[rho + 1];
    return;
  }
  const uint64_t B = g.bucket_base[js + 1] - g.bucket_base[js];
  const uint64_t Rn = g.range_base[js + 1] - g.range_base[js];
  const uint64_t lr = rho - g.range_base[js];
  first = g.bucket_base[js] + lr * B / Rn;
  end = g.bucket_base[js] + (lr + 1) * B / Rn;
}

// largest j < J with base[j] <= x (base strictly increasing, base[0] <= x)
__device__ inline uint32_t find_struct(const uint64_t* base, uint32_t J, uint64_t x) {
  uint32_t lo = 0, hi = J;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (base[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// start slot in [0, span-1] = [0, m-64]: high word of mix64(key^salt) * span
__device__ inline uint64_t start_of(uint64_t key, uint64_t salt, uint64_t span) {
  return __umul64hi(mix64(key ^ salt), span);
}
// coefficient row; bit j <-> slot s+j, bit 0 always set
__device__ inline uint64_t row_of(uint64_t key, const LayerGeom& g) {
  return mix64(key ^ g.salt_c) | 1ull;
}
// position of a key's chunk in the insertion order of its bucket:
// 0 = offsets [t_hi,64) (chunk 3, inserted first), 1 = [t_lo,t_hi), 2 = [0,t_lo)
__device__ inline uint32_t rank_of(uint32_t o, const LayerGeom& g) {
  if (g.plain) return 0;
  return o >= g.t_hi ? 0u : (o >= g.t_lo ? 1u : 2u);
}
// sort digits per bucket: 3 chunks (2-bit thresholds, final layer), or one
// per offset in decreasing order (1+-bit thresholds: any offset can be the
// threshold, so a bucket's records are ordered by offset)
__device__ __host__ inline uint32_t digits_per_bucket(const LayerGeom& g) {
  return (g.thr_mode == 1 && !g.plain) ? 64u : 3u;
}

// One 16-byte element of a layer's item stream. The stream holds, for every
// bucket in order, a header item followed by the bucket's records in chunk
// (rank) order - with 1+-bit thresholds in decreasing offset order:
//   header : c = number of records | (largest offset << 32) | (records at
//            offset 0 << 40), meta = records of rank 0 | records of rank 1
//            << 32 (2-bit thresholds)
//   record : c = key, meta = value (bits 0..31) | offset in the bucket
//            (bits 32..37) | rank (bits 40..41)
// The record of sorted key position p in bucket beta sits at item p+beta+1,
// the header of bucket beta at item bstart[beta]+beta.
struct alignas(16) Rec {
  uint64_t c;
  uint64_t meta;
};
__device__ inline uint32_t head_count(const Rec& h) { return (uint32_t)h.c; }

__device__ inline uint32_t meta_value(uint64_t meta) { return (uint32_t)meta; }
__device__ inline uint32_t meta_offset(uint64_t meta) { return (uint32_t)(meta >> 32) & 63u; }
__device__ inline uint32_t meta_rank(uint64_t meta) { return (uint32_t)(meta >> 40) & 3u; }

// Query-side description of one layer (BuRR layers and the final one).
struct QueryLayer {
  uint64_t salt_s, salt_c, span;
  const uint64_t* codes; // 2-bit: packed codes, bucket beta at bits 2*(beta%32) of word beta/32;
                         // 1+-bit: bit beta%64 of word beta/64 set if the bucket bumps
  const uint64_t* W;     // column-interleaved solution words, W[k*r + col]
  const uint32_t* rank;  // 1+-bit: set bits before each block of 8 bit words
  const uint8_t* thr;    // 1+-bit: threshold - 1 of each bumping bucket, in bucket order
  uint32_t t_lo, t_hi;
  uint32_t plain;        // final layer: no threshold check
  uint32_t empty;        // final layer without keys: answer 0
  uint32_t thr_mode;     // 0: 2-bit, 1: 1+-bit thresholds
  uint32_t pad;
};

constexpr int kMaxQueryLayers = 33;
struct QueryPlan {
  QueryLayer layer[kMaxQueryLayers];
  uint32_t nlayers; // BuRR layers + 1 (final)
  uint32_t r;
  uint32_t aligned; // every layer's W is 16-byte aligned and r is even: 16-byte loads
};

}  // namespace burr
