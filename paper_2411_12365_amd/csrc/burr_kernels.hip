// burr_kernels.hip - HIP kernels of the BuRR library for gfx950 (CDNA4).
//
// Per layer (Sec. 2 and Sec. 3 of the paper):
//   sort      : two-level partition of the keys by (bucket, chunk); level 1
//               scatters into coarse bins of 2048 buckets through LDS
//               histograms, level 2 orders one bin per workgroup in LDS and
//               writes 16-byte records (row + value/offset/chunk)
//   solve     : one lane per range; banded GF(2) insertion against a ring of
//               128 rows in LDS, bucket by bucket, chunks of decreasing
//               offset, 2-bit thresholds, forced bumps at the range end
//   backsub   : one lane per range, column-interleaved output words
//   gather    : bumped keys (a suffix of every bucket) -> next layer input
//   query     : one lane per key, layer walk, two-word window, popcount parity
#include "burr_kernels.h"

namespace burr {

// ---------------------------------------------------------------------------
// Block-wide exclusive scan (wave scan with cross-lane shuffles + LDS totals)
// ---------------------------------------------------------------------------
template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* wsum, uint32_t* total) {
  constexpr int NW = NT / 64;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= (uint32_t)d) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < (uint32_t)NW ? wsum[lane] : 0u;
    uint32_t wi = w;
#pragma unroll
    for (int d = 1; d < NW; d <<= 1) {
      uint32_t y = __shfl_up(wi, d, 64);
      if (lane >= (uint32_t)d) wi += y;
    }
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

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(uint32_t* data, size_t n,
                                                             uint32_t* sums) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t total;
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t tot = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? data[base + k] : 0u;
    tot += v[k];
  }
  uint32_t run = block_exclusive_scan<kScanThreads>(tot, wsum, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) data[base + k] = run;
    run += v[k];
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
  if (tiles == 1) {
    k_scan_tile<<<1, kScanThreads, 0, s>>>(data, n, nullptr);
    return hipGetLastError();
  }
  k_scan_tile<<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(tmp, tiles, tmp + tiles, s);
  if (e != hipSuccess) return e;
  k_scan_add<<<(unsigned)tiles, kScanThreads, 0, s>>>(data, n, tmp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sorting
// ---------------------------------------------------------------------------
constexpr int kL1Threads = 256;
constexpr int kL2Threads = 512;

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

__global__ __launch_bounds__(kL1Threads) void k_l1_hist(const uint64_t* __restrict__ keys,
                                                         LayerGeom g, uint32_t nbins,
                                                         uint32_t groups, uint64_t per_group,
                                                         uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < nbins; i += kL1Threads) hist[i] = 0;
  __syncthreads();
  const uint64_t lo = (uint64_t)blockIdx.x * per_group;
  const uint64_t hi = lo + per_group < g.nkeys ? lo + per_group : g.nkeys;
  KeyWalk w(g, lo + threadIdx.x);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kL1Threads) {
    w.advance(g, i);
    const uint64_t s = start_of(keys[i], g.salt_s, w.span);
    atomicAdd(&hist[(uint32_t)((w.bb + (s >> 6)) / kBucketsPerBin)], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nbins; i += kL1Threads)
    counts[(size_t)i * groups + blockIdx.x] = hist[i];
}

template <typename VT>
__global__ __launch_bounds__(kL1Threads) void k_l1_scatter(
    const uint64_t* __restrict__ keys, const VT* __restrict__ vals, LayerGeom g,
    uint32_t nbins, uint32_t groups, uint64_t per_group, const uint32_t* __restrict__ offs,
    uint32_t mask_values, uint32_t filter, uint64_t fp_salt, uint64_t* __restrict__ tk,
    uint32_t* __restrict__ tv, uint64_t* __restrict__ ts) {
  extern __shared__ uint32_t cur[];
  for (uint32_t i = threadIdx.x; i < nbins; i += kL1Threads)
    cur[i] = offs[(size_t)i * groups + blockIdx.x];
  __syncthreads();
  const uint64_t lo = (uint64_t)blockIdx.x * per_group;
  const uint64_t hi = lo + per_group < g.nkeys ? lo + per_group : g.nkeys;
  KeyWalk w(g, lo + threadIdx.x);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kL1Threads) {
    w.advance(g, i);
    const uint64_t key = keys[i];
    uint32_t v;
    if (filter && mask_values)
      v = (uint32_t)(mix64(key ^ fp_salt) >> (64 - w.r));
    else if (mask_values)
      v = (uint32_t)vals[i] & (w.r >= 32 ? 0xffffffffu : ((1u << w.r) - 1u));
    else
      v = (uint32_t)vals[i];
    const uint64_t slot = 64 * w.bb + start_of(key, g.salt_s, w.span);
    const uint32_t pos = atomicAdd(&cur[(uint32_t)((slot >> 6) / kBucketsPerBin)], 1u);
    tk[pos] = key;
    tv[pos] = v;
    ts[pos] = slot;
  }
}

// Forced threshold index of global bucket beta: the last bucket of a range
// that is not its structure's last range must bump every key that starts
// past its first slot (b = w = 64), so its threshold is the smallest 2-bit
// value above the largest offset of such a key (Sec. 3 "Bumping").
__device__ inline uint32_t forced_kf(uint64_t beta, uint32_t maxoff, uint32_t count,
                                     const LayerGeom& g) {
  if (g.plain || count == 0 || maxoff == 0) return 0;
  const uint32_t j = find_struct(g.bucket_base, g.J, beta);
  const uint64_t B = g.bucket_base[j + 1] - g.bucket_base[j];
  const uint64_t R = g.range_base[j + 1] - g.range_base[j];
  const uint64_t b = beta - g.bucket_base[j];
  const uint64_t rho = ((b + 1) * R - 1) / B;
  if (rho + 1 >= R) return 0;
  if ((rho + 1) * B / R != b + 1) return 0;
  return maxoff >= g.t_hi ? 3u : (maxoff >= g.t_lo ? 2u : 1u);
}

__global__ __launch_bounds__(kL2Threads) void k_l2_sort(
    const uint64_t* __restrict__ tk, const uint32_t* __restrict__ tv,
    const uint64_t* __restrict__ ts, LayerGeom g, uint32_t nbins, uint32_t groups,
    const uint32_t* __restrict__ offs, uint64_t* __restrict__ ok, Rec* __restrict__ items,
    uint32_t* __restrict__ bstart) {
  __shared__ uint32_t hist[kDigitsPerBin];
  __shared__ uint32_t maxoff[kBucketsPerBin];
  __shared__ uint32_t wsum[kL2Threads / 64];
  const uint32_t bin = blockIdx.x;
  const uint64_t lo = offs[(size_t)bin * groups];
  const uint64_t hi = bin + 1 < nbins ? offs[(size_t)(bin + 1) * groups] : g.nkeys;
  const uint64_t bbase = (uint64_t)bin * kBucketsPerBin;
  for (uint32_t i = threadIdx.x; i < kDigitsPerBin; i += kL2Threads) hist[i] = 0;
  for (uint32_t i = threadIdx.x; i < kBucketsPerBin; i += kL2Threads) maxoff[i] = 0;
  __syncthreads();
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kL2Threads) {
    const uint64_t slot = ts[i];
    const uint32_t b = (uint32_t)((slot >> 6) - bbase);
    const uint32_t o = (uint32_t)slot & 63u;
    atomicAdd(&hist[b * 3u + rank_of(o, g)], 1u);
    atomicMax(&maxoff[b], o);
  }
  __syncthreads();
  // exclusive scan of the 6144 digit counts, 12 per thread
  constexpr int kPer = kDigitsPerBin / kL2Threads;
  uint32_t loc[kPer];
  uint32_t tot = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    loc[k] = hist[threadIdx.x * kPer + k];
    tot += loc[k];
  }
  uint32_t run = block_exclusive_scan<kL2Threads>(tot, wsum, nullptr);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    hist[threadIdx.x * kPer + k] = run;
    run += loc[k];
  }
  __syncthreads();
  // bucket starts and bucket headers
  for (uint32_t b = threadIdx.x; b < kBucketsPerBin; b += kL2Threads) {
    const uint64_t beta = bbase + b;
    if (beta >= g.nbuckets) continue;
    const uint32_t first = hist[3 * b];
    const uint32_t next = (b + 1 < kBucketsPerBin) ? hist[3 * b + 3] : (uint32_t)(hi - lo);
    const uint32_t count = next - first;
    bstart[beta] = (uint32_t)(lo + first);
    Rec hd;
    hd.c = (uint64_t)count | ((uint64_t)forced_kf(beta, maxoff[b], count, g) << 32);
    hd.meta = 0;
    items[lo + first + beta] = hd;
  }
  if (bin + 1 == nbins && threadIdx.x == 0) bstart[g.nbuckets] = (uint32_t)hi;
  __syncthreads();
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kL2Threads) {
    const uint64_t key = tk[i];
    const uint64_t slot = ts[i];
    const uint32_t o = (uint32_t)slot & 63u;
    const uint32_t rk = rank_of(o, g);
    const uint64_t beta = slot >> 6;
    const uint32_t d = (uint32_t)(beta - bbase) * 3u + rk;
    const uint64_t pos = lo + atomicAdd(&hist[d], 1u);
    ok[pos] = key;
    Rec rc;
    rc.c = row_of(key, g);
    rc.meta = (uint64_t)tv[i] | ((uint64_t)o << 32) | ((uint64_t)rk << 40);
    items[pos + beta + 1] = rc;
  }
}

hipError_t sort_layer(const SortArgs& a, hipStream_t s) {
  const uint64_t per_group = (a.g.nkeys + a.groups - 1) / a.groups;
  const size_t hist_bytes = (size_t)a.nbins * sizeof(uint32_t);
  k_l1_hist<<<a.groups, kL1Threads, hist_bytes, s>>>(a.keys, a.g, a.nbins, a.groups,
                                                     per_group, a.counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(a.counts, (size_t)a.nbins * a.groups, a.scan_tmp, s);
  if (e != hipSuccess) return e;
  switch (a.vbytes) {
    case 1:
      k_l1_scatter<uint8_t><<<a.groups, kL1Threads, hist_bytes, s>>>(
          a.keys, (const uint8_t*)a.vals, a.g, a.nbins, a.groups, per_group, a.counts,
          a.mask_values, a.filter, a.fp_salt, a.tmp_keys, a.tmp_vals, a.tmp_slot);
      break;
    case 2:
      k_l1_scatter<uint16_t><<<a.groups, kL1Threads, hist_bytes, s>>>(
          a.keys, (const uint16_t*)a.vals, a.g, a.nbins, a.groups, per_group, a.counts,
          a.mask_values, a.filter, a.fp_salt, a.tmp_keys, a.tmp_vals, a.tmp_slot);
      break;
    default:
      k_l1_scatter<uint32_t><<<a.groups, kL1Threads, hist_bytes, s>>>(
          a.keys, (const uint32_t*)a.vals, a.g, a.nbins, a.groups, per_group, a.counts,
          a.mask_values, a.filter, a.fp_salt, a.tmp_keys, a.tmp_vals, a.tmp_slot);
      break;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_l2_sort<<<a.nbins, kL2Threads, 0, s>>>(a.tmp_keys, a.tmp_vals, a.tmp_slot, a.g, a.nbins,
                                           a.groups, a.counts, a.out_keys, a.out_rec, a.bstart);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Solve: one lane per range
// ---------------------------------------------------------------------------
// Every lane owns one range and walks its item stream (a header per bucket,
// then the bucket's records). The hot loop touches LDS only: the 128-row ring
// (coefficient rows and values) and a FIFO of the lane's next kFifo items.
// Global loads are issued once per round of kRoundIters iterations into
// registers and committed to the FIFO at the end of the round, so no wave
// waits on a global load inside a round.
//
// One iteration = K elimination steps for every lane still eliminating, then
// the outcome of finished equations, then the lanes that need their next item
// take it (usually the next record of the same bucket; bucket ends and
// headers are the rare path).
enum : uint32_t {
  ST_ELIM = 0,      // eliminating the current equation
  ST_PLACE = 1,     // found an empty slot at i
  ST_REDUNDANT = 2, // reduced to 0 = 0
  ST_CONFLICT = 3,  // reduced to 0 = v with v != 0
  ST_WANT = 4,      // needs item x
  ST_DONE = 5
};

#ifndef BURR_ROUND_ITERS
#define BURR_ROUND_ITERS 4
#endif
#ifndef BURR_SOLVE_K
#define BURR_SOLVE_K 8
#endif
constexpr int kFifo = 8;  // must match the 8 staged registers below
constexpr int kRoundIters = BURR_ROUND_ITERS;
constexpr uint32_t kNoSplit = 0xffffffffu;

// Records the state of the first lane that stops with an internal error.
__device__ inline void solve_diag(uint64_t* d, uint32_t code, uint64_t rho, uint32_t js,
                                  uint32_t x, uint32_t xend, uint32_t q, uint32_t nq,
                                  uint32_t state, bool open, uint32_t written, uint32_t rend,
                                  uint32_t kf, uint32_t curk, uint32_t i, uint64_t fb) {
  if (!d || atomicCAS((unsigned long long*)d, 0ull, 1ull) != 0ull) return;
  d[1] = code;
  d[2] = rho;
  d[3] = js;
  d[4] = x;
  d[5] = xend;
  d[6] = q;
  d[7] = nq;
  d[8] = state;
  d[9] = open;
  d[10] = written;
  d[11] = rend;
  d[12] = kf;
  d[13] = curk;
  d[14] = i;
  d[15] = fb;
}

template <typename VT>
constexpr size_t solve_lds_bytes() {
  return kRing * 64 * sizeof(uint64_t) + kFifo * 64 * sizeof(Rec) + kRing * 64 * sizeof(VT);
}

template <typename VT, int K>
__global__ __launch_bounds__(64) void k_solve(SolveArgs a) {
  extern __shared__ uint64_t lds[];
  uint64_t* ringC = lds;                                  // [kRing][64]
  Rec* fifo = reinterpret_cast<Rec*>(lds + kRing * 64);   // [kFifo][64]
  VT* ringV = reinterpret_cast<VT*>(fifo + kFifo * 64);   // [kRing][64]
  const LayerGeom g = a.g;
  const uint32_t lane = threadIdx.x;
  const uint64_t rho = (uint64_t)blockIdx.x * 64 + lane;

  uint32_t state = ST_DONE;
  uint64_t fb = 0;
  uint32_t nq = 0;
  uint32_t x = 0, xend = 0;  // item cursor and end of the range's items
  uint32_t js = 0;           // structure of the range
  if (rho < g.nranges) {
    js = find_struct(g.range_base, g.J, rho);
    const uint64_t B = g.bucket_base[js + 1] - g.bucket_base[js];
    const uint64_t R = g.range_base[js + 1] - g.range_base[js];
    const uint64_t lr = rho - g.range_base[js];
    const uint64_t f0 = lr * B / R;
    fb = g.bucket_base[js] + f0;
    nq = (uint32_t)((lr + 1) * B / R - f0);
    x = a.bstart[fb] + (uint32_t)fb;
    xend = a.bstart[fb + nq] + (uint32_t)(fb + nq);
    state = ST_WANT;
  }
  const uint64_t P0 = fb * 64;
  const uint32_t limit = 64u * nq;  // rows of kept keys end inside the range
  uint32_t q = 0xffffffffu;   // bucket index inside the range
  uint32_t rend = x;          // item index past the current bucket's records
  bool open = false;          // a bucket is being processed
  uint32_t kf = 0, code = 0, curk = 4, chunk_start = 0, split_at = kNoSplit;
  uint32_t i = 0, v = 0;
  uint64_t c = 0;
  uint64_t vm0 = 0, vm1 = 0;  // valid ring rows (bit p <-> ring position p)
  uint64_t pm0 = 0, pm1 = 0;  // rows placed by the current chunk
  uint64_t steps = 0;
#ifdef BURR_SOLVE_DEBUG
  uint64_t dbg_active = 0, dbg_elim = 0, dbg_stall = 0;
#endif

  // Each item needs at most 64 elimination steps, so a lane is done after
  // far fewer iterations than this cap; reaching it means a logic error, and
  // the lane stops (fail = 3) instead of keeping the wave alive.
  uint64_t iter_left = (uint64_t)(xend - x) * 80u + 4096u;
  uint32_t written = x;  // items [x, written) are in the FIFO
  const uint32_t last_item = a.nrec - 1;
  const uint4* rec4 = reinterpret_cast<const uint4*>(a.rec);
  uint4* fifo4 = reinterpret_cast<uint4*>(fifo);

  while (true) {
    const uint32_t ld0 = written > x ? written : x;
    const uint32_t ld1 = (x + kFifo < xend) ? x + kFifo : xend;
    const uint32_t ldn = ld1 > ld0 ? ld1 - ld0 : 0;
    // unconditional loads (clamped index) into named registers: a
    // conditional load, or an array, makes the compiler copy or spill the
    // value and wait for it at once
#define BURR_STAGE_LOAD(j) \
    const uint4 st##j = rec4[ld0 + j < last_item ? ld0 + j : last_item];
    BURR_STAGE_LOAD(0) BURR_STAGE_LOAD(1) BURR_STAGE_LOAD(2) BURR_STAGE_LOAD(3)
    BURR_STAGE_LOAD(4) BURR_STAGE_LOAD(5) BURR_STAGE_LOAD(6) BURR_STAGE_LOAD(7)
#undef BURR_STAGE_LOAD

    for (int it = 0; it < kRoundIters; ++it) {
      if (state != ST_DONE && iter_left-- == 0) {
        a.fail[js] = 3u;
        solve_diag(a.diag, 3, rho, js, x, xend, q, nq, state, open, written, rend, kf, curk, i,
                   fb);
        state = ST_DONE;
      }
#ifdef BURR_SOLVE_DEBUG
      dbg_active += state != ST_DONE;
      dbg_elim += state == ST_ELIM;
      dbg_stall += state == ST_WANT;
#endif
      // ---- K elimination steps ----
      // branch-free: every lane reads its ring row; selects keep the state
      // of lanes that are not eliminating
#pragma unroll
      for (int u = 0; u < K; ++u) {
        const uint32_t p = i & (kRing - 1);
        const uint64_t row = ringC[p * 64 + lane];
        const uint32_t rv = ringV[p * 64 + lane];
        const uint64_t vmw = (p & 64) ? vm1 : vm0;
        const bool elim = state == ST_ELIM;
        const bool valid = ((vmw >> (p & 63)) & 1ull) != 0;
        const uint64_t cx = c ^ row;
        const uint32_t vx = v ^ rv;
        const bool cont = elim && valid && cx != 0;
        const uint32_t j = (uint32_t)__builtin_ctzg(cx, 64);  // defined for cx == 0
        const uint32_t fin = !valid ? ST_PLACE : (vx == 0 ? ST_REDUNDANT : ST_CONFLICT);
        steps += (elim && valid) ? 1u : 0u;
        c = cont ? (cx >> j) : c;
        v = cont ? vx : v;
        i = cont ? i + j : i;
        state = (elim && !cont) ? fin : state;
      }

      // ---- outcome of finished equations (common path) ----
      if (state == ST_PLACE && i >= limit) {
        if (a.spillC && i < limit + 64u) {
          // final-layer segment: the row belongs past the segment end; keep it
          // in the ring (its half is free during the last bucket) and in the
          // segment's spill buffer
          const uint32_t p = i & (kRing - 1);
          ringC[p * 64 + lane] = c;
          ringV[p * 64 + lane] = (VT)v;
          const uint64_t bit = 1ull << (p & 63);
          if (p & 64) vm1 |= bit; else vm0 |= bit;
          a.spillC[rho * 64 + (i - limit)] = c;
          a.spillV[rho * 64 + (i - limit)] = v;
          state = ST_WANT;
        } else {
          // unreachable for kept keys of a BuRR layer; stop instead of
          // writing outside the range
          a.fail[js] = 2u;
          solve_diag(a.diag, 2, rho, js, x, xend, q, nq, state, open, written, rend, kf, curk,
                     i, fb);
          state = ST_DONE;
        }
      }
      if (state == ST_PLACE) {
        {
          const uint32_t p = i & (kRing - 1);
          ringC[p * 64 + lane] = c;
          ringV[p * 64 + lane] = (VT)v;
          const uint64_t bit = 1ull << (p & 63);
          const bool hi_half = (p & 64) != 0;
          vm1 |= hi_half ? bit : 0;
          pm1 |= hi_half ? bit : 0;
          vm0 |= hi_half ? 0 : bit;
          pm0 |= hi_half ? 0 : bit;
          a.rowsC[P0 + i] = c;
          a.rowsV[P0 + i] = v;
          state = ST_WANT;
        }
      }
      state = state == ST_REDUNDANT ? ST_WANT : state;
      // next record of the same bucket straight from the FIFO
      if (state == ST_WANT && x != rend && x < written) {
        const Rec rc = fifo[(x % kFifo) * 64 + lane];
        const uint32_t k = 3u - meta_rank(rc.meta);
        if (k > kf) {
          const bool newk = k != curk;
          pm0 = newk ? 0 : pm0;
          pm1 = newk ? 0 : pm1;
          chunk_start = newk ? x : chunk_start;
          curk = k;
          c = rc.c;
          v = meta_value(rc.meta);
          i = 64u * q + meta_offset(rc.meta);
          ++x;
          state = ST_ELIM;
        }
      }
      // ---- rare paths: conflicts, bucket ends, headers, forced bumps ----
      if (!__any(state == ST_CONFLICT ||
                 (state == ST_WANT && (x == rend ? (open || x < written) : x < written))))
        continue;
      if (state == ST_CONFLICT) {
        if (g.plain) {
          a.fail[js] = 1u;
          state = ST_DONE;
        } else {
          vm0 &= ~pm0;  // undo the chunk; the rest of the bucket is bumped
          vm1 &= ~pm1;
          code = curk;
          split_at = chunk_start;
          x = rend;
          state = ST_WANT;
        }
      }
      // ---- lanes take their next item ----
      // Up to three flat passes; each pass may end a bucket, open the next
      // one from its header and take a record. A lane whose next item has not
      // reached the FIFO waits for the next round.
#pragma unroll
      for (int pass = 0; pass < 3; ++pass) {
        if (pass > 0 && !__any(state == ST_WANT && (x == rend ? (open || x < written) : x < written)))
          break;
        if (state == ST_WANT && x == rend && open) {
          // end of the current bucket: publish code and bump count
          const uint64_t beta = fb + q;
          if (!g.plain) {
            a.code8[beta] = (uint8_t)code;
            a.bump[beta] = rend - (split_at == kNoSplit ? rend : split_at);
          }
          open = false;
          if (q + 1 == nq) {
            a.occ[beta] = (q & 1) ? vm1 : vm0;
            if (a.spill_occ) a.spill_occ[rho] = (q & 1) ? vm0 : vm1;
            state = ST_DONE;
          }
        }
        if (state == ST_WANT && x == rend && !open && x < written) {
          // header of the next bucket; bucket q-1 is final: publish its
          // occupancy and free its ring half
          const Rec hd = fifo[(x % kFifo) * 64 + lane];
          ++q;
          if (q >= 1) {
            const uint64_t beta = fb + q - 1;
            const bool odd = ((q - 1) & 1) != 0;
            a.occ[beta] = odd ? vm1 : vm0;
            vm1 = odd ? 0 : vm1;
            vm0 = odd ? vm0 : 0;
          }
          kf = head_kf(hd);
          code = kf;
          curk = 4;
          pm0 = 0;
          pm1 = 0;
          split_at = kNoSplit;
          rend = x + 1 + head_count(hd);
          ++x;
          open = true;
        }
        if (state == ST_WANT && x != rend && x < written) {
          // a record of the current bucket
          const Rec rc = fifo[(x % kFifo) * 64 + lane];
          const uint32_t k = 3u - meta_rank(rc.meta);
          if (k <= kf) {
            // forced part of a range's last bucket: the rest is bumped
            split_at = x;
            x = rend;
          } else {
            const bool newk = k != curk;
            pm0 = newk ? 0 : pm0;
            pm1 = newk ? 0 : pm1;
            chunk_start = newk ? x : chunk_start;
            curk = k;
            c = rc.c;
            v = meta_value(rc.meta);
            i = 64u * q + meta_offset(rc.meta);
            ++x;
            state = ST_ELIM;
          }
        }
      }
    }
    // ---- round end: commit this round's loads to the FIFO ----
#define BURR_STAGE_COMMIT(j) \
    if (j < ldn) fifo4[((ld0 + j) % kFifo) * 64 + lane] = st##j;
    BURR_STAGE_COMMIT(0) BURR_STAGE_COMMIT(1) BURR_STAGE_COMMIT(2) BURR_STAGE_COMMIT(3)
    BURR_STAGE_COMMIT(4) BURR_STAGE_COMMIT(5) BURR_STAGE_COMMIT(6) BURR_STAGE_COMMIT(7)
#undef BURR_STAGE_COMMIT
    if (ldn) written = ld0 + ldn;
    if (!__any(state != ST_DONE)) break;
  }
  if (a.steps) atomicAdd((unsigned long long*)a.steps, (unsigned long long)steps);
#ifdef BURR_SOLVE_DEBUG
  if (a.steps) {
    atomicAdd((unsigned long long*)a.steps + 1, (unsigned long long)dbg_active);
    atomicAdd((unsigned long long*)a.steps + 2, (unsigned long long)dbg_elim);
    atomicAdd((unsigned long long*)a.steps + 3, (unsigned long long)dbg_stall);
  }
#endif
}

template <typename VT, int K>
static hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.g.nranges + 63) / 64);
  const size_t lds = solve_lds_bytes<VT>();
  (void)hipFuncSetAttribute((const void*)k_solve<VT, K>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  k_solve<VT, K><<<blocks, 64, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t solve_layer(const SolveArgs& a, hipStream_t s) {
  if (a.g.r <= 8) return launch_solve<uint8_t, BURR_SOLVE_K>(a, s);
  if (a.g.r <= 16) return launch_solve<uint16_t, BURR_SOLVE_K>(a, s);
  return launch_solve<uint32_t, BURR_SOLVE_K>(a, s);
}

// ---------------------------------------------------------------------------
// Back-substitution: one lane per range, from the range end down
// ---------------------------------------------------------------------------
template <int RMAX>
__global__ __launch_bounds__(256) void k_backsub(const uint64_t* __restrict__ rowsC,
                                                 const uint32_t* __restrict__ rowsV,
                                                 const uint64_t* __restrict__ occ, LayerGeom g,
                                                 uint64_t* __restrict__ W,
                                                 const uint32_t* __restrict__ bnd) {
  const uint64_t rho = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (rho >= g.nranges) return;
  const uint32_t j = find_struct(g.range_base, g.J, rho);
  const uint64_t B = g.bucket_base[j + 1] - g.bucket_base[j];
  const uint64_t R = g.range_base[j + 1] - g.range_base[j];
  const uint64_t lr = rho - g.range_base[j];
  const uint64_t fb = g.bucket_base[j] + lr * B / R;
  const uint64_t lb = g.bucket_base[j] + (lr + 1) * B / R;
  const uint32_t r = g.rbits[j];
  const uint64_t wb = g.word_base[j], bb = g.bucket_base[j];  // block k at wb + (k-bb)*r
  uint64_t win[RMAX];  // bit j of win[col] = column col of Z[i+1+j]
#pragma unroll
  for (int col = 0; col < RMAX; ++col) win[col] = 0;
  if (bnd) {
    // rows near the end may reach the 63 slots after it: start from their values
    for (uint32_t t = 0; t < 63; ++t) {
      const uint32_t z = bnd[rho * 64 + t];
#pragma unroll
      for (int col = 0; col < RMAX; ++col) win[col] |= (uint64_t)((z >> col) & 1u) << t;
    }
  }
  for (uint64_t k = lb; k-- > fb;) {
    const uint64_t oc = occ[k];
    uint64_t out[RMAX];
#pragma unroll
    for (int col = 0; col < RMAX; ++col) out[col] = 0;
    for (int tt = 63; tt >= 0; --tt) {
      uint32_t z = 0;
      if ((oc >> tt) & 1ull) {
        const uint64_t slot = k * 64 + (uint64_t)tt;
        const uint64_t C = rowsC[slot] >> 1;
        const uint32_t V = rowsV[slot];
#pragma unroll
        for (int col = 0; col < RMAX; ++col)
          if ((uint32_t)col < r)
            z |= ((V >> col) ^ (uint32_t)__popcll(C & win[col])) & 1u ? (1u << col) : 0u;
      }
#pragma unroll
      for (int col = 0; col < RMAX; ++col) {
        if ((uint32_t)col < r) {
          const uint64_t b = (z >> col) & 1u;
          win[col] = (win[col] << 1) | b;
          out[col] |= b << tt;
        }
      }
    }
    for (uint32_t col = 0; col < r && col < (uint32_t)RMAX; ++col)
      W[wb + (k - bb) * r + col] = out[col];
  }
}

hipError_t back_substitute(const uint64_t* rowsC, const uint32_t* rowsV, const uint64_t* occ,
                           const LayerGeom& g, uint64_t* W, hipStream_t s, const uint32_t* bnd) {
  const unsigned blocks = (unsigned)((g.nranges + 255) / 256);
  if (g.r <= 8)
    k_backsub<8><<<blocks, 256, 0, s>>>(rowsC, rowsV, occ, g, W, bnd);
  else if (g.r <= 16)
    k_backsub<16><<<blocks, 256, 0, s>>>(rowsC, rowsV, occ, g, W, bnd);
  else
    k_backsub<32><<<blocks, 256, 0, s>>>(rowsC, rowsV, occ, g, W, bnd);
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

constexpr uint32_t kMergeWin = 384;  // slots of the right group staged in LDS

// One workgroup per segment p; it merges at level G when p starts a left
// group of G segments inside its structure and a right group follows.
__global__ __launch_bounds__(64) void k_merge(FinalArgs a, uint32_t G) {
  __shared__ uint64_t wc[kMergeWin];
  __shared__ uint32_t wv[kMergeWin];
  __shared__ uint64_t wocc[kMergeWin / 64];
  const LayerGeom g = a.g;
  const uint64_t p = blockIdx.x;
  const SegBounds sp = seg_bounds(p, g);
  const uint64_t lp = p - sp.first;
  if (lp % (2ull * G) != 0 || lp + G >= sp.count) return;
  const uint64_t R0 = p + G;
  const uint64_t lastL = R0 - 1;
  const uint64_t lastR = (lp + 2ull * G < sp.count ? p + 2ull * G : sp.first + sp.count) - 1;
  const uint64_t start = seg_bounds(R0, g).start;
  const uint64_t endR = seg_bounds(lastR, g).end;  // slot after the right group
  // window: slots [start, start + win); slots >= endR are the right group's
  // spill zone, which the window holds either completely or not at all
  const uint64_t span = endR + 64 - start;
  const uint64_t body = endR - start;
  const uint32_t win = (uint32_t)(span <= kMergeWin ? span : (body < kMergeWin ? body : kMergeWin));
  const uint32_t lane = threadIdx.x;
  for (uint32_t t = lane; t < win; t += 64) {
    const uint64_t slot = start + t;
    if (slot < endR) {
      wc[t] = a.rowsC[slot];
      wv[t] = a.rowsV[slot];
    } else {
      wc[t] = a.spillC[lastR * 64 + (slot - endR)];
      wv[t] = a.spillV[lastR * 64 + (slot - endR)];
    }
  }
  for (uint32_t b = lane; b < win / 64; b += 64) {
    const uint64_t slot = start + 64ull * b;
    wocc[b] = slot < endR ? a.occ[slot / 64] : a.spill_occ[lastR];
  }
  __syncthreads();
  if (lane == 0) {
    uint64_t pend = a.spill_occ[lastL];
    bool bad = false, internal = false;
    while (pend && !bad) {
      const uint32_t t0 = (uint32_t)__builtin_ctzll(pend);
      pend &= pend - 1;
      uint64_t c = a.spillC[lastL * 64 + t0];
      uint32_t v = a.spillV[lastL * 64 + t0];
      uint32_t i = t0;  // relative to start (the left group ends where the right one begins)
      while (true) {
        bool occupied;
        uint64_t row;
        uint32_t rv;
        if (i < win) {
          occupied = (wocc[i / 64] >> (i % 64)) & 1ull;
          row = wc[i];
          rv = wv[i];
        } else {
          // beyond the staged window: read the right group in global memory
          const uint64_t slot = start + i;
          if (slot < endR) {
            occupied = (a.occ[slot / 64] >> (slot % 64)) & 1ull;
            row = a.rowsC[slot];
            rv = a.rowsV[slot];
          } else {
            const uint64_t t = slot - endR;
            if (t >= 64) {  // unreachable: rows end at most 62 slots past the group
              bad = true;
              internal = true;
              break;
            }
            occupied = (a.spill_occ[lastR] >> t) & 1ull;
            row = a.spillC[lastR * 64 + t];
            rv = a.spillV[lastR * 64 + t];
          }
        }
        if (!occupied) {
          if (i < win) {
            wc[i] = c;
            wv[i] = v;
            wocc[i / 64] |= 1ull << (i % 64);
          } else {
            const uint64_t slot = start + i;
            if (slot < endR) {
              a.rowsC[slot] = c;
              a.rowsV[slot] = v;
              a.occ[slot / 64] |= 1ull << (slot % 64);
            } else {
              const uint64_t t = slot - endR;
              a.spillC[lastR * 64 + t] = c;
              a.spillV[lastR * 64 + t] = v;
              a.spill_occ[lastR] |= 1ull << t;
            }
          }
          break;
        }
        c ^= row;
        v ^= rv;
        if (c == 0) {
          if (v != 0) bad = true;  // inconsistent: this table size fails
          break;
        }
        const uint32_t j = (uint32_t)__builtin_ctzll(c);
        c >>= j;
        i += j;
      }
    }
    if (bad) a.fail[sp.j] = internal ? 2u : 1u;
    a.spill_occ[lastL] = 0;
  }
  __syncthreads();
  for (uint32_t t = lane; t < win; t += 64) {
    const uint64_t slot = start + t;
    if (slot < endR) {
      a.rowsC[slot] = wc[t];
      a.rowsV[slot] = wv[t];
    } else {
      a.spillC[lastR * 64 + (slot - endR)] = wc[t];
      a.spillV[lastR * 64 + (slot - endR)] = wv[t];
    }
  }
  for (uint32_t b = lane; b < win / 64; b += 64) {
    const uint64_t slot = start + 64ull * b;
    if (slot < endR)
      a.occ[slot / 64] = wocc[b];
    else
      a.spill_occ[lastR] = wocc[b];
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

// Per segment, back-substitute with the 63 values after the segment unknown:
// every slot's value is z0 (zero boundary) xor the boundary values selected
// by a 63-bit dependence word X. Only the first 63 slots' (z0, X) are kept.
__global__ __launch_bounds__(64) void k_final_partial(FinalArgs a) {
  __shared__ uint32_t zwin[64 * 64];
  __shared__ uint64_t xwin[64 * 64];
  const LayerGeom g = a.g;
  const uint32_t lane = threadIdx.x;
  const uint64_t p = (uint64_t)blockIdx.x * 64 + lane;
  if (p >= g.nranges) return;
  const SegBounds sb = seg_bounds(p, g);
  const uint64_t start = sb.start, end = sb.end;
  for (uint64_t i = end; i-- > start;) {
    uint32_t z = 0;
    uint64_t X = 0;
    if ((a.occ[i / 64] >> (i % 64)) & 1ull) {
      z = a.rowsV[i];
      uint64_t bits = a.rowsC[i] >> 1;
      while (bits) {
        const uint32_t k = (uint32_t)__builtin_ctzll(bits) + 1;
        bits &= bits - 1;
        const uint64_t slot = i + k;
        if (slot < end) {
          z ^= zwin[(slot % 64) * 64 + lane];
          X ^= xwin[(slot % 64) * 64 + lane];
        } else {
          X ^= 1ull << (slot - end);
        }
      }
    }
    zwin[(i % 64) * 64 + lane] = z;
    xwin[(i % 64) * 64 + lane] = X;
    if (i - start < 63) {
      a.z0first[p * 64 + (i - start)] = z;
      a.xfirst[p * 64 + (i - start)] = X;
    }
  }
}

// One workgroup per structure, from its last segment down: the boundary of
// segment p-1 is the true value of segment p's first 63 slots = z0 xor (X
// applied to segment p's boundary).
__global__ __launch_bounds__(64) void k_final_scan(FinalArgs a) {
  __shared__ uint32_t b[64];
  const uint32_t t = threadIdx.x;
  const LayerGeom g = a.g;
  const uint32_t j = blockIdx.x;
  const uint64_t first = g.range_base[j], last = g.range_base[j + 1];
  b[t] = 0;  // nothing lies past the structure's last segment
  __syncthreads();
  for (uint64_t p = last; p-- > first;) {
    a.bnd[p * 64 + t] = b[t];
    uint32_t z = 0;
    if (t < 63) {
      z = a.z0first[p * 64 + t];
      uint64_t X = a.xfirst[p * 64 + t];
      while (X) {
        const uint32_t k = (uint32_t)__builtin_ctzll(X);
        X &= X - 1;
        z ^= b[k];
      }
    }
    __syncthreads();
    b[t] = z;
    __syncthreads();
  }
}

hipError_t final_boundaries(const FinalArgs& a, hipStream_t s) {
  const uint64_t P = a.g.nranges;
  k_final_partial<<<(unsigned)((P + 63) / 64), 64, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_final_scan<<<a.g.J, 64, 0, s>>>(a);
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
  uint64_t word = 0;
  for (uint64_t t = 0; t < 32; ++t) {
    const uint64_t b = wl * 32 + t;
    if (b < B) word |= (uint64_t)(code8[g.bucket_base[j] + b] & 3u) << (2 * t);
  }
  words[w] = word;
}

hipError_t pack_codes(const uint8_t* code8, const LayerGeom& g, uint64_t ncode_words,
                      uint64_t* words, hipStream_t s) {
  if (ncode_words == 0) return hipSuccess;
  k_pack_codes<<<(unsigned)((ncode_words + 255) / 256), 256, 0, s>>>(code8, g, ncode_words,
                                                                     words);
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

__global__ void k_gather(const uint64_t* __restrict__ sorted_keys, const Rec* __restrict__ rec,
                         const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ off,
                         uint64_t B, uint64_t* __restrict__ nk, uint32_t* __restrict__ nv) {
  const uint64_t beta = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (beta >= B) return;
  const uint32_t o = off[beta];
  const uint32_t cnt = off[beta + 1] - o;
  const uint32_t src = bstart[beta + 1] - cnt;
  for (uint32_t j = 0; j < cnt; ++j) {
    nk[o + j] = sorted_keys[src + j];
    nv[o + j] = meta_value(rec[src + j + beta + 1].meta);
  }
}

hipError_t gather_bumped(const uint64_t* sorted_keys, const Rec* rec, const uint32_t* bstart,
                         const uint32_t* off, uint64_t B, uint64_t* next_keys,
                         uint32_t* next_vals, hipStream_t s) {
  if (B == 0) return hipSuccess;
  k_gather<<<(unsigned)((B + 255) / 256), 256, 0, s>>>(sorted_keys, rec, bstart, off, B,
                                                       next_keys, next_vals);
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
// Query: one lane per key
// ---------------------------------------------------------------------------
template <typename OT>
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
    if (!L.plain) {
      const uint64_t beta = s >> 6;
      const uint32_t o = (uint32_t)s & 63u;
      const uint32_t code = (uint32_t)(L.codes[beta >> 5] >> (2 * (beta & 31))) & 3u;
      const uint32_t th = code == 0 ? 0u : (code == 1 ? L.t_lo : (code == 2 ? L.t_hi : 64u));
      if (o < th) continue;
    }
    const uint64_t c = mix64(key ^ L.salt_c) | 1ull;
    const uint32_t sh = (uint32_t)s & 63u;
    const uint64_t* w = L.W + (s >> 6) * r;
    for (uint32_t col = 0; col < r; ++col) {
      uint64_t win = w[col] >> sh;
      if (sh) win |= w[r + col] << (64 - sh);
      res |= ((uint32_t)__popcll(win & c) & 1u) << col;
    }
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
  if (out_bytes == 1)
    k_query<uint8_t><<<blocks, 256, 0, s>>>(plan, keys, n, (uint8_t*)out, contains, fp_salt);
  else if (out_bytes == 2)
    k_query<uint16_t><<<blocks, 256, 0, s>>>(plan, keys, n, (uint16_t*)out, contains, fp_salt);
  else
    k_query<uint32_t><<<blocks, 256, 0, s>>>(plan, keys, n, (uint32_t*)out, contains, fp_salt);
  return hipGetLastError();
}

}  // namespace burr
