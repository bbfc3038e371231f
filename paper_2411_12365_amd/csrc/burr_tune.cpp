// burr_tune.cpp - autotuner of the range split of batched builds.
//
// The number of ranges of a layer trades sequential depth against boundary
// bumps (Sec. 3 "Minimum Buckets per Thread"): short ranges give more
// independent wavefronts and shorter insertion chains, but every range end
// bumps about one bucket of keys into the next layer and adds table space.
// Which minimum of buckets per range is fastest depends on the structure
// size and on how many structures share the device, so it is measured: per
// size class, synthetic batches are built once per candidate and timed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/burr.h"
#include "burr_internal.h"
#include "burr_kernels.h"

namespace {

struct DeviceInputs {
  uint64_t* keys = nullptr;
  void* vals = nullptr;
  ~DeviceInputs() {
    if (keys) (void)hipFree(keys);
    if (vals) (void)hipFree(vals);
  }
};

uint32_t value_bytes(uint32_t r) { return r <= 8 ? 1 : (r <= 16 ? 2 : 4); }

}  // namespace

namespace {

// Best-of-reps seconds of one batched build (after a warm-up) and its table
// bits, or an error code in *rc.
double time_batch(const uint64_t* keys, const void* vals, const std::vector<uint64_t>& off,
                  const std::vector<uint32_t>& rs, const burr_params* p,
                  const std::vector<burr_tune_entry>& table, uint32_t reps, double* bits,
                  int* rc) {
  double best = 0;
  for (uint32_t t = 0; t <= reps; ++t) {  // t = 0: warm-up
    const auto t0 = std::chrono::steady_clock::now();
    burr_batch* b = burr_build_batch_tuned(keys, vals, off.data(), rs.data(),
                                           (uint32_t)rs.size(), p, table.data(),
                                           (uint32_t)table.size());
    const auto t1 = std::chrono::steady_clock::now();
    if (!b) {
      *rc = burr_last_error();
      return 0;
    }
    const double sec = std::chrono::duration<double>(t1 - t0).count();
    if (t == 1 || (t > 1 && sec < best)) best = sec;
    if (t == reps && bits) *bits = (double)burr_batch_table_bits(b);
    burr_batch_free(b);
  }
  *rc = BURR_OK;
  return best;
}

// Tuning on a mix of structure sizes: coordinate descent over the classes,
// starting from p->minbpt everywhere; a class takes another candidate if the
// whole mixed batch builds more than 3 % faster with it, or if its tables are
// smaller by at least the fraction of time it costs, while it stays within
// 3 % of the fastest time seen and of the untuned batch's time (space counts
// where time is a draw, as in the paper's Fig. 4 trade-off, but a slower
// candidate has to save as large a share of space as it costs in time; the 3 %
// margin is above the timing noise of the repeats).
int tune_mix(const burr_params* p, uint32_t r, const uint64_t* sizes, uint64_t nsizes,
             const uint64_t* n_max, uint32_t nclasses, const uint32_t* candidates,
             uint32_t ncandidates, uint32_t reps, burr_tune_entry* out) {
  std::vector<uint64_t> off(nsizes + 1, 0);
  for (uint64_t i = 0; i < nsizes; ++i) off[i + 1] = off[i] + sizes[i];
  const uint64_t total = off.back();
  if (total == 0 || nsizes > 0xffffffffull) return burr_set_error(BURR_E_INVALID);
  std::vector<uint32_t> rs(nsizes, r);
  const uint32_t vb = value_bytes(r);
  DeviceInputs in;
  if (hipMalloc((void**)&in.keys, total * 8) != hipSuccess ||
      (!p->filter_mode && hipMalloc(&in.vals, total * vb) != hipSuccess))
    return burr_set_error(BURR_E_NOMEM);
  hipStream_t s = (hipStream_t)p->stream;
  const uint64_t vmask = r >= 32 ? 0xffffffffull : ((1ull << r) - 1);
  if (burr::fill_stream(in.keys, in.vals, vb, total, 0x5eed0001ull, 0x5eed0002ull, vmask, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return burr_set_error(BURR_E_DEVICE);
  std::vector<burr_tune_entry> table(nclasses);
  for (uint32_t c = 0; c < nclasses; ++c) {
    table[c] = burr_tune_entry{};
    table[c].n_max = n_max[c];
    table[c].minbpt = p->minbpt ? p->minbpt : 1;
  }
  int rc = BURR_OK;
  double bits = 0;
  double cur = time_batch(in.keys, in.vals, off, rs, p, table, reps, &bits, &rc);
  if (rc != BURR_OK) return burr_set_error(rc);
  const double untuned = cur;
  double fastest = cur;  // fastest mixed batch seen
  for (uint32_t c = 0; c < nclasses; ++c) {
    const uint32_t keep = table[c].minbpt;
    uint32_t best = keep;
    double best_t = cur, best_bits = bits;
    for (uint32_t k = 0; k < ncandidates; ++k) {
      if (candidates[k] == keep) continue;
      table[c].minbpt = candidates[k];
      double b2 = 0;
      const double t = time_batch(in.keys, in.vals, off, rs, p, table, reps, &b2, &rc);
      if (rc != BURR_OK) return burr_set_error(rc);
      const bool faster = t < best_t * 0.97;
      const double cost = (t - best_t) / best_t;            // time added (< 0: saved)
      const double saved = (best_bits - b2) / best_bits;    // space saved
      const bool smaller = saved > 0 && saved >= cost && t <= fastest * 1.03 &&
                           t <= untuned * 1.03;
      if (faster || smaller) {
        best = candidates[k];
        best_t = t;
        best_bits = b2;
      }
      fastest = std::min(fastest, t);
    }
    table[c].minbpt = best;
    cur = best_t;
    bits = best_bits;
  }
  for (uint32_t c = 0; c < nclasses; ++c) {
    out[c] = table[c];
    out[c].ns_per_key = cur * 1e9 / (double)total;
    out[c].bits_per_key = bits / (double)total;
  }
  burr_set_error(BURR_OK);
  return BURR_OK;
}

}  // namespace

extern "C" int burr_autotune(const burr_params* p, uint32_t r, const uint64_t* sizes,
                             uint64_t nsizes, const uint64_t* n_max, uint32_t nclasses,
                             const uint32_t* candidates, uint32_t ncandidates,
                             uint64_t keys_per_trial, uint32_t reps, burr_tune_entry* out) {
  if (!p || !n_max || !candidates || !out || nclasses == 0 || ncandidates == 0 || r < 1 ||
      r > 32 || reps == 0 || (!sizes && keys_per_trial == 0) || (sizes && nsizes == 0))
    return burr_set_error(BURR_E_INVALID);
  for (uint32_t c = 0; c < nclasses; ++c)
    if (n_max[c] == 0 || (c > 0 && n_max[c] <= n_max[c - 1]))
      return burr_set_error(BURR_E_INVALID);
  for (uint32_t k = 0; k < ncandidates; ++k)
    if (candidates[k] == 0) return burr_set_error(BURR_E_INVALID);
  if (sizes) return tune_mix(p, r, sizes, nsizes, n_max, nclasses, candidates, ncandidates, reps,
                             out);

  // inputs for the largest trial batch, made once
  uint64_t cap = 0;
  for (uint32_t c = 0; c < nclasses; ++c) cap = std::max(cap, std::max(keys_per_trial, n_max[c]));
  const uint32_t vb = value_bytes(r);
  DeviceInputs in;
  if (hipMalloc((void**)&in.keys, cap * 8) != hipSuccess ||
      (!p->filter_mode && hipMalloc(&in.vals, cap * vb) != hipSuccess))
    return burr_set_error(BURR_E_NOMEM);
  hipStream_t s = (hipStream_t)p->stream;
  const uint64_t vmask = r >= 32 ? 0xffffffffull : ((1ull << r) - 1);
  if (burr::fill_stream(in.keys, in.vals, vb, cap, 0x5eed0001ull, 0x5eed0002ull, vmask, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return burr_set_error(BURR_E_DEVICE);

  for (uint32_t c = 0; c < nclasses; ++c) {
    // representative size: geometric middle of the class
    const double lo = c ? (double)n_max[c - 1] : std::max(1.0, n_max[0] / 4.0);
    const uint64_t size = std::max<uint64_t>(1, (uint64_t)std::llround(std::sqrt(lo * n_max[c])));
    const uint64_t count = std::max<uint64_t>(1, std::min<uint64_t>(keys_per_trial / size,
                                                                    cap / size));
    if (count > 0xffffffffull) return burr_set_error(BURR_E_INVALID);
    std::vector<uint64_t> off(count + 1);
    for (uint64_t i = 0; i <= count; ++i) off[i] = i * size;
    std::vector<uint32_t> rs(count, r);
    const double keys = (double)off.back();

    std::vector<double> ns(ncandidates), bits(ncandidates);
    for (uint32_t k = 0; k < ncandidates; ++k) {
      burr_tune_entry one{};
      one.n_max = ~0ull;
      one.minbpt = candidates[k];
      double best = 0;
      for (uint32_t t = 0; t <= reps; ++t) {  // t = 0: warm-up
        const auto t0 = std::chrono::steady_clock::now();
        burr_batch* b = burr_build_batch_tuned(in.keys, in.vals, off.data(), rs.data(),
                                               (uint32_t)count, p, &one, 1);
        const auto t1 = std::chrono::steady_clock::now();
        if (!b) return burr_last_error();
        const double sec = std::chrono::duration<double>(t1 - t0).count();
        if (t == 1 || (t > 1 && sec < best)) best = sec;
        if (t == reps) bits[k] = (double)burr_batch_table_bits(b) / keys;
        burr_batch_free(b);
      }
      ns[k] = best * 1e9 / keys;
    }
    // the fastest candidate; among those within 3 % of it (timing noise),
    // the parameter block's own value if it is one, else the smallest tables
    uint32_t pick = 0;
    for (uint32_t k = 1; k < ncandidates; ++k)
      if (ns[k] < ns[pick]) pick = k;
    const double fastest = ns[pick];
    int def = -1;
    for (uint32_t k = 0; k < ncandidates; ++k)
      if (candidates[k] == p->minbpt && ns[k] <= fastest * 1.03) def = (int)k;
    if (def >= 0) {
      pick = (uint32_t)def;
    } else {
      for (uint32_t k = 0; k < ncandidates; ++k)
        if (ns[k] <= fastest * 1.03 && bits[k] < bits[pick]) pick = k;
    }
    out[c].n_max = n_max[c];
    out[c].minbpt = candidates[pick];
    out[c].reserved = 0;
    out[c].ns_per_key = ns[pick];
    out[c].bits_per_key = bits[pick];
  }
  burr_set_error(BURR_OK);
  return BURR_OK;
}
