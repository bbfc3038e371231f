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

extern "C" int burr_autotune(const burr_params* p, uint32_t r, const uint64_t* n_max,
                             uint32_t nclasses, const uint32_t* candidates, uint32_t ncandidates,
                             uint64_t keys_per_trial, uint32_t reps, burr_tune_entry* out) {
  if (!p || !n_max || !candidates || !out || nclasses == 0 || ncandidates == 0 || r < 1 ||
      r > 32 || keys_per_trial == 0 || reps == 0)
    return burr_set_error(BURR_E_INVALID);
  for (uint32_t c = 0; c < nclasses; ++c)
    if (n_max[c] == 0 || (c > 0 && n_max[c] <= n_max[c - 1]))
      return burr_set_error(BURR_E_INVALID);
  for (uint32_t k = 0; k < ncandidates; ++k)
    if (candidates[k] == 0) return burr_set_error(BURR_E_INVALID);

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
    uint32_t pick = 0;
    for (uint32_t k = 1; k < ncandidates; ++k)
      if (ns[k] < ns[pick]) pick = k;
    const double fastest = ns[pick];
    for (uint32_t k = 0; k < ncandidates; ++k)
      if (ns[k] <= fastest * 1.03 && bits[k] < bits[pick]) pick = k;
    out[c].n_max = n_max[c];
    out[c].minbpt = candidates[pick];
    out[c].reserved = 0;
    out[c].ns_per_key = ns[pick];
    out[c].bits_per_key = bits[pick];
  }
  burr_set_error(BURR_OK);
  return BURR_OK;
}
