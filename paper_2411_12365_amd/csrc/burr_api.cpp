// burr_api.cpp - C ABI of the BuRR library (include/burr.h): parameter
// checks, layer planning, workspace, the per-layer launch sequence, export
// and import.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/burr.h"
#include "burr_kernels.h"

using namespace burr;

namespace {

thread_local int g_last_error = BURR_OK;

int set_error(int code) {
  g_last_error = code;
  return code;
}

constexpr uint64_t kExportMagic = 0x3170786552527542ull;  // "BuRRexp1"
constexpr uint32_t kExportVersion = 1;
constexpr uint32_t kMaxLayers = 32;

uint32_t value_bytes(uint32_t r) { return r <= 8 ? 1 : (r <= 16 ? 2 : 4); }

// Device memory through the caller's allocator, or HIP's stream-ordered pool.
struct Allocator {
  burr_alloc_fn fn = nullptr;
  burr_free_fn ffn = nullptr;
  void* ctx = nullptr;
  hipStream_t s = nullptr;

  void* get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (fn) return fn(bytes, (void*)s, ctx);
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    if (ffn)
      ffn(p, (void*)s, ctx);
    else
      (void)hipFreeAsync(p, s);
  }
};

void keep_pool_memory(int dev) {
  static bool done[64] = {false};
  if (dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

struct DevLayer {
  uint64_t n = 0, m = 0, B = 0, R = 0, bumped = 0;
  double ms_sort = 0, ms_solve = 0, ms_backsub = 0, ms_gather = 0;
  uint64_t ncode = 0, nW = 0;  // words
  uint64_t* codes = nullptr;
  uint64_t* W = nullptr;
  uint64_t* keys = nullptr;    // kept input keys (debug flag)
  uint64_t steps = 0;
};

}  // namespace

struct burr_handle {
  burr_params p{};
  uint32_t r = 0;
  uint64_t n = 0;
  uint32_t built = 0;
  DevLayer layer[kMaxLayers];
  DevLayer fin;
  uint64_t fin_attempt = 0;
  hipStream_t stream = nullptr;
  Allocator al;
  burr_stats st{};
};

namespace {

bool params_ok(const burr_params* p, uint32_t r, const void* values, uint64_t n) {
  if (!p || p->abi_version != BURR_ABI_VERSION) return false;
  if (r < 1 || r > 32) return false;
  if (p->bucket != kBucket) return false;  // the kernels handle b = w = 64
  if (!(p->t_lo > 0 && p->t_lo < p->t_hi && p->t_hi < p->bucket)) return false;
  if (!p->load_num || !p->load_den || !p->final_num || !p->final_den) return false;
  if (p->final_num < p->final_den) return false;
  if (p->layers > kMaxLayers - 1) return false;
  if (!p->ranges || !p->final_attempts) return false;
  if (!p->filter_mode && !values && n > 0) return false;
  if (n >= 0xfff00000ull) return false;  // record indices are 32-bit
  return true;
}

uint64_t ceil_div(unsigned __int128 a, unsigned __int128 b) { return (uint64_t)((a + b - 1) / b); }

// BuRR layer geometry: m = b * max(1, ceil(load * n / b)) slots, B = m/b
// buckets, R = min(ranges, B / max(minbpt, 2)) ranges (at least 1).
LayerGeom plan_layer(const burr_params& p, uint64_t n, uint32_t layer, uint32_t r) {
  LayerGeom g{};
  uint64_t nb = ceil_div((unsigned __int128)n * p.load_num, (unsigned __int128)p.load_den * kBucket);
  if (nb < 1) nb = 1;
  g.m = nb * kBucket;
  g.nbuckets = nb;
  uint64_t per = p.minbpt < 2 ? 2 : p.minbpt;
  uint64_t R = nb / per;
  if (R > p.ranges) R = p.ranges;
  if (R < 1) R = 1;
  g.nranges = R;
  g.salt_s = mix64(p.seed ^ (2ull * layer + 1ull));
  g.salt_c = mix64(p.seed ^ (2ull * layer + 2ull));
  g.span = g.m - kWidth + 1;
  g.t_lo = p.t_lo;
  g.t_hi = p.t_hi;
  g.plain = 0;
  g.r = r;
  return g;
}

// Final plain ribbon: m = 64 * max(1, ceil(n * (final + a/10) / 64)).
LayerGeom plan_final(const burr_params& p, uint64_t n, uint32_t attempt, uint32_t r) {
  LayerGeom g{};
  unsigned __int128 num =
      (unsigned __int128)n * ((uint64_t)p.final_num * 10u + (uint64_t)attempt * p.final_den);
  uint64_t nb = ceil_div(num, (unsigned __int128)p.final_den * 10u * kWidth);
  if (nb < 1) nb = 1;
  g.m = nb * kWidth;
  g.nbuckets = nb;
  g.nranges = 1;
  g.salt_s = mix64(p.seed ^ (2ull * p.layers + 1ull));
  g.salt_c = mix64(p.seed ^ (2ull * p.layers + 2ull));
  g.span = g.m - kWidth + 1;
  g.t_lo = p.t_lo;
  g.t_hi = p.t_hi;
  g.plain = 1;
  g.r = r;
  return g;
}

// Reusable device workspace of one build; grows on demand.
struct Workspace {
  Allocator* al;
  std::vector<void*> owned;
  uint64_t cap_keys = 0, cap_m = 0, cap_B = 0, cap_counts = 0;
  uint64_t *keysA = nullptr, *keysT = nullptr, *keysS = nullptr;
  uint32_t *valsA = nullptr, *valsT = nullptr;
  Rec* rec = nullptr;
  uint64_t* rowsC = nullptr;
  uint32_t* rowsV = nullptr;
  uint64_t* occ = nullptr;
  uint8_t* code8 = nullptr;
  uint32_t *bump = nullptr, *bstart = nullptr, *counts = nullptr, *scan_tmp = nullptr;
  uint32_t* fail = nullptr;
  uint64_t* steps = nullptr;

  explicit Workspace(Allocator* a) : al(a) {}
  ~Workspace() {
    for (void* p : owned) al->put(p);
  }
  template <typename T>
  bool alloc(T*& ptr, uint64_t count) {
    ptr = (T*)al->get(count * sizeof(T));
    if (!ptr) return false;
    owned.push_back(ptr);
    return true;
  }
  bool reserve_keys(uint64_t n) {
    if (n <= cap_keys && keysA) return true;
    cap_keys = std::max<uint64_t>(n, 1);
    return alloc(keysA, cap_keys) && alloc(keysT, cap_keys) && alloc(keysS, cap_keys) &&
           alloc(valsA, cap_keys) && alloc(valsT, cap_keys);
  }
  uint64_t cap_items = 0;
  bool reserve_items(uint64_t count) {  // item stream: one record per key + one header per bucket
    if (count <= cap_items && rec) return true;
    cap_items = count;
    return alloc(rec, count);
  }
  bool reserve_slots(uint64_t m) {
    if (m <= cap_m && rowsC) return true;
    cap_m = m;
    return alloc(rowsC, m) && alloc(rowsV, m) && alloc(occ, m / 64 + 1);
  }
  bool reserve_buckets(uint64_t B) {
    if (B <= cap_B && bump) return reserve_scan(B + 1);
    cap_B = B;
    return alloc(code8, B + 1) && alloc(bump, B + 1) && alloc(bstart, B + 1) &&
           reserve_scan(B + 1);
  }
  bool reserve_counts(uint64_t c) {
    if (c <= cap_counts && counts) return reserve_scan(c + 1);
    cap_counts = c;
    return alloc(counts, c + 1) && reserve_scan(c + 1);
  }
  uint64_t cap_scan = 0;
  bool reserve_scan(uint64_t n) {
    const uint64_t need = scan_tmp_words(n) + 64;
    if (need <= cap_scan && scan_tmp) return true;
    cap_scan = need;
    return alloc(scan_tmp, need);
  }
  bool misc() { return alloc(fail, 64) && alloc(steps, 8); }
  // final layer segments
  uint64_t cap_seg = 0;
  uint64_t *spillC = nullptr, *spill_occ = nullptr, *xfirst = nullptr;
  uint32_t *spillV = nullptr, *z0first = nullptr, *bnd = nullptr;
  bool reserve_segments(uint64_t P) {
    if (P <= cap_seg && spillC) return true;
    cap_seg = P;
    return alloc(spillC, P * 64) && alloc(spillV, P * 64) && alloc(spill_occ, P) &&
           alloc(xfirst, P * 64) && alloc(z0first, P * 64) && alloc(bnd, P * 64);
  }
};

#define HIP_TRY(expr)                                     \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) {                               \
      fprintf(stderr, "burr: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(_e), \
              __FILE__, __LINE__);                        \
      return set_error(BURR_E_DEVICE);                    \
    }                                                     \
  } while (0)

// final layer: buckets per independently solved segment
constexpr uint64_t kFinalSegBuckets = 4;

uint32_t sort_groups(uint64_t n, uint32_t nbins) {
  // level-1 workgroups: enough to fill the chip, few enough that the
  // bins x groups count matrix stays small
  uint64_t g = (n + 4095) / 4096;
  uint64_t cap = nbins > 4096 ? 1024 : 2048;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (uint32_t)g;
}

// Sort one layer's n keys (device) by (bucket, chunk) into ws.keysS / ws.rec / ws.bstart.
int run_sort(Workspace& ws, const uint64_t* keys, const void* vals, uint32_t vbytes,
             bool first_layer, bool filter, uint64_t fp_salt, uint64_t n, const LayerGeom& g,
             hipStream_t s) {
  SortArgs a{};
  a.keys = keys;
  a.vals = vals;
  a.vbytes = vbytes;
  a.mask_values = first_layer ? 1u : 0u;
  a.filter = filter ? 1u : 0u;
  a.fp_salt = fp_salt;
  a.n = n;
  a.g = g;
  a.nbins = (uint32_t)((g.nbuckets + kBucketsPerBin - 1) / kBucketsPerBin);
  if (a.nbins > kMaxBins) return set_error(BURR_E_INVALID);
  a.groups = sort_groups(n, a.nbins);
  if (!ws.reserve_counts((uint64_t)a.nbins * a.groups)) return set_error(BURR_E_NOMEM);
  a.counts = ws.counts;
  a.scan_tmp = ws.scan_tmp;
  a.tmp_keys = ws.keysT;
  a.tmp_vals = ws.valsT;
  a.out_keys = ws.keysS;
  if (!ws.reserve_items(n + g.nbuckets)) return set_error(BURR_E_NOMEM);
  a.out_rec = ws.rec;
  a.bstart = ws.bstart;
  HIP_TRY(sort_layer(a, s));
  return BURR_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0;
  return ms;
}

int build_impl(burr_handle* h, const uint64_t* keys, const void* values) {
  const burr_params& p = h->p;
  const uint32_t r = h->r;
  hipStream_t s = h->stream;
  const uint64_t fp_salt = mix64(~p.seed);
  Workspace ws(&h->al);
  if (!ws.misc()) return set_error(BURR_E_NOMEM);
  hipEvent_t ev[6];
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 6; i++) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};
  HIP_TRY(hipEventRecord(ev[0], s));

  uint64_t cur_n = h->n;
  const uint64_t* cur_keys = keys;
  const void* cur_vals = values;
  uint32_t cur_vbytes = value_bytes(r);
  bool first = true;
  double ms_sort = 0, ms_solve = 0;
  if (!ws.reserve_keys(cur_n)) return set_error(BURR_E_NOMEM);

  uint32_t li = 0;
  while (li < p.layers && cur_n > 0) {
    DevLayer& L = h->layer[li];
    const LayerGeom g = plan_layer(p, cur_n, li, r);
    L.n = cur_n;
    L.m = g.m;
    L.B = g.nbuckets;
    L.R = g.nranges;
    if (p.flags & BURR_FLAG_KEEP_LAYER_KEYS) {
      L.keys = (uint64_t*)h->al.get(cur_n * 8);
      if (!L.keys) return set_error(BURR_E_NOMEM);
      HIP_TRY(hipMemcpyAsync(L.keys, cur_keys, cur_n * 8, hipMemcpyDeviceToDevice, s));
    }
    if (!ws.reserve_slots(g.m) || !ws.reserve_buckets(g.nbuckets)) return set_error(BURR_E_NOMEM);
    HIP_TRY(hipEventRecord(ev[1], s));
    int rc = run_sort(ws, cur_keys, cur_vals, cur_vbytes, first, p.filter_mode != 0, fp_salt,
                      cur_n, g, s);
    if (rc != BURR_OK) return rc;

    SolveArgs sa{};
    sa.rec = ws.rec;
    sa.bstart = ws.bstart;
    sa.g = g;
    sa.rowsC = ws.rowsC;
    sa.rowsV = ws.rowsV;
    sa.occ = ws.occ;
    sa.code8 = ws.code8;
    sa.bump = ws.bump;
    sa.fail = ws.fail;
    sa.steps = ws.steps;
    sa.nrec = (uint32_t)(cur_n + g.nbuckets);
    HIP_TRY(hipMemsetAsync(ws.steps, 0, 64, s));
    HIP_TRY(hipMemsetAsync(ws.fail, 0, 4, s));
    HIP_TRY(hipEventRecord(ev[2], s));
    HIP_TRY(solve_layer(sa, s));
    HIP_TRY(hipEventRecord(ev[4], s));

    L.ncode = (g.nbuckets + 31) / 32;
    L.nW = (g.m / 64) * r;
    L.codes = (uint64_t*)h->al.get(L.ncode * 8);
    L.W = (uint64_t*)h->al.get(L.nW * 8);
    if (!L.codes || !L.W) return set_error(BURR_E_NOMEM);
    HIP_TRY(back_substitute(ws.rowsC, ws.rowsV, ws.occ, g, L.W, s));
    HIP_TRY(pack_codes(ws.code8, g.nbuckets, L.codes, s));
    HIP_TRY(hipEventRecord(ev[3], s));

    // bumped keys: exclusive scan of per-bucket counts, then gather
    HIP_TRY(hipMemsetAsync(ws.bump + g.nbuckets, 0, 4, s));
    HIP_TRY(scan_exclusive(ws.bump, g.nbuckets + 1, ws.scan_tmp, s));
    uint32_t nnext = 0, failed = 0;
    uint64_t steps = 0;
    HIP_TRY(hipMemcpyAsync(&failed, ws.fail, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&nnext, ws.bump + g.nbuckets, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&steps, ws.steps, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(gather_bumped(ws.keysS, ws.rec, ws.bstart, ws.bump, g.nbuckets, ws.keysA, ws.valsA,
                          s));
    HIP_TRY(hipEventRecord(ev[5], s));
    HIP_TRY(hipStreamSynchronize(s));
#ifdef BURR_SOLVE_DEBUG
    {
      uint64_t d[4];
      if (hipMemcpy(d, ws.steps, 32, hipMemcpyDeviceToHost) == hipSuccess)
        fprintf(stderr, "solve-debug layer %u: steps %llu lane-iters %llu elim-iters %llu want-iters %llu\n",
                li, (unsigned long long)d[0], (unsigned long long)d[1], (unsigned long long)d[2],
                (unsigned long long)d[3]);
    }
#endif
    if (failed) {
      fprintf(stderr, "burr: internal error %u in the insertion kernel, layer %u\n", failed, li);
      return set_error(BURR_E_DEVICE);
    }
    L.ms_sort = elapsed_ms(ev[1], ev[2]);
    L.ms_solve = elapsed_ms(ev[2], ev[4]);
    L.ms_backsub = elapsed_ms(ev[4], ev[3]);
    L.ms_gather = elapsed_ms(ev[3], ev[5]);
    ms_sort += L.ms_sort;
    ms_solve += L.ms_solve + L.ms_backsub;
    L.bumped = nnext;
    L.steps = steps;
    cur_n = nnext;
    cur_keys = ws.keysA;
    cur_vals = ws.valsA;
    cur_vbytes = 4;
    first = false;
    ++li;
  }
  h->built = li;

  // final plain ribbon layer
  DevLayer& F = h->fin;
  F.n = cur_n;
  HIP_TRY(hipEventRecord(ev[1], s));
  if (p.flags & BURR_FLAG_KEEP_LAYER_KEYS) {
    F.keys = (uint64_t*)h->al.get(cur_n * 8 + 8);
    if (!F.keys) return set_error(BURR_E_NOMEM);
    if (cur_n) HIP_TRY(hipMemcpyAsync(F.keys, cur_keys, cur_n * 8, hipMemcpyDeviceToDevice, s));
  }
  if (cur_n == 0) {
    F.m = 0;
    F.nW = 0;
    h->fin_attempt = 0;
  } else {
    bool solved = false;
    for (uint32_t a = 0; a < p.final_attempts && !solved; ++a) {
      const LayerGeom g = plan_final(p, cur_n, a, r);
      if (!ws.reserve_slots(g.m) || !ws.reserve_buckets(g.nbuckets)) return set_error(BURR_E_NOMEM);
      int rc = run_sort(ws, cur_keys, cur_vals, cur_vbytes, first, p.filter_mode != 0, fp_salt,
                        cur_n, g, s);
      if (rc != BURR_OK) return rc;
      // The table is cut into segments of kFinalSegBuckets buckets solved in
      // parallel; rows crossing a segment end are merged afterwards.
      LayerGeom gs = g;
      gs.nranges = std::max<uint64_t>(1, g.nbuckets / kFinalSegBuckets);
      if (!ws.reserve_segments(gs.nranges)) return set_error(BURR_E_NOMEM);
      HIP_TRY(hipMemsetAsync(ws.fail, 0, 4, s));
      HIP_TRY(hipMemsetAsync(ws.steps, 0, 64, s));
      HIP_TRY(hipMemsetAsync(ws.spill_occ, 0, gs.nranges * 8, s));
      SolveArgs sa{};
      sa.rec = ws.rec;
      sa.bstart = ws.bstart;
      sa.g = gs;
      sa.rowsC = ws.rowsC;
      sa.rowsV = ws.rowsV;
      sa.occ = ws.occ;
      sa.fail = ws.fail;
      sa.steps = ws.steps;
      sa.nrec = (uint32_t)(cur_n + g.nbuckets);
      sa.spillC = ws.spillC;
      sa.spillV = ws.spillV;
      sa.spill_occ = ws.spill_occ;
      HIP_TRY(solve_layer(sa, s));
      FinalArgs fa{};
      fa.g = gs;
      fa.rowsC = ws.rowsC;
      fa.rowsV = ws.rowsV;
      fa.occ = ws.occ;
      fa.spillC = ws.spillC;
      fa.spillV = ws.spillV;
      fa.spill_occ = ws.spill_occ;
      fa.fail = ws.fail;
      fa.z0first = ws.z0first;
      fa.xfirst = ws.xfirst;
      fa.bnd = ws.bnd;
      HIP_TRY(final_merge(fa, s));
      uint32_t failed = 0;
      uint64_t steps = 0;
      HIP_TRY(hipMemcpyAsync(&failed, ws.fail, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(&steps, ws.steps, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      F.steps += steps;
      if (failed >= 2) {
        fprintf(stderr, "burr: internal error %u in the final layer\n", failed);
        return set_error(BURR_E_DEVICE);
      }
      if (failed) continue;
      F.m = g.m;
      F.nW = (g.m / 64) * r;
      F.W = (uint64_t*)h->al.get(F.nW * 8);
      if (!F.W) return set_error(BURR_E_NOMEM);
      HIP_TRY(final_boundaries(fa, s));
      HIP_TRY(back_substitute(ws.rowsC, ws.rowsV, ws.occ, gs, F.W, s, ws.bnd));
      h->fin_attempt = a;
      solved = true;
    }
    if (!solved) return set_error(BURR_E_UNSOLVABLE);
  }
  HIP_TRY(hipEventRecord(ev[2], s));
  HIP_TRY(hipStreamSynchronize(s));

  burr_stats& st = h->st;
  memset(&st, 0, sizeof(st));
  st.n = h->n;
  st.r = r;
  st.layers_built = h->built;
  uint64_t bytes = 0;
  for (uint32_t i = 0; i < h->built; ++i) {
    st.layer[i].n = h->layer[i].n;
    st.layer[i].m = h->layer[i].m;
    st.layer[i].nbuckets = h->layer[i].B;
    st.layer[i].nranges = h->layer[i].R;
    st.layer[i].bumped = h->layer[i].bumped;
    st.layer[i].steps = h->layer[i].steps;
    st.layer[i].ms_sort = h->layer[i].ms_sort;
    st.layer[i].ms_solve = h->layer[i].ms_solve;
    st.layer[i].ms_backsub = h->layer[i].ms_backsub;
    st.layer[i].ms_gather = h->layer[i].ms_gather;
    bytes += (h->layer[i].ncode + h->layer[i].nW) * 8;
  }
  st.final_n = F.n;
  st.final_m = F.m;
  st.final_attempt = h->fin_attempt;
  st.table_bytes = bytes + F.nW * 8;
  st.ms_sort = ms_sort;
  st.ms_solve = ms_solve;
  st.ms_final = elapsed_ms(ev[1], ev[2]);
  st.ms_total = elapsed_ms(ev[0], ev[2]);
  return BURR_OK;
}

void free_layer(Allocator& al, DevLayer& L) {
  al.put(L.codes);
  al.put(L.W);
  al.put(L.keys);
  L.codes = nullptr;
  L.W = nullptr;
  L.keys = nullptr;
}

burr_handle* new_handle(const burr_params* p) {
  burr_handle* h = new (std::nothrow) burr_handle();
  if (!h) return nullptr;
  h->p = *p;
  h->stream = (hipStream_t)p->stream;
  h->al.fn = p->alloc;
  h->al.ffn = p->free;
  h->al.ctx = p->alloc_ctx;
  h->al.s = h->stream;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) keep_pool_memory(dev);
  return h;
}

QueryPlan make_plan(const burr_handle* h) {
  QueryPlan plan{};
  plan.r = h->r;
  uint32_t l = 0;
  for (; l < h->built; ++l) {
    const DevLayer& L = h->layer[l];
    QueryLayer& q = plan.layer[l];
    q.salt_s = mix64(h->p.seed ^ (2ull * l + 1ull));
    q.salt_c = mix64(h->p.seed ^ (2ull * l + 2ull));
    q.span = L.m - kWidth + 1;
    q.codes = L.codes;
    q.W = L.W;
    q.t_lo = h->p.t_lo;
    q.t_hi = h->p.t_hi;
    q.plain = 0;
    q.empty = 0;
  }
  QueryLayer& f = plan.layer[l];
  f.salt_s = mix64(h->p.seed ^ (2ull * h->p.layers + 1ull));
  f.salt_c = mix64(h->p.seed ^ (2ull * h->p.layers + 2ull));
  f.span = h->fin.m ? h->fin.m - kWidth + 1 : 1;
  f.codes = nullptr;
  f.W = h->fin.W;
  f.plain = 1;
  f.empty = h->fin.m == 0;
  plan.nlayers = l + 1;
  return plan;
}

// little-endian writer that also counts
struct Out {
  uint8_t* buf;
  size_t cap;
  size_t len = 0;
  void put(uint64_t v, int bytes) {
    for (int i = 0; i < bytes; i++) {
      if (buf && len < cap) buf[len] = (uint8_t)(v >> (8 * i));
      len++;
    }
  }
  void put_words(const std::vector<uint64_t>& w) {
    for (uint64_t x : w) put(x, 8);
  }
};

struct In {
  const uint8_t* buf;
  size_t len;
  size_t off = 0;
  bool ok = true;
  uint64_t get(int bytes) {
    if (off + bytes > len) {
      ok = false;
      return 0;
    }
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)buf[off + i] << (8 * i);
    off += bytes;
    return v;
  }
};

}  // namespace

extern "C" {

void burr_default_params(burr_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->abi_version = BURR_ABI_VERSION;
  p->bucket = 64;
  p->load_num = 97;
  p->load_den = 100;
  p->final_num = 110;
  p->final_den = 100;
  p->layers = 3;
  p->t_lo = 16;
  p->t_hi = 32;
  p->ranges = 1;
  p->minbpt = 16;
  p->final_attempts = 16;
  p->filter_mode = 0;
  p->flags = 0;
  p->seed = 0;
}

burr_handle* burr_build(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                        const burr_params* p) {
  if (!params_ok(p, r, values, n) || (n > 0 && !keys)) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  burr_handle* h = new_handle(p);
  if (!h) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  h->r = r;
  h->n = n;
  int rc = build_impl(h, keys, values);
  if (rc != BURR_OK) {
    burr_free(h);
    set_error(rc);
    return nullptr;
  }
  set_error(BURR_OK);
  return h;
}

int burr_query(const burr_handle* h, const uint64_t* keys, uint64_t n, void* out, void* stream) {
  if (!h || (n > 0 && (!keys || !out))) return set_error(BURR_E_INVALID);
  QueryPlan plan = make_plan(h);
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  if (query(plan, keys, n, out, value_bytes(h->r), 0, 0, s) != hipSuccess)
    return set_error(BURR_E_DEVICE);
  return BURR_OK;
}

int burr_contains(const burr_handle* h, const uint64_t* keys, uint64_t n, uint8_t* out,
                  void* stream) {
  if (!h || !h->p.filter_mode || (n > 0 && (!keys || !out))) return set_error(BURR_E_INVALID);
  QueryPlan plan = make_plan(h);
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  if (query(plan, keys, n, out, 1, 1, mix64(~h->p.seed), s) != hipSuccess)
    return set_error(BURR_E_DEVICE);
  return BURR_OK;
}

void burr_free(burr_handle* h) {
  if (!h) return;
  for (uint32_t i = 0; i < kMaxLayers; ++i) free_layer(h->al, h->layer[i]);
  free_layer(h->al, h->fin);
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

int burr_get_stats(const burr_handle* h, burr_stats* s) {
  if (!h || !s) return set_error(BURR_E_INVALID);
  *s = h->st;
  return BURR_OK;
}

int burr_export(const burr_handle* h, void* host_buf, size_t cap, size_t* needed) {
  if (!h) return set_error(BURR_E_INVALID);
  Out o{(uint8_t*)host_buf, host_buf ? cap : 0};
  const burr_params& p = h->p;
  o.put(kExportMagic, 8);
  const uint32_t hdr[16] = {kExportVersion, kWidth,        p.bucket,  h->r,         p.load_num,
                            p.load_den,     p.final_num,   p.final_den, p.layers,   p.t_lo,
                            p.t_hi,         p.ranges,      p.minbpt,  p.final_attempts,
                            p.filter_mode,  h->built};
  for (uint32_t x : hdr) o.put(x, 4);
  o.put(p.seed, 8);
  o.put(h->n, 8);
  std::vector<uint64_t> tmp;
  auto copy_words = [&](const uint64_t* d, uint64_t nw) -> bool {
    tmp.assign(nw, 0);
    if (nw && hipMemcpy(tmp.data(), d, nw * 8, hipMemcpyDeviceToHost) != hipSuccess) return false;
    return true;
  };
  const bool fill = host_buf != nullptr;
  for (uint32_t l = 0; l < h->built; ++l) {
    const DevLayer& L = h->layer[l];
    o.put(L.n, 8);
    o.put(L.m, 8);
    o.put(L.R, 8);
    if (fill) {
      if (!copy_words(L.codes, L.ncode)) return set_error(BURR_E_DEVICE);
      o.put_words(tmp);
      if (!copy_words(L.W, L.nW)) return set_error(BURR_E_DEVICE);
      o.put_words(tmp);
    } else {
      o.len += (L.ncode + L.nW) * 8;
    }
  }
  o.put(h->fin.n, 8);
  o.put(h->fin.m, 8);
  o.put(h->fin_attempt, 8);
  if (fill) {
    if (!copy_words(h->fin.W, h->fin.nW)) return set_error(BURR_E_DEVICE);
    o.put_words(tmp);
  } else {
    o.len += h->fin.nW * 8;
  }
  if (needed) *needed = o.len;
  if (host_buf && o.len > cap) return set_error(BURR_E_INVALID);
  return BURR_OK;
}

burr_handle* burr_import(const void* host_buf, size_t len, const burr_params* pin) {
  burr_params def;
  burr_default_params(&def);
  if (pin) {
    def.stream = pin->stream;
    def.alloc = pin->alloc;
    def.free = pin->free;
    def.alloc_ctx = pin->alloc_ctx;
  }
  In in{(const uint8_t*)host_buf, host_buf ? len : 0};
  if (in.get(8) != kExportMagic) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  uint32_t hdr[16];
  for (auto& x : hdr) x = (uint32_t)in.get(4);
  if (!in.ok || hdr[0] != kExportVersion || hdr[1] != kWidth || hdr[2] != kBucket ||
      hdr[3] < 1 || hdr[3] > 32 || hdr[15] >= kMaxLayers) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  def.bucket = hdr[2];
  def.load_num = hdr[4];
  def.load_den = hdr[5];
  def.final_num = hdr[6];
  def.final_den = hdr[7];
  def.layers = hdr[8];
  def.t_lo = hdr[9];
  def.t_hi = hdr[10];
  def.ranges = hdr[11];
  def.minbpt = hdr[12];
  def.final_attempts = hdr[13];
  def.filter_mode = hdr[14];
  def.seed = in.get(8);
  burr_handle* h = new_handle(&def);
  if (!h) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  h->r = hdr[3];
  h->n = in.get(8);
  h->built = hdr[15];
  auto load_words = [&](uint64_t nw, uint64_t** dst) -> bool {
    if (in.off + nw * 8 > in.len) return false;
    *dst = (uint64_t*)h->al.get(nw * 8 + 8);
    if (!*dst) return false;
    if (nw && hipMemcpy(*dst, in.buf + in.off, nw * 8, hipMemcpyHostToDevice) != hipSuccess)
      return false;
    in.off += nw * 8;
    return true;
  };
  bool ok = in.ok;
  for (uint32_t l = 0; ok && l < h->built; ++l) {
    DevLayer& L = h->layer[l];
    L.n = in.get(8);
    L.m = in.get(8);
    L.R = in.get(8);
    if (!in.ok || L.m % 64 || L.m < 64) { ok = false; break; }
    L.B = L.m / 64;
    L.ncode = (L.B + 31) / 32;
    L.nW = (L.m / 64) * h->r;
    ok = load_words(L.ncode, &L.codes) && load_words(L.nW, &L.W);
  }
  if (ok) {
    h->fin.n = in.get(8);
    h->fin.m = in.get(8);
    h->fin_attempt = in.get(8);
    ok = in.ok && h->fin.m % 64 == 0;
    if (ok) {
      h->fin.nW = (h->fin.m / 64) * h->r;
      ok = load_words(h->fin.nW, &h->fin.W);
    }
  }
  if (!ok || in.off != in.len) {
    burr_free(h);
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  h->st.n = h->n;
  h->st.r = h->r;
  h->st.layers_built = h->built;
  set_error(BURR_OK);
  return h;
}

int64_t burr_debug_layer_keys(const burr_handle* h, uint32_t layer, uint64_t* host_out,
                              uint64_t cap) {
  if (!h || layer > h->built || !(h->p.flags & BURR_FLAG_KEEP_LAYER_KEYS))
    return set_error(BURR_E_INVALID);
  const DevLayer& L = layer < h->built ? h->layer[layer] : h->fin;
  uint64_t n = L.n;
  if (host_out && cap) {
    uint64_t c = std::min(n, cap);
    if (c && hipMemcpy(host_out, L.keys, c * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(BURR_E_DEVICE);
  }
  return (int64_t)n;
}

int burr_last_error(void) { return g_last_error; }

const char* burr_error_string(int code) {
  switch (code) {
    case BURR_OK: return "ok";
    case BURR_E_INVALID: return "invalid argument";
    case BURR_E_NOMEM: return "out of memory";
    case BURR_E_UNSOLVABLE: return "final layer unsolvable (conflicting duplicate keys?)";
    case BURR_E_DEVICE: return "HIP device error";
    case BURR_E_BUDGET: return "request exceeds the memory budget";
    default: return "unknown error";
  }
}

}  // extern "C"
