// burr_api.cpp - C ABI of the BuRR library (include/burr.h): parameter
// checks, layer planning, workspace, the per-layer launch sequence, export
// and import.
//
// Every build is a batch: one or more independent structures whose layers
// are built together - each kernel launch covers the same layer of every
// structure that still has keys (a single build is a batch of one). The
// members share one device allocation per layer for their threshold codes
// and solution words; a handle is a view of one member.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <functional>
#include <new>
#include <thread>
#include <vector>

#include "../../include/burr.h"
#include "burr_internal.h"
#include "burr_kernels.h"

using namespace burr;

namespace {

thread_local int g_last_error = BURR_OK;

int set_error(int code) {
  g_last_error = code;
  return code;
}

constexpr uint64_t kExportMagic = 0x3170786552527542ull;  // "BuRRexp1"
constexpr uint32_t kExportVersion = 2;
constexpr uint32_t kMaxLayers = 32;
constexpr uint64_t kFinalSegBuckets = 4;  // final layer: buckets per segment
// Row sets (rows, values, occupancy and the layer table): BuRR layer L uses
// set L % kBurrSets, the final layer set kBurrSets; layer L + kBurrSets is
// the first to reuse layer L's set, after its back-substitution.
constexpr int kBurrSets = 3;
constexpr int kRowSets = kBurrSets + 1;
// Waves of a back-substitution on the side stream: it overlaps the deeper
// layers, whose insertions are bound by their waves' latency, and takes a
// bounded share of the device (2 waves per SIMD, or a quarter of its full
// grid if that is wider) so that it slows them less
// and does not hold back their short launches behind a full grid (measured
// at 100M keys: 5.35 ms of device time against 5.37 with a full grid and
// 5.39 with one wave per SIMD)
constexpr uint32_t kSideBacksubWaves = 2048;
// layers of at least this many structures start their back-substitution
// right after the gather of the bumped keys (measured with 200,000
// structures: 43.3-43.9 -> 42.2-42.6 ms per batch; a single 100M-key build
// started early took 5.70 instead of 5.50 ms)
constexpr uint32_t kEarlyBacksubStructs = 4096;
// item indices (one per key plus one per bucket) are 32-bit
constexpr uint64_t kMaxKeys = 0xf0000000ull;

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

// A few host threads for the per-structure loops of large batches (the
// tables of hundreds of thousands of structures are planned, copied and
// read back per layer, and a single core's memory bandwidth made that
// milliseconds per layer). Created on first use and kept for the life of
// the process: the threads are detached and the pool is never destroyed, so
// no static destructor waits for them at exit.
class Workers {
 public:
  static Workers& get() {
    static Workers* w = new Workers();
    return *w;
  }
  uint32_t size() const { return nthreads_ + 1; }
  // fn(k) for every k in [0, n), on the workers and the calling thread; one
  // job at a time (concurrent callers take turns). fn must not throw.
  void run(uint32_t n, const std::function<void(uint32_t)>& fn) {
    if (nthreads_ == 0 || n <= 1) {
      for (uint32_t k = 0; k < n; ++k) fn(k);
      return;
    }
    std::lock_guard<std::mutex> one(run_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &fn;
      njob_ = n;
      next_.store(0);
      ++gen_;
    }
    start_.notify_all();
    for (uint32_t k; (k = next_.fetch_add(1)) < n;) fn(k);
    // every task is claimed; wait for the workers still running one
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return busy_ == 0; });
    job_ = nullptr;
  }

 private:
  Workers() {
    const unsigned hw = std::thread::hardware_concurrency();
    const uint32_t want = hw > 1 ? std::min(hw, 8u) - 1 : 0u;
    // a thread that cannot be created leaves the pool smaller (the caller
    // runs every task itself when there is none)
    for (uint32_t i = 0; i < want; ++i) {
      try {
        std::thread([this] { loop(); }).detach();
      } catch (...) {
        break;
      }
      ++nthreads_;
    }
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      // a worker that wakes after its job ended (job_ reset) waits for the next
      start_.wait(lk, [&] { return gen_ != seen && job_ != nullptr; });
      seen = gen_;
      const std::function<void(uint32_t)>* f = job_;
      const uint32_t n = njob_;
      ++busy_;
      lk.unlock();
      for (uint32_t k; (k = next_.fetch_add(1)) < n;) (*f)(k);
      lk.lock();
      if (--busy_ == 0) done_.notify_all();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable start_, done_;
  const std::function<void(uint32_t)>* job_ = nullptr;  // guarded by mu_
  uint32_t njob_ = 0, busy_ = 0;                         // guarded by mu_
  uint64_t gen_ = 0;                                     // guarded by mu_
  std::atomic<uint32_t> next_{0};
  uint32_t nthreads_ = 0;
};

// Loops over at least this many structures run on the workers, in chunks
// of at least kParallelChunk.
constexpr size_t kParallelStructs = 32768;
constexpr size_t kParallelChunk = 8192;
size_t parallel_chunks(size_t n) {
  if (n < kParallelStructs) return 1;
  return std::min<size_t>(4 * Workers::get().size(), n / kParallelChunk);
}

// Host copy of a layer's per-structure table (see LayerGeom).
struct Table {
  std::vector<uint64_t> key_off{0}, span, bucket_base{0}, range_base{0}, word_base{0},
      code_base{0}, thr_base{0}, rank_base{0};
  std::vector<uint32_t> rbits;
  uint32_t thr_mode = 0;  // 1: 1+-bit thresholds (bit words, bytes, rank directory)
  // threshold words of a structure with B buckets: 2-bit codes or 1+-bit bits
  uint64_t code_words(uint64_t B) const { return thr_mode ? (B + 63) / 64 : (B + 31) / 32; }
  void reserve(size_t J) {
    for (auto* v : {&key_off, &span, &bucket_base, &range_base, &word_base, &code_base,
                    &thr_base, &rank_base})
      v->reserve(J + 1);
    rbits.reserve(J);
  }
  // the whole table at once: geo(i, &n, &m, &R, &r) gives structure i's keys,
  // slots, ranges and value bits (called from several threads for large J)
  template <class Geo>
  void fill(size_t J, Geo geo) {
    key_off.resize(J + 1);
    span.resize(J);
    bucket_base.resize(J + 1);
    range_base.resize(J + 1);
    word_base.resize(J + 1);
    code_base.resize(J + 1);
    thr_base.resize(J + 1);
    rank_base.resize(J + 1);
    rbits.resize(J);
    const size_t nch = parallel_chunks(J);
    if (nch == 1) {  // one pass
      uint64_t ko = 0, bb = 0, rb = 0, wb = 0, cb = 0, tb = 0, kb = 0;
      for (size_t i = 0; i < J; ++i) {
        uint64_t n, m, R;
        uint32_t r;
        geo(i, &n, &m, &R, &r);
        const uint64_t B = m / 64;
        key_off[i] = ko;
        span[i] = m - kWidth + 1;
        bucket_base[i] = bb;
        range_base[i] = rb;
        word_base[i] = wb;
        code_base[i] = cb;
        thr_base[i] = tb;
        rank_base[i] = kb;
        rbits[i] = r;
        ko += n;
        bb += B;
        rb += R;
        wb += B * r;
        cb += code_words(B);
        tb += B;
        kb += (code_words(B) + 7) / 8;
      }
      key_off[J] = ko;
      bucket_base[J] = bb;
      range_base[J] = rb;
      word_base[J] = wb;
      code_base[J] = cb;
      thr_base[J] = tb;
      rank_base[J] = kb;
      return;
    }
    // in chunks on the host workers: pass 1 stores every structure's own
    // sizes and sums them per chunk, pass 2 turns them into running offsets
    // (key_off, bucket_base, range_base, word_base, code_base, thr_base,
    // rank_base)
    uint64_t* const base[7] = {key_off.data(),  bucket_base.data(), range_base.data(),
                               word_base.data(), code_base.data(),   thr_base.data(),
                               rank_base.data()};
    std::vector<uint64_t> csum(7 * (nch + 1), 0);
    auto lo_of = [&](size_t c) { return J * c / nch; };
    Workers::get().run((uint32_t)nch, [&](uint32_t c) {
      uint64_t sn = 0, sB = 0, sR = 0, sW = 0, sC = 0, sK = 0;
      uint64_t *const ko = key_off.data(), *const bb = bucket_base.data(),
                      *const rb = range_base.data(), *const wb = word_base.data(),
                      *const cb = code_base.data(), *const tb = thr_base.data(),
                      *const kb = rank_base.data(), *const sp = span.data();
      uint32_t* const rr = rbits.data();
      for (size_t i = lo_of(c); i < lo_of(c + 1); ++i) {
        uint64_t n, m, R;
        uint32_t r;
        geo(i, &n, &m, &R, &r);
        const uint64_t B = m / 64, cw = code_words(B);
        ko[i] = n;
        bb[i] = B;
        rb[i] = R;
        wb[i] = B * r;
        cb[i] = cw;
        tb[i] = B;
        kb[i] = (cw + 7) / 8;
        sp[i] = m - kWidth + 1;
        rr[i] = r;
        sn += n;
        sB += B;
        sR += R;
        sW += B * r;
        sC += cw;
        sK += (cw + 7) / 8;
      }
      const uint64_t sum[7] = {sn, sB, sR, sW, sC, sB, sK};
      for (int k = 0; k < 7; ++k) csum[7 * (c + 1) + k] = sum[k];
    });
    for (size_t c = 1; c <= nch; ++c)  // chunk sums to chunk offsets
      for (int k = 0; k < 7; ++k) csum[7 * c + k] += csum[7 * (c - 1) + k];
    Workers::get().run((uint32_t)nch, [&](uint32_t c) {
      for (int k = 0; k < 7; ++k) {
        uint64_t run = csum[7 * c + k];
        uint64_t* const a = base[k];
        for (size_t i = lo_of(c); i < lo_of(c + 1); ++i) {
          const uint64_t v = a[i];
          a[i] = run;
          run += v;
        }
      }
    });
    for (int k = 0; k < 7; ++k) base[k][J] = csum[7 * nch + k];
  }
  // next structure: n keys, m slots, R ranges (final layer: segments), r value bits
  void add(uint64_t n, uint64_t m, uint64_t R, uint32_t r) {
    const uint64_t B = m / 64;
    key_off.push_back(key_off.back() + n);
    span.push_back(m - kWidth + 1);
    bucket_base.push_back(bucket_base.back() + B);
    range_base.push_back(range_base.back() + R);
    word_base.push_back(word_base.back() + B * r);
    code_base.push_back(code_base.back() + code_words(B));
    thr_base.push_back(thr_base.back() + B);
    rank_base.push_back(rank_base.back() + (code_words(B) + 7) / 8);
    rbits.push_back(r);
  }
  uint32_t J() const { return (uint32_t)rbits.size(); }
};

// one layer of one member, as derived from its layer's table
struct MemberLayer {
  uint64_t n = 0, m = 0, R = 0, bumped = 0;
  uint64_t code_off = 0, ncode = 0;  // words of the layer's shared code (1+-bit: bit) array
  uint64_t word_off = 0, nW = 0;     // words of the layer's shared solution array
  uint64_t key_off = 0;              // debug: first key in the layer's kept key array
  uint64_t thr_off = 0, K = 0;       // 1+-bit: first threshold byte, thresholds
  uint64_t rank_off = 0, nrank = 0;  // 1+-bit: rank directory entries
  uint64_t range_off = 0;            // first global range (cut points)
};

// storage shared by all members of a batch for one layer, and the geometry
// of the members with keys in it: ids ascending, entry k of the table and of
// `bumped` (keys passed to the next layer) belongs to member ids[k]
struct LayerStore {
  uint64_t* codes = nullptr;  // 2-bit code words, or 1+-bit bit words
  uint64_t* W = nullptr;
  uint8_t* thr = nullptr;     // 1+-bit: thresholds - 1 (table.thr_base per structure)
  uint32_t* rank = nullptr;   // 1+-bit: rank directory (table.rank_base per structure)
  uint32_t* kcount = nullptr; // 1+-bit: thresholds per structure (device)
  std::vector<uint32_t> kthr; // the same on the host, after the build
  uint32_t* rfirst = nullptr; // with a cut strategy: first bucket of every range (+1)
  uint64_t* keys = nullptr;  // kept input keys (debug flag)
  uint64_t steps = 0;
  double ms_sort = 0, ms_solve = 0, ms_backsub = 0, ms_gather = 0;
  std::vector<uint32_t> ids;
  Table t;
  std::vector<uint32_t> bumped;
};

// the final plain layer of one member
struct FinalLayer {
  uint64_t n = 0, m = 0, nW = 0;
};

struct Member {
  uint64_t n = 0;
  uint32_t r = 0;
  uint32_t built = 0;  // BuRR layers with keys (their records sit in the layer stores)
  uint32_t minbpt = 0;  // minimum buckets per range of this structure (0: the batch's)
  FinalLayer fin;
  uint64_t fin_attempt = 0;
  const uint64_t* fin_W = nullptr;
  const uint64_t* fin_keys = nullptr;  // debug
};

}  // namespace

struct burr_handle {
  struct burr_batch* b = nullptr;
  uint32_t idx = 0;
  bool owner = false;  // a single build: freeing the handle frees the batch
};

struct burr_batch {
  burr_params p{};
  hipStream_t stream = nullptr;
  Allocator al;
  std::vector<Member> members;
  std::vector<burr_handle> views;
  LayerStore layers[kMaxLayers];
  std::vector<void*> owned;  // every device allocation of the batch
  uint64_t table_bytes = 0;  // device bytes held for tables (arena + extra allocations)
  uint8_t* arena = nullptr;  // one allocation that the layers' tables are carved from
  uint64_t arena_cap = 0, arena_used = 0;
  double ms_total = 0, ms_final = 0;
  bool no_alloc = false;  // tables live in caller memory (the arena) only

  void* alloc(uint64_t bytes) {
    if (no_alloc) return nullptr;
    void* p = al.get(bytes);
    if (p) owned.push_back(p);
    return p;
  }
  // table storage: from the arena while it lasts, else its own allocation
  void* alloc_table(uint64_t bytes) {
    bytes = (bytes + 255) & ~255ull;
    if (arena && arena_used + bytes <= arena_cap) {
      void* p = arena + arena_used;
      arena_used += bytes;
      return p;
    }
    void* p = alloc(bytes);
    if (p) table_bytes += bytes;
    return p;
  }
};

namespace {

// member idx's record of layer l < its built count
MemberLayer layer_of(const burr_batch* b, uint32_t idx, uint32_t l) {
  const LayerStore& LS = b->layers[l];
  const size_t k = std::lower_bound(LS.ids.begin(), LS.ids.end(), idx) - LS.ids.begin();
  const Table& t = LS.t;
  MemberLayer L;
  L.n = t.key_off[k + 1] - t.key_off[k];
  L.m = t.span[k] + kWidth - 1;
  L.R = t.range_base[k + 1] - t.range_base[k];
  L.bumped = LS.bumped[k];
  L.code_off = t.code_base[k];
  L.ncode = t.code_base[k + 1] - t.code_base[k];
  L.word_off = t.word_base[k];
  L.nW = t.word_base[k + 1] - t.word_base[k];
  L.key_off = t.key_off[k];
  L.thr_off = t.thr_base[k];
  L.K = k < LS.kthr.size() ? LS.kthr[k] : 0;
  L.rank_off = t.rank_base[k];
  L.nrank = t.rank_base[k + 1] - t.rank_base[k];
  L.range_off = t.range_base[k];
  return L;
}

bool params_ok(const burr_params* p) {
  if (!p || p->abi_version != BURR_ABI_VERSION) return false;
  if (p->bucket != kBucket) return false;  // the kernels handle b = w = 64
  if (!(p->t_lo > 0 && p->t_lo < p->t_hi && p->t_hi < p->bucket)) return false;
  if (!p->load_num || !p->load_den || !p->final_num || !p->final_den) return false;
  if (p->final_num < p->final_den) return false;
  if (p->layers > kMaxLayers - 1) return false;
  if (!p->ranges || !p->final_attempts) return false;
  if (p->threshold_mode > 1 || p->cut_strategy > 3) return false;
  return true;
}

uint64_t ceil_div(unsigned __int128 a, unsigned __int128 b) { return (uint64_t)((a + b - 1) / b); }

// BuRR layer: m = b * max(1, ceil(load * n / b)) slots, B = m/b buckets,
// R = min(ranges, B / max(minbpt, 2)) ranges, at least 1 (minbpt: the
// structure's own value, 0 = the parameter block's).
void plan_layer(const burr_params& p, uint64_t n, uint64_t* m, uint64_t* R, uint32_t minbpt = 0) {
  const uint64_t den = (uint64_t)p.load_den * kBucket;
  uint64_t nb = n <= (~0ull - den) / p.load_num
                    ? (n * p.load_num + den - 1) / den
                    : ceil_div((unsigned __int128)n * p.load_num, (unsigned __int128)den);
  if (nb < 1) nb = 1;
  if (!minbpt) minbpt = p.minbpt;
  const uint64_t per = minbpt < 2 ? 2 : minbpt;
  uint64_t r = nb / per;
  if (r > p.ranges) r = p.ranges;
  if (r < 1) r = 1;
  *m = nb * kBucket;
  *R = r;
}

// Division by a divisor fixed for a whole build, by a precomputed
// reciprocal: q = high word of n * floor(2^64 / d) is q or q-1, one
// correction step fixes it (the tables of large batches plan hundreds of
// thousands of structures per layer).
struct FastDiv {
  uint64_t d = 1, M = 0;
  FastDiv() = default;
  explicit FastDiv(uint64_t dd) : d(dd), M(dd > 1 ? (uint64_t)(((unsigned __int128)1 << 64) / dd) : 0) {}
  uint64_t div(uint64_t n) const {
    if (d == 1) return n;
    uint64_t q = (uint64_t)(((unsigned __int128)n * M) >> 64);
    if (n - q * d >= d) ++q;
    return q;
  }
};

// plan_layer for many structures of one build
struct LayerPlanner {
  const burr_params& p;
  FastDiv den, per;
  uint64_t lim;  // up to lim keys, n * load_num + den - 1 fits 64 bits
  explicit LayerPlanner(const burr_params& pp)
      : p(pp), den((uint64_t)pp.load_den * kBucket), per(pp.minbpt < 2 ? 2 : pp.minbpt),
        lim((~0ull - den.d) / pp.load_num) {}
  void plan(uint64_t n, uint32_t minbpt, uint64_t* m, uint64_t* R) const {
    uint64_t nb = n <= lim ? den.div(n * p.load_num + den.d - 1)
                           : ceil_div((unsigned __int128)n * p.load_num, (unsigned __int128)den.d);
    if (nb < 1) nb = 1;
    if (!minbpt) minbpt = p.minbpt;
    const uint64_t pr = minbpt < 2 ? 2 : minbpt;
    uint64_t r = pr == per.d ? per.div(nb) : nb / pr;
    if (r > p.ranges) r = p.ranges;
    if (r < 1) r = 1;
    *m = nb * kBucket;
    *R = r;
  }
};

// Final plain ribbon, attempt a: m = 64 * max(1, ceil(n * (final + a/10) / 64)).
uint64_t plan_final(const burr_params& p, uint64_t n, uint32_t attempt) {
  const unsigned __int128 num =
      (unsigned __int128)n * ((uint64_t)p.final_num * 10u + (uint64_t)attempt * p.final_den);
  uint64_t nb = ceil_div(num, (unsigned __int128)p.final_den * 10u * kWidth);
  if (nb < 1) nb = 1;
  return nb * kWidth;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) {                                                            \
      fprintf(stderr, "burr: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(_e), \
              __FILE__, __LINE__);                                                     \
      return set_error(BURR_E_DEVICE);                                                 \
    }                                                                                  \
  } while (0)

// Device workspace of a build; grows on demand. Two modes:
//  - with the build's allocator (caller callbacks or the stream-ordered pool):
//    outgrown buffers are released with the workspace, after every launch
//    that used them;
//  - kept between builds (al == nullptr, plain hipMalloc): an outgrown buffer
//    is freed at once; hipFree waits for the device first, so a buffer that
//    the previous layer's last kernels still use is never freed under them
//    (the next layer is planned while they run).
struct Workspace {
  Allocator* al;
  std::vector<void*> owned;
  std::vector<size_t> owned_bytes;
  uint64_t bytes = 0;           // device bytes held
  uint8_t* host = nullptr;      // pinned staging of layer tables (host -> device)
  size_t host_cap = 0;
  uint32_t* hres = nullptr;     // pinned copy of the per-layer results
  size_t hres_cap = 0;
  uint32_t* res = nullptr;      // per-layer results: fail[J], soff[J+1], steps (u64)
  uint64_t cap_res = 0;
  uint64_t cap_keys = 0, cap_B = 0, cap_items = 0, cap_scan = 0;
  uint64_t cap_seg = 0, cap_tab[kRowSets] = {}, cap_J = 0, cap_c1 = 0, cap_c2 = 0, cap_plan = 0;
  uint64_t* keysA = nullptr;  // next layer's keys
  uint32_t* valsA = nullptr;
  uint4 *p1 = nullptr, *p2 = nullptr;  // sort intermediates (12- or 16-byte records)
  uint32_t *counts1 = nullptr, *counts2 = nullptr;
  uint32_t *binlo = nullptr, *nch = nullptr, *cbase = nullptr, *sstart = nullptr;
  Rec* rec = nullptr;
  // row arrays: BuRR layer L inserts into set L % kBurrSets while the
  // back-substitutions of earlier layers read theirs on the side stream;
  // the final layer has the last set
  uint64_t* rowsC[kRowSets] = {};
  uint32_t* rowsV[kRowSets] = {};
  uint64_t* occ[kRowSets] = {};
  uint64_t cap_m[kRowSets] = {};
  hipStream_t side = nullptr;  // back-substitution (default priority, non-blocking)
  std::vector<hipEvent_t> evs;  // a build's timing and ordering events, kept for the next
  // host lists of the members with keys in the current and the next layer
  // and their key counts, kept for the next build (fresh allocations of
  // that size cost page faults on every build)
  std::vector<uint32_t> h_active, h_next_active;
  std::vector<uint64_t> h_cur_n, h_next_n;
  std::vector<uint64_t> h_rm;  // per member: minbpt << 32 | value bits (compact for planning)
  // per-bucket codes of a BuRR layer, one buffer per row set: a layer's
  // codes are packed on the side stream before its back-substitution,
  // while the next layer's insertion writes the other buffer
  uint8_t* codes8[kBurrSets] = {};
  uint64_t cap_codes[kBurrSets] = {};
  uint32_t *bump = nullptr, *bstart = nullptr, *scan_tmp = nullptr;
  uint32_t* pcount = nullptr;  // 1+-bit thresholds: popcounts of the bit words, scanned
  uint64_t cap_pc = 0;
  uint32_t* fail = nullptr;  // per structure
  uint32_t* soff = nullptr;  // per structure: first bumped key
  uint64_t* steps = nullptr;
  uint64_t* tab[kRowSets] = {};  // layer tables, one per row set
  uint64_t* diag = nullptr;  // insertion-kernel diagnostics (16 u64)
  uint64_t *spillC = nullptr, *spill_occ = nullptr, *xfirst = nullptr;
  uint32_t *spillV = nullptr, *z0first = nullptr, *bnd = nullptr;
  // scratch mode (builds that allocate nothing): every device buffer is
  // carved from a fixed region, the host staging and results use the fixed
  // arrays below (pageable), and nothing is freed
  uint8_t* scr = nullptr;
  uint64_t scr_cap = 0, scr_used = 0;
  uint64_t fixed_host[64];
  uint32_t fixed_res[64];

  explicit Workspace(Allocator* a) : al(a) {}
  Workspace(uint8_t* region, uint64_t cap) : al(nullptr), scr(region), scr_cap(cap) {}
  ~Workspace() {
    for (void* p : owned) {
      if (al)
        al->put(p);
      else
        (void)hipFree(p);
    }
    if (host && !scr) (void)hipHostFree(host);
    if (hres && !scr) (void)hipHostFree(hres);
    if (side) (void)hipStreamDestroy(side);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
  // at least n events (created once per workspace; a build records all it uses)
  hipEvent_t* events(size_t n) {
    while (evs.size() < n) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      evs.push_back(e);
    }
    return evs.data();
  }
  hipStream_t side_stream() {
    if (!side && hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess)
      side = nullptr;
    return side;
  }
  template <typename T>
  bool alloc(T*& ptr, uint64_t count) {
    const size_t b = ((count * sizeof(T)) + 255) & ~(size_t)255;
    if (scr) {  // carve from the fixed region; an outgrown buffer stays where it is
      const uint64_t need = b ? b : 256;
      if (need > scr_cap - scr_used) {
        ptr = nullptr;
        return false;
      }
      ptr = reinterpret_cast<T*>(scr + scr_used);
      scr_used += need;
      bytes += need;
      return true;
    }
    if (!al) {  // kept between builds: replace the outgrown buffer
      for (size_t k = 0; ptr && k < owned.size(); ++k)
        if (owned[k] == (void*)ptr) {
          (void)hipFree(owned[k]);
          bytes -= owned_bytes[k];
          owned.erase(owned.begin() + k);
          owned_bytes.erase(owned_bytes.begin() + k);
          break;
        }
      void* p = nullptr;
      if (hipMalloc(&p, b ? b : 256) != hipSuccess) {
        ptr = nullptr;
        return false;
      }
      ptr = (T*)p;
    } else {
      ptr = (T*)al->get(b);
      if (!ptr) return false;
    }
    owned.push_back((void*)ptr);
    owned_bytes.push_back(b);
    bytes += b;
    return true;
  }
  // pinned host staging of at least `need` bytes
  bool reserve_host(size_t need) {
    if (scr) {
      host = reinterpret_cast<uint8_t*>(fixed_host);
      host_cap = sizeof(fixed_host);
      return need <= host_cap;
    }
    if (need <= host_cap && host) return true;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    host_cap = std::max<size_t>(need, 1 << 16);
    if (hipHostMalloc((void**)&host, host_cap, hipHostMallocDefault) != hipSuccess) {
      host = nullptr;
      host_cap = 0;
      return false;
    }
    return true;
  }
  // fail[J] | soff[J+1] | pad | steps u64[4], on the device and pinned on the host
  bool reserve_results(uint64_t J) {
    const uint64_t words = 2 * J + 12;
    if (words > cap_res || !res) {
      cap_res = words;
      if (!alloc(res, words)) return false;
    }
    if (scr) {
      hres = fixed_res;
      hres_cap = sizeof(fixed_res);
      if (words * 4 > hres_cap) return false;
    } else if (words * 4 > hres_cap || !hres) {
      if (hres) (void)hipHostFree(hres);
      hres = nullptr;
      hres_cap = words * 4;
      if (hipHostMalloc((void**)&hres, hres_cap, hipHostMallocDefault) != hipSuccess) {
        hres = nullptr;
        hres_cap = 0;
        return false;
      }
    }
    fail = res;
    soff = res + J;
    steps = reinterpret_cast<uint64_t*>(res + 2 * J + 2);
    return true;
  }
  uint64_t results_words(uint64_t J) const { return 2 * J + 10; }
  bool reserve_keys(uint64_t n) {
    if (n <= cap_keys && keysA) return true;
    cap_keys = std::max<uint64_t>(n, 1);
    return alloc(keysA, cap_keys) && alloc(valsA, cap_keys) && alloc(p1, cap_keys) &&
           alloc(p2, cap_keys);
  }
  bool reserve_items(uint64_t count) {  // one record per key + one header per bucket
    if (count <= cap_items && rec) return true;
    cap_items = count;
    return alloc(rec, count);
  }
  bool reserve_slots(uint64_t m, int set) {
    if (m <= cap_m[set] && rowsC[set]) return true;
    cap_m[set] = m;
    return alloc(rowsC[set], m) && alloc(rowsV[set], m) && alloc(occ[set], m / 64 + 1);
  }
  bool reserve_scan(uint64_t n) {
    const uint64_t need = scan_tmp_words(n) + 64;
    if (need <= cap_scan && scan_tmp) return true;
    cap_scan = need;
    return alloc(scan_tmp, need);
  }
  bool reserve_codes(uint64_t B, int set) {
    if (B <= cap_codes[set] && codes8[set]) return true;
    cap_codes[set] = B;
    return alloc(codes8[set], B + 1);
  }
  bool reserve_buckets(uint64_t B) {
    if (B <= cap_B && bump) return reserve_scan(B + 1);
    cap_B = B;
    return alloc(bump, B + 1) && alloc(bstart, B + 1) &&
           reserve_scan(B + 1);
  }
  bool reserve_sort(const SortPlan& sp) {
    const uint64_t c1 = (uint64_t)sp.nb1 * sp.G1, c2 = sort_counts2_words(sp);
    const uint64_t pl = std::max<uint64_t>(sp.nb1, sp.nsub) + 1;
    if ((c1 > cap_c1 || !counts1) && !alloc(counts1, (cap_c1 = c1) + 1)) return false;
    if ((c2 > cap_c2 || !counts2) && !alloc(counts2, (cap_c2 = c2) + 1)) return false;
    if (pl > cap_plan || !binlo) {
      cap_plan = pl;
      if (!alloc(binlo, pl) || !alloc(nch, pl) || !alloc(cbase, pl) || !alloc(sstart, pl))
        return false;
    }
    return reserve_scan(std::max(c1, c2) + 1);
  }
  bool reserve_structs(uint64_t J) { return reserve_results(J); }
  bool reserve_pcount(uint64_t words) {
    if (words <= cap_pc && pcount) return reserve_scan(words + 1);
    cap_pc = words;
    return alloc(pcount, words + 1) && reserve_scan(words + 1);
  }
  bool reserve_table(uint64_t words, int set) {
    if (words <= cap_tab[set] && tab[set]) return true;
    cap_tab[set] = words;
    return alloc(tab[set], words);
  }
  bool reserve_segments(uint64_t P) {
    if (P <= cap_seg && spillC) return true;
    cap_seg = P;
    return alloc(spillC, P * 64) && alloc(spillV, P * 64) && alloc(spill_occ, P) &&
           alloc(xfirst, P * 64) && alloc(z0first, P * 64) && alloc(bnd, P * 64);
  }
};

void print_diag(const uint64_t* d) {
  uint64_t h[16] = {0};
  if (hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess || !h[0]) return;
  fprintf(stderr,
          "burr: wave state: code %llu range %llu structure %llu header item %llu records %llu "
          "bucket %llu of %llu candidates %llu kept %llu threshold %llu forced %llu first "
          "bucket %llu\n",
          (unsigned long long)h[1], (unsigned long long)h[2], (unsigned long long)h[3],
          (unsigned long long)h[4], (unsigned long long)h[5], (unsigned long long)h[6],
          (unsigned long long)h[7], (unsigned long long)h[8], (unsigned long long)h[10],
          (unsigned long long)h[11], (unsigned long long)h[12], (unsigned long long)h[15]);
}

// Uploads a table (one device buffer) and fills the geometry's pointers and totals.
// The table goes to ws.tab[set]: a layer's back-substitution reads it on the
// side stream while the next layer uploads its own into the other buffer.
int upload_table(Workspace& ws, const Table& t, LayerGeom& g, hipStream_t s, int set) {
  const uint64_t J = t.J();
  const uint64_t words = 8 * (J + 1) + (J + 1) / 2 + 1;
  if (!ws.reserve_table(words, set) || !ws.reserve_host(words * 8)) return set_error(BURR_E_NOMEM);
  uint64_t* const tab = ws.tab[set];
  // the pinned staging is reused only after the stream has passed this copy
  // (the host waits for each layer's results, which follow it on the stream)
  uint64_t* h = reinterpret_cast<uint64_t*>(ws.host);
  // only the words no copy below fills are cleared: the last word of the
  // span run, the odd half word after rbits and the trailing pad word
  h[2 * (J + 1) - 1] = 0;
  h[8 * (J + 1) + J / 2] = 0;
  h[words - 1] = 0;
  struct Piece {
    void* dst;
    const void* src;
    size_t bytes;
  };
  const Piece parts[9] = {
      {h, t.key_off.data(), (J + 1) * 8},
      {h + (J + 1), t.span.data(), J * 8},
      {h + 2 * (J + 1), t.bucket_base.data(), (J + 1) * 8},
      {h + 3 * (J + 1), t.range_base.data(), (J + 1) * 8},
      {h + 4 * (J + 1), t.word_base.data(), (J + 1) * 8},
      {h + 5 * (J + 1), t.code_base.data(), (J + 1) * 8},
      {h + 6 * (J + 1), t.thr_base.data(), (J + 1) * 8},
      {h + 7 * (J + 1), t.rank_base.data(), (J + 1) * 8},
      {h + 8 * (J + 1), t.rbits.data(), J * 4},
  };
  // large tables: each array in pieces, copied by the host workers
  const size_t nch = parallel_chunks(J);
  if (nch == 1) {
    for (const Piece& c : parts) memcpy(c.dst, c.src, c.bytes);
  } else {
    Workers::get().run((uint32_t)(9 * nch), [&](uint32_t k) {
      const Piece& c = parts[k / nch];
      const size_t i = k % nch, lo = c.bytes * i / nch / 8 * 8,
                   hi = i + 1 == nch ? c.bytes : c.bytes * (i + 1) / nch / 8 * 8;
      memcpy((char*)c.dst + lo, (const char*)c.src + lo, hi - lo);
    });
  }
  HIP_TRY(hipMemcpyAsync(tab, h, words * 8, hipMemcpyHostToDevice, s));
  g.key_off = tab;
  g.span = tab + (J + 1);
  g.bucket_base = tab + 2 * (J + 1);
  g.range_base = tab + 3 * (J + 1);
  g.word_base = tab + 4 * (J + 1);
  g.code_base = tab + 5 * (J + 1);
  g.thr_base = tab + 6 * (J + 1);
  g.rank_base = tab + 7 * (J + 1);
  g.rbits = (const uint32_t*)(tab + 8 * (J + 1));
  g.J = (uint32_t)J;
  g.nkeys = t.key_off.back();
  g.nbuckets = t.bucket_base.back();
  g.m = 64 * g.nbuckets;
  g.nranges = t.range_base.back();
  g.r = *std::max_element(t.rbits.begin(), t.rbits.end());
  return BURR_OK;
}

// Sorts one layer's keys by (bucket, chunk) into the item stream ws.rec and ws.bstart.
int run_sort(Workspace& ws, const uint64_t* keys, const void* vals, uint32_t vbytes,
             bool first_layer, bool filter, uint64_t fp_salt, const LayerGeom& g,
             hipStream_t s, const SortClear& clear) {
  SortArgs a{};
  a.keys = keys;
  a.vals = vals;
  a.vbytes = vbytes;
  a.mask_values = first_layer ? 1u : 0u;
  a.filter = filter ? 1u : 0u;
  a.fp_salt = fp_salt;
  a.g = g;
  a.plan = plan_sort(g.nkeys, g.nbuckets, g.J);
  if (!ws.reserve_sort(a.plan)) return set_error(BURR_E_NOMEM);
  if (!ws.reserve_items(g.nkeys + g.nbuckets)) return set_error(BURR_E_NOMEM);
  a.counts1 = ws.counts1;
  a.counts2 = ws.counts2;
  a.scan_tmp = ws.scan_tmp;
  a.binlo = ws.binlo;
  a.nch = ws.nch;
  a.cbase = ws.cbase;
  a.sstart = ws.sstart;
  a.r1 = ws.p1;
  a.r2 = ws.p2;
  a.out_rec = ws.rec;
  a.bstart = ws.bstart;
  a.clear = clear;
  HIP_TRY(sort_layer(a, s));
  return BURR_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0;
  return ms;
}

// Final plain layer of the listed members at one attempt index each. Their
// final keys lie contiguously at `keys`, in list order. The table is cut
// into segments of kFinalSegBuckets buckets that are solved in parallel;
// rows crossing a segment end are merged afterwards. fails[i] = 1 if member
// list[i]'s system was inconsistent at this size (then it keeps no table).
int final_attempt(burr_batch* b, Workspace& ws, int set, const std::vector<uint32_t>& list,
                  const std::vector<uint32_t>& attempt, const uint64_t* keys, const void* vals,
                  uint32_t vbytes, bool first_layer, std::vector<uint32_t>& fails) {
  const burr_params& p = b->p;
  hipStream_t s = b->stream;
  Table t;
  uint64_t max_seg = 1;
  for (size_t i = 0; i < list.size(); ++i) {
    const Member& mb = b->members[list[i]];
    const uint64_t m = plan_final(p, mb.fin.n, attempt[i]);
    const uint64_t P = std::max<uint64_t>(1, (m / 64) / kFinalSegBuckets);
    max_seg = std::max(max_seg, P);
    t.add(mb.fin.n, m, P, mb.r);
  }
  LayerGeom g{};
  g.salt_s = mix64(p.seed ^ (2ull * p.layers + 1ull));
  g.salt_c = mix64(p.seed ^ (2ull * p.layers + 2ull));
  g.t_lo = p.t_lo;
  g.t_hi = p.t_hi;
  g.plain = 1;
  int rc = upload_table(ws, t, g, s, set);
  if (rc != BURR_OK) return rc;
  if (!ws.reserve_slots(g.m, set) || !ws.reserve_buckets(g.nbuckets) ||
      !ws.reserve_structs(g.J) || !ws.reserve_segments(g.nranges))
    return set_error(BURR_E_NOMEM);
  // the sort also clears the failure flags and the segments' spill occupancy
  const SortClear clear{{ws.res, reinterpret_cast<uint32_t*>(ws.spill_occ)},
                        {ws.results_words(g.J), 2 * g.nranges}};
  rc = run_sort(ws, keys, vals, vbytes, first_layer, p.filter_mode != 0, mix64(~p.seed), g, s,
                clear);
  if (rc != BURR_OK) return rc;
  SolveArgs sa{};
  sa.rec = ws.rec;
  sa.bstart = ws.bstart;
  sa.g = g;
  sa.rowsC = ws.rowsC[set];
  sa.rowsV = ws.rowsV[set];
  sa.occ = ws.occ[set];
  sa.fail = ws.fail;
  sa.nrec = (uint32_t)(g.nkeys + g.nbuckets);
  sa.spillC = ws.spillC;
  sa.spillV = ws.spillV;
  sa.spill_occ = ws.spill_occ;
  sa.diag = ws.diag;
  HIP_TRY(solve_layer(sa, s));
  FinalArgs fa{};
  fa.g = g;
  fa.rowsC = ws.rowsC[set];
  fa.rowsV = ws.rowsV[set];
  fa.occ = ws.occ[set];
  fa.spillC = ws.spillC;
  fa.spillV = ws.spillV;
  fa.spill_occ = ws.spill_occ;
  fa.fail = ws.fail;
  fa.z0first = ws.z0first;
  fa.xfirst = ws.xfirst;
  fa.bnd = ws.bnd;
  HIP_TRY(final_merge(fa, max_seg, s));
  // boundaries and back-substitution run for every listed member; the
  // words of a member that failed are never referenced
  HIP_TRY(final_boundaries(fa, s));
  uint64_t* W = (uint64_t*)b->alloc_table(t.word_base.back() * 8 + 8);
  if (!W) return set_error(BURR_E_NOMEM);
  HIP_TRY(back_substitute(ws.rowsC[set], ws.rowsV[set], g, W, s, ws.bnd));
  HIP_TRY(hipMemcpyAsync(ws.hres, ws.res, g.J * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  fails.assign(ws.hres, ws.hres + g.J);
  for (size_t i = 0; i < list.size(); ++i) {
    if (fails[i] >= 2) {
      fprintf(stderr, "burr: internal error %u in the final layer\n", fails[i]);
      print_diag(ws.diag);
      return set_error(BURR_E_DEVICE);
    }
    if (fails[i]) continue;
    Member& mb = b->members[list[i]];
    mb.fin.m = 64 * (t.bucket_base[i + 1] - t.bucket_base[i]);
    mb.fin.nW = t.word_base[i + 1] - t.word_base[i];
    mb.fin_W = W + t.word_base[i];
    mb.fin_attempt = attempt[i];
  }
  return BURR_OK;
}

// Builds every member of b. Member i's keys are keys[off[i], off[i+1]), its
// values the same range of `values` (elements of value_bytes(max r) bytes).
// Workspaces kept between builds, per device (plain hipMalloc memory), up
// to a total size per device: the environment variable
// BURR_WORKSPACE_CACHE_BYTES, else a quarter of the device's memory.
// burr_release_workspaces() frees them.
constexpr int kMaxDevices = 64;
std::mutex g_ws_mu;
std::vector<Workspace*> g_ws_free[kMaxDevices];

uint64_t ws_cache_limit(int dev) {
  static const char* env = getenv("BURR_WORKSPACE_CACHE_BYTES");
  if (env) return strtoull(env, nullptr, 10);
  static uint64_t lim[kMaxDevices] = {};  // read under g_ws_mu
  if (!lim[dev]) {
    size_t total = 0;
    if (hipDeviceTotalMem(&total, dev) != hipSuccess || total == 0) total = 64ull << 30;
    lim[dev] = total / 4;
  }
  return lim[dev];
}

// The workspace of one build: taken from the cache unless the caller
// supplied an allocator or opted out (BURR_FLAG_NO_WORKSPACE_CACHE).
struct WsLease {
  Workspace* ws = nullptr;
  int dev = -1;
  bool cached = false;
  hipStream_t s;
  WsLease(Allocator* al, const burr_params& p, hipStream_t st) : s(st) {
    cached = !al->fn && !(p.flags & BURR_FLAG_NO_WORKSPACE_CACHE) &&
             hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices;
    if (cached) {
      std::lock_guard<std::mutex> lk(g_ws_mu);
      if (!g_ws_free[dev].empty()) {
        ws = g_ws_free[dev].back();
        g_ws_free[dev].pop_back();
      }
    }
    if (!ws) ws = new (std::nothrow) Workspace(cached ? nullptr : al);
  }
  ~WsLease() {
    if (!ws) return;
    if (!cached) {
      if (ws->side) (void)hipStreamSynchronize(ws->side);
      delete ws;
      return;
    }
    (void)hipStreamSynchronize(s);  // no launch of this build may still use it
    if (ws->side) (void)hipStreamSynchronize(ws->side);
    std::unique_lock<std::mutex> lk(g_ws_mu);
    uint64_t held = ws->bytes;
    for (Workspace* w : g_ws_free[dev]) held += w->bytes;
    if (held <= ws_cache_limit(dev)) {
      g_ws_free[dev].push_back(ws);
      return;
    }
    lk.unlock();
    delete ws;
  }
};

// Device bytes the tables of a batch are expected to need, from its layer-0
// table: layer 0 exactly (solution words, and at most one 2-bit code word per
// 32 buckets plus one per structure), deeper layers at the bump-rate bound,
// plus the final layer; 1+-bit thresholds add at most a byte per bucket, the
// rank directory and a count; cut points half a word per range.
uint64_t batch_table_estimate(const burr_params& p, const Table& t) {
  const uint64_t J = t.J(), B = t.bucket_base.back();
  uint64_t words = t.word_base.back() + B / 32 + J;
  if (p.threshold_mode == 1) words += B / 8 + B / 1024 + 4 * J;
  if (p.cut_strategy) words += t.range_base.back() / 2 + J;
  return words * 8 * 116 / 100 + 4096ull * (p.layers + 2);
}

// The same from the members' sizes, for a batch that builds no BuRR layer
// (no layers, or no keys).
uint64_t batch_table_estimate(const burr_batch* b, const std::vector<uint64_t>& off) {
  Table t;
  t.thr_mode = b->p.threshold_mode;
  const LayerPlanner planner(b->p);
  t.fill(b->members.size(), [&](size_t i, uint64_t* n, uint64_t* m, uint64_t* R, uint32_t* r) {
    *n = off[i + 1] - off[i];
    *r = b->members[i].r;
    planner.plan(*n, b->members[i].minbpt, m, R);
  });
  return batch_table_estimate(b->p, t);
}

// Host vectors of freed batches (layer tables, member lists, member
// records), kept for the next batches: a large batch's per-layer tables are
// megabytes, and fresh allocations of that size come back from the C library
// as new pages whose first-touch faults cost milliseconds per layer.
struct HostPool {
  std::mutex mu;
  std::vector<LayerStore> layers;  // only their host vectors are used
  std::vector<std::vector<Member>> members;
  std::vector<std::vector<burr_handle>> views;
  static constexpr size_t kMaxLayers = 8, kMaxBatches = 2;
};
HostPool g_host;

// host vectors of an earlier layer for a layer of J structures: the
// smallest kept ones that hold J entries, else the largest
void take_host(LayerStore& LS, size_t J) {
  std::lock_guard<std::mutex> lk(g_host.mu);
  if (g_host.layers.empty()) return;
  size_t pick = 0;
  for (size_t i = 1; i < g_host.layers.size(); ++i) {
    const size_t c = g_host.layers[i].ids.capacity(), cp = g_host.layers[pick].ids.capacity();
    if ((c >= J && (cp < J || c < cp)) || (cp < J && c > cp)) pick = i;
  }
  LayerStore& src = g_host.layers[pick];
  LS.t = std::move(src.t);
  LS.ids = std::move(src.ids);
  LS.bumped = std::move(src.bumped);
  g_host.layers.erase(g_host.layers.begin() + (ptrdiff_t)pick);
}

// Optional host timing of the batched build's phases (-DBURR_HOST_TIMING).
#ifdef BURR_HOST_TIMING
struct HostClock {
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char* what, uint32_t li) {
    const auto n = std::chrono::steady_clock::now();
    fprintf(stderr, "host %-12s layer %u %.3f ms\n", what, li,
            std::chrono::duration<double, std::milli>(n - t).count());
    t = n;
  }
};
#define HOST_LAP(hc, what, li) hc.lap(what, li)
#else
struct HostClock {};
#define HOST_LAP(hc, what, li)
#endif

int build_batch(burr_batch* b, const uint64_t* keys, const void* values,
                const std::vector<uint64_t>& off, Workspace* fixed_ws = nullptr) {
  HostClock hc;
  (void)hc;
  const LayerPlanner planner(b->p);
  const burr_params& p = b->p;
  hipStream_t s = b->stream;
  const uint64_t fp_salt = mix64(~p.seed);
  const uint32_t M = (uint32_t)b->members.size();
  // the workspace: the caller's (scratch builds), else one from the cache
  // or made for this build
  std::unique_ptr<WsLease> lease;
  Workspace* wsp = fixed_ws;
  if (!wsp) {
    lease.reset(new (std::nothrow) WsLease(&b->al, p, s));
    if (!lease || !lease->ws) return set_error(BURR_E_NOMEM);
    wsp = lease->ws;
  }
  Workspace& ws = *wsp;
  // the members' value bits and range split, compact: the layer tables are
  // planned from them (the Member records are 72 bytes apart)
  uint32_t rmax = 1;
  ws.h_rm.resize(M);
  for (uint32_t i = 0; i < M; ++i) {
    const Member& mb = b->members[i];
    rmax = std::max(rmax, mb.r);
    ws.h_rm[i] = (uint64_t)mb.minbpt << 32 | mb.r;
  }
  // the table arena (scratch builds bring the caller's table memory): sized
  // from the layer-0 table once it is planned, below
  auto make_arena = [&](uint64_t bytes) {
    b->arena_cap = bytes;
    b->arena = (uint8_t*)b->alloc(b->arena_cap);
    b->table_bytes = b->arena_cap;
    return b->arena != nullptr;
  };
  // events: [0] start, 7 per layer, then the final layer's start and end
  hipEvent_t* const ev = ws.events(3 + 7 * (size_t)p.layers);
  if (!ev) return set_error(BURR_E_DEVICE);
  hipEvent_t* const evfin = ev + 1 + 7 * p.layers;
  // back-substitution on the workspace's side stream when the workspace is
  // kept between builds; a per-build workspace (server, caller allocator)
  // keeps it on the build's stream rather than create a stream per build
  hipStream_t side = s;
  if (!ws.al && !ws.scr) {
    side = ws.side_stream();
    if (!side) return set_error(BURR_E_DEVICE);
  }
  auto bs_end = [&](uint32_t li) { return ev[1 + 7 * (size_t)li + 4]; };  // layer li's back-substitution done
  // A layer's back-substitution is queued once the next layer's insertion is
  // queued, and starts when the next layer's sort is done (the last BuRR
  // layer's is queued before the final layer): its grid fills the device, so
  // started right after the layer's insertion it held back the gather of the
  // bumped keys and the next sort, which are on the build's critical path;
  // beside the next insertion it overlaps the deeper layers' small launches.
  // A layer of kEarlyBacksubStructs or more structures starts it right after
  // the gather instead: the host then plans the next layer's table for
  // milliseconds, and the device would otherwise idle meanwhile.
  // Layer li+2 reuses layer li's row set and table buffer only after waiting
  // for bs_end(li), which is recorded by then.
  struct PendingBacksub {
    bool on = false;
    uint32_t li = 0;
    int set = 0;
    LayerGeom g{};
    uint64_t* W = nullptr;
    uint64_t ncode = 0;         // 2-bit codes to pack first (0: packed already)
    uint64_t* codes = nullptr;
  } pend;
  // after: an event of the build's stream the back-substitution also waits
  // for (the next layer's sort done), or null
  auto launch_backsub = [&](hipEvent_t after) -> int {
    if (!pend.on) return BURR_OK;
    pend.on = false;
    hipEvent_t* const e = ev + 1 + 7 * (size_t)pend.li;
    HIP_TRY(hipStreamWaitEvent(side, e[2], 0));
    if (after) HIP_TRY(hipStreamWaitEvent(side, after, 0));
    HIP_TRY(hipEventRecord(e[3], side));
    if (pend.ncode) HIP_TRY(pack_codes(ws.codes8[pend.set], pend.g, pend.ncode, pend.codes, side));
    HIP_TRY(back_substitute(ws.rowsC[pend.set], ws.rowsV[pend.set], pend.g, pend.W, side,
                            nullptr, side != s ? kSideBacksubWaves : 0u));
    HIP_TRY(hipEventRecord(e[4], side));
    return BURR_OK;
  };
  if (!ws.reserve_keys(off.back()) || (!ws.diag && !ws.alloc(ws.diag, 16)))
    return set_error(BURR_E_NOMEM);
  HIP_TRY(hipMemsetAsync(ws.diag, 0, 16 * 8, s));
  HIP_TRY(hipEventRecord(ev[0], s));

  // members with keys in the current layer, in key order, and their key counts
  std::vector<uint32_t>& active = ws.h_active;
  std::vector<uint64_t>& cur_n = ws.h_cur_n;
  std::vector<uint32_t>& next_active = ws.h_next_active;
  std::vector<uint64_t>& next_n = ws.h_next_n;
  {  // stored by index (push_back reloads the vector's end on every element)
    active.resize(M);
    cur_n.resize(M);
    uint32_t* const pa = active.data();
    uint64_t* const pn = cur_n.data();
    uint32_t k = 0;
    for (uint32_t i = 0; i < M; ++i) {
      const uint64_t n = off[i + 1] - off[i];
      pa[k] = i;
      pn[k] = n;
      k += n != 0 ? 1u : 0u;
    }
    active.resize(k);
    cur_n.resize(k);
  }
  next_active.reserve(active.size());
  next_n.reserve(active.size());
  const uint64_t* cur_keys = keys;
  const void* cur_vals = values;
  uint32_t cur_vbytes = value_bytes(rmax);
  bool first = true;

  uint32_t nlayers = 0;  // layers launched
  for (uint32_t li = 0; li < p.layers && !active.empty(); ++li) {
    LayerStore& LS = b->layers[li];
    // sort, solve, solved, back-substitution start and end (side stream), results, end
    hipEvent_t* const el = ev + 1 + 7 * li;
    const int set = (int)(li % kBurrSets);
    take_host(LS, active.size());
    Table t = std::move(LS.t);
    t.thr_mode = p.threshold_mode;
    const uint64_t* const rm = ws.h_rm.data();
    t.fill(active.size(), [&](size_t a, uint64_t* n, uint64_t* m, uint64_t* R, uint32_t* r) {
      const uint64_t x = rm[active[a]];
      *n = cur_n[a];
      *r = (uint32_t)x;
      planner.plan(*n, (uint32_t)(x >> 32), m, R);
    });
    HOST_LAP(hc, "fill", li);
    if (!b->arena && !make_arena(batch_table_estimate(p, t))) return set_error(BURR_E_NOMEM);
    LayerGeom g{};
    g.salt_s = mix64(p.seed ^ (2ull * li + 1ull));
    g.salt_c = mix64(p.seed ^ (2ull * li + 2ull));
    g.t_lo = p.t_lo;
    g.t_hi = p.t_hi;
    g.plain = 0;
    g.thr_mode = p.threshold_mode;
    g.cut_strategy = p.cut_strategy;
    g.cut_search = p.cut_search;
    const bool cuts = p.cut_strategy != 0;
    HOST_LAP(hc, "table", li);
    // this table buffer and row set were last read by the back-substitution
    // of layer li-kBurrSets (side stream)
    if (li >= kBurrSets) HIP_TRY(hipStreamWaitEvent(s, bs_end(li - kBurrSets), 0));
    int rc = upload_table(ws, t, g, s, set);
    if (rc != BURR_OK) return rc;
    if (!ws.reserve_slots(g.m, set) || !ws.reserve_buckets(g.nbuckets) ||
        !ws.reserve_codes(g.nbuckets, set) || !ws.reserve_structs(g.J))
      return set_error(BURR_E_NOMEM);
    LS.codes = (uint64_t*)b->alloc_table(t.code_base.back() * 8);
    LS.W = (uint64_t*)b->alloc_table(t.word_base.back() * 8);
    if (!LS.codes || !LS.W) return set_error(BURR_E_NOMEM);
    if (p.threshold_mode == 1) {
      LS.thr = (uint8_t*)b->alloc_table(t.thr_base.back());
      LS.rank = (uint32_t*)b->alloc_table(t.rank_base.back() * 4);
      LS.kcount = (uint32_t*)b->alloc_table(g.J * 4);
      if (!LS.thr || !LS.rank || !LS.kcount || !ws.reserve_pcount(t.code_base.back()))
        return set_error(BURR_E_NOMEM);
    }
    if (cuts) {
      LS.rfirst = (uint32_t*)b->alloc_table((g.nranges + 1) * 4);
      if (!LS.rfirst) return set_error(BURR_E_NOMEM);
    }
    HOST_LAP(hc, "upload", li);
    if (p.flags & BURR_FLAG_KEEP_LAYER_KEYS) {
      LS.keys = (uint64_t*)b->alloc(g.nkeys * 8);
      if (!LS.keys) return set_error(BURR_E_NOMEM);
      HIP_TRY(hipMemcpyAsync(LS.keys, cur_keys, g.nkeys * 8, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipEventRecord(el[0], s));
    // the sort also clears the insertion's results (failure flags, step
    // counter) and the last entry of the bump counts, which the scan after
    // the insertion reads
    const SortClear clear{{ws.res, ws.bump + g.nbuckets}, {ws.results_words(g.J), 1}};
    rc = run_sort(ws, cur_keys, cur_vals, cur_vbytes, first, p.filter_mode != 0, fp_salt, g, s,
                  clear);
    if (rc != BURR_OK) return rc;
    if (cuts) {  // range ends chosen from the sorted buckets (kept with the tables)
      HIP_TRY(choose_cuts(ws.rec, ws.bstart, g, LS.rfirst, s));
      g.rfirst = LS.rfirst;
    }

    SolveArgs sa{};
    sa.rec = ws.rec;
    sa.bstart = ws.bstart;
    sa.g = g;
    sa.rowsC = ws.rowsC[set];
    sa.rowsV = ws.rowsV[set];
    sa.occ = ws.occ[set];
    sa.code8 = ws.codes8[set];
    sa.bump = ws.bump;
    sa.fail = ws.fail;
    sa.steps = ws.steps;
    sa.diag = ws.diag;
    sa.nrec = (uint32_t)(g.nkeys + g.nbuckets);
    HIP_TRY(hipEventRecord(el[1], s));
    HIP_TRY(solve_layer(sa, s));
    HIP_TRY(hipEventRecord(el[2], s));
    // the previous layer's back-substitution now (side stream), this layer's
    // once the next layer's insertion is queued
    rc = launch_backsub(el[1]);
    if (rc != BURR_OK) return rc;
    pend.on = true;
    pend.li = li;
    pend.set = set;
    pend.g = g;
    pend.W = LS.W;
    pend.ncode = 0;
    pend.codes = LS.codes;
    // 2-bit codes are packed with the back-substitution (side stream; the
    // next layer's insertion writes the other code buffer); 1+-bit
    // thresholds now, as their packing shares the build stream's scan buffers
    if (p.threshold_mode == 1)
      HIP_TRY(pack_thresholds(ws.codes8[set], g, t.code_base.back(), LS.codes, ws.pcount,
                              ws.scan_tmp, LS.thr, LS.rank, LS.kcount, s));
    else
      pend.ncode = t.code_base.back();

    // per-structure bump counts (an exclusive scan of the per-bucket counts)
    // go to the host first: they are all the next layer's planning needs, so
    // the host plans and launches it while back-substitution and the gather
    // of the bumped keys still run (the next layer's keys stay grouped by
    // structure in structure order)
    HIP_TRY(scan_exclusive(ws.bump, g.nbuckets + 1, ws.scan_tmp, s));
    HIP_TRY(struct_offsets(ws.bump, g, ws.soff, s));
    HIP_TRY(hipMemcpyAsync(ws.hres, ws.res, ws.results_words(g.J) * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(el[5], s));
    HIP_TRY(gather_bumped(ws.rec, ws.bstart, ws.bump, g.nbuckets, ws.keysA, ws.valsA, s));
    HIP_TRY(hipEventRecord(el[6], s));
    if (g.J >= kEarlyBacksubStructs) {
      rc = launch_backsub(el[6]);
      if (rc != BURR_OK) return rc;
    }
    nlayers = li + 1;
    HOST_LAP(hc, "launch", li);
    HIP_TRY(hipEventSynchronize(el[5]));
    HOST_LAP(hc, "device", li);
    const uint32_t* fails = ws.hres;
    const uint32_t* soff = ws.hres + g.J;
    const uint64_t steps = *reinterpret_cast<const uint64_t*>(ws.hres + 2 * g.J + 2);
#ifdef BURR_SOLVE_STATS
    {
      const uint64_t* st = reinterpret_cast<const uint64_t*>(ws.hres + 2 * g.J + 2);
      fprintf(stderr, "solve-stats layer %u: keys %llu buckets %llu steps %llu trips %llu passes %llu "
              "active-lanes %llu\n", li, (unsigned long long)g.nkeys,
              (unsigned long long)g.nbuckets, (unsigned long long)st[0], (unsigned long long)st[1],
              (unsigned long long)st[2], (unsigned long long)st[3]);
    }
#endif
    LS.steps = steps;
    // bump counts and the members that go on (in chunks on the host workers
    // for large layers): pass 1 counts them per chunk, pass 2 lists them
    const size_t NA = active.size();
    LS.bumped.resize(NA);
    const size_t nrc = parallel_chunks(NA);
    std::vector<uint64_t> cnext(nrc + 1, 0), cfail(nrc, ~0ull);
    auto rlo = [&](size_t c) { return NA * c / nrc; };
    auto pass1 = [&](uint32_t c) {
      uint64_t k = 0;
      for (size_t a = rlo(c); a < rlo(c + 1); ++a) {
        if (fails[a] && cfail[c] == ~0ull) cfail[c] = a;
        const uint32_t nb = soff[a + 1] - soff[a];
        LS.bumped[a] = nb;
        b->members[active[a]].built = li + 1;
        k += nb != 0;
      }
      cnext[c + 1] = k;
    };
    if (nrc == 1)
      pass1(0);
    else
      Workers::get().run((uint32_t)nrc, pass1);
    for (size_t c = 0; c < nrc; ++c)
      if (cfail[c] != ~0ull) {
        fprintf(stderr, "burr: internal error %u in the insertion kernel, layer %u\n",
                fails[cfail[c]], li);
        print_diag(ws.diag);
        return set_error(BURR_E_DEVICE);
      }
    for (size_t c = 1; c <= nrc; ++c) cnext[c] += cnext[c - 1];
    next_active.resize(cnext[nrc]);
    next_n.resize(cnext[nrc]);
    auto pass2 = [&](uint32_t c) {
      uint64_t k = cnext[c];
      for (size_t a = rlo(c); a < rlo(c + 1); ++a)
        if (LS.bumped[a]) {
          next_active[k] = active[a];
          next_n[k] = LS.bumped[a];
          ++k;
        }
    };
    if (nrc == 1)
      pass2(0);
    else
      Workers::get().run((uint32_t)nrc, pass2);
    LS.ids.assign(active.begin(), active.end());
    LS.t = std::move(t);
    active.swap(next_active);
    cur_n.swap(next_n);
    HOST_LAP(hc, "records", li);
    cur_keys = ws.keysA;
    cur_vals = ws.valsA;
    cur_vbytes = 4;
    first = false;
  }

  // final plain layer of every member that still has keys
  HIP_TRY(hipEventRecord(evfin[0], s));
  std::vector<uint64_t> fin_off(active.size() + 1, 0);
  for (size_t a = 0; a < active.size(); ++a) {
    b->members[active[a]].fin.n = cur_n[a];
    fin_off[a + 1] = fin_off[a] + cur_n[a];
  }
  if ((p.flags & BURR_FLAG_KEEP_LAYER_KEYS) && !active.empty()) {
    uint64_t* kk = (uint64_t*)b->alloc(fin_off.back() * 8);
    if (!kk) return set_error(BURR_E_NOMEM);
    HIP_TRY(hipMemcpyAsync(kk, cur_keys, fin_off.back() * 8, hipMemcpyDeviceToDevice, s));
    for (size_t a = 0; a < active.size(); ++a) b->members[active[a]].fin_keys = kk + fin_off[a];
  }
  if (!b->arena && !make_arena(batch_table_estimate(b, off))) return set_error(BURR_E_NOMEM);
  // the final layer's table and rows go to a set of their own
  const int fset = kBurrSets;
  {  // the last BuRR layer's back-substitution overlaps the final layer
    const int rc = launch_backsub(nullptr);
    if (rc != BURR_OK) return rc;
  }
  if (!active.empty()) {
    std::vector<uint32_t> zero(active.size(), 0), fails;
    int rc = final_attempt(b, ws, fset, active, zero, cur_keys, cur_vals, cur_vbytes, first, fails);
    if (rc != BURR_OK) return rc;
    // rare: a member whose final system was inconsistent retries alone with
    // larger tables (Sec. 3: the last layer grows until it succeeds)
    for (size_t a = 0; a < active.size(); ++a) {
      if (!fails[a]) continue;
      const void* v = cur_vals ? (const void*)((const uint8_t*)cur_vals + fin_off[a] * cur_vbytes)
                               : nullptr;
      bool solved = false;
      for (uint32_t att = 1; att < p.final_attempts && !solved; ++att) {
        std::vector<uint32_t> one(1, active[a]), at(1, att), f1;
        rc = final_attempt(b, ws, fset, one, at, cur_keys + fin_off[a], v, cur_vbytes, first, f1);
        if (rc != BURR_OK) return rc;
        solved = f1[0] == 0;
      }
      if (!solved) return set_error(BURR_E_UNSOLVABLE);
    }
  }
  if (nlayers >= 1) HIP_TRY(hipStreamWaitEvent(s, bs_end(nlayers - 1), 0));
  HIP_TRY(hipEventRecord(evfin[1], s));
  HIP_TRY(hipStreamSynchronize(s));
  HOST_LAP(hc, "final", p.layers);
  for (uint32_t li = 0; li < nlayers; ++li) {
    const hipEvent_t* el = ev + 1 + 7 * li;
    LayerStore& LS = b->layers[li];
    LS.ms_sort = elapsed_ms(el[0], el[1]);
    LS.ms_solve = elapsed_ms(el[1], el[2]);
    LS.ms_backsub = elapsed_ms(el[3], el[4]);
    LS.ms_gather = elapsed_ms(el[2], el[6]);
    LS.kthr.clear();
    if (LS.kcount) {  // thresholds kept per structure (1+-bit)
      LS.kthr.resize(LS.t.J());
      HIP_TRY(hipMemcpy(LS.kthr.data(), LS.kcount, LS.kthr.size() * 4, hipMemcpyDeviceToHost));
    }
  }
  b->ms_final = elapsed_ms(evfin[0], evfin[1]);
  b->ms_total = elapsed_ms(ev[0], evfin[1]);
  return BURR_OK;
}

burr_batch* new_batch(const burr_params* p, uint32_t count, bool no_alloc = false) {
  burr_batch* b = new (std::nothrow) burr_batch();
  if (!b) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_host.mu);
    if (!g_host.members.empty()) {
      b->members = std::move(g_host.members.back());
      g_host.members.pop_back();
      b->members.clear();
    }
    if (!g_host.views.empty()) {
      b->views = std::move(g_host.views.back());
      g_host.views.pop_back();
      b->views.clear();
    }
  }
  b->p = *p;
  b->stream = (hipStream_t)p->stream;
  b->al.fn = p->alloc;
  b->al.ffn = p->free;
  b->al.ctx = p->alloc_ctx;
  b->al.s = b->stream;
  b->members.resize(count);
  b->views.resize(count);
  for (uint32_t i = 0; i < count; ++i) {
    b->views[i].b = b;
    b->views[i].idx = i;
  }
  b->no_alloc = no_alloc;
  int dev = 0;
  if (!no_alloc && hipGetDevice(&dev) == hipSuccess) keep_pool_memory(dev);
  return b;
}

void free_batch(burr_batch* b) {
  if (!b) return;
  for (void* q : b->owned) b->al.put(q);
  (void)hipStreamSynchronize(b->stream);
  {
    std::lock_guard<std::mutex> lk(g_host.mu);
    for (LayerStore& LS : b->layers) {
      if (LS.ids.capacity() == 0 || g_host.layers.size() >= HostPool::kMaxLayers) continue;
      LayerStore keep;
      keep.t = std::move(LS.t);
      keep.ids = std::move(LS.ids);
      keep.bumped = std::move(LS.bumped);
      g_host.layers.push_back(std::move(keep));
    }
    if (g_host.members.size() < HostPool::kMaxBatches) {
      g_host.members.push_back(std::move(b->members));
      g_host.views.push_back(std::move(b->views));
    }
  }
  delete b;
}

QueryPlan make_plan(const burr_batch* b, const Member& mb) {
  QueryPlan plan{};
  plan.r = mb.r;
  uint32_t l = 0;
  for (; l < mb.built; ++l) {
    const MemberLayer& L = layer_of(b, (uint32_t)(&mb - b->members.data()), l);
    QueryLayer& q = plan.layer[l];
    q.salt_s = mix64(b->p.seed ^ (2ull * l + 1ull));
    q.salt_c = mix64(b->p.seed ^ (2ull * l + 2ull));
    q.span = L.m - kWidth + 1;
    q.codes = b->layers[l].codes + L.code_off;
    q.W = b->layers[l].W + L.word_off;
    q.t_lo = b->p.t_lo;
    q.t_hi = b->p.t_hi;
    q.plain = 0;
    q.empty = 0;
    q.thr_mode = b->p.threshold_mode;
    if (q.thr_mode == 1) {
      q.rank = b->layers[l].rank + L.rank_off;
      q.thr = b->layers[l].thr + L.thr_off;
    }
  }
  QueryLayer& f = plan.layer[l];
  f.salt_s = mix64(b->p.seed ^ (2ull * b->p.layers + 1ull));
  f.salt_c = mix64(b->p.seed ^ (2ull * b->p.layers + 2ull));
  f.span = mb.fin.m ? mb.fin.m - kWidth + 1 : 1;
  f.codes = nullptr;
  f.W = mb.fin_W;
  f.plain = 1;
  f.empty = mb.fin.m == 0;
  plan.nlayers = l + 1;
  plan.aligned = mb.r % 2 == 0;
  for (uint32_t k = 0; k < plan.nlayers; ++k)
    if (reinterpret_cast<uintptr_t>(plan.layer[k].W) % 16 != 0) plan.aligned = 0;
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

const Member* member_of(const burr_handle* h) {
  if (!h || !h->b || h->idx >= h->b->members.size()) return nullptr;
  return &h->b->members[h->idx];
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Bound on the fraction of a layer's keys passed to the next layer, for
// memory estimates only (about 6-7 % at 0.97 slots per key and 2-bit
// thresholds; small structures see more).
constexpr double kBumpBound = 0.12;

uint64_t estimate_table(uint64_t n, uint32_t r, const burr_params& p, uint64_t* n_final) {
  uint64_t bytes = 0, cur = n;
  for (uint32_t l = 0; l < p.layers && cur > 0; ++l) {
    uint64_t m, R;
    plan_layer(p, cur, &m, &R);
    const uint64_t B = m / 64;
    if (p.threshold_mode == 1) {  // bit words, threshold bytes, rank directory, count
      const uint64_t bw = (B + 63) / 64;
      bytes += align256(bw * 8) + align256(B) + align256((bw + 7) / 8 * 4) + align256(4);
    } else {
      bytes += align256((B + 31) / 32 * 8);
    }
    if (p.cut_strategy) bytes += align256((R + 1) * 4);
    bytes += align256(B * r * 8);
    cur = (uint64_t)((double)cur * kBumpBound) + (cur > 0 ? 1 : 0);
  }
  if (n_final) *n_final = cur;
  if (cur > 0) bytes += align256(plan_final(p, cur, 0) / 64 * r * 8 + 8);
  return bytes;
}

}  // namespace

uint64_t burr_batch_device_bytes(const burr_batch* b) { return b ? b->table_bytes : 0; }

uint64_t burr_batch_table_bits(const burr_batch* b) {
  if (!b) return 0;
  uint64_t words = 0;
  for (const LayerStore& LS : b->layers) {
    if (LS.ids.empty()) continue;
    words += LS.t.code_base.back() + LS.t.word_base.back();
    for (uint32_t k : LS.kthr) words += 1 + (k + 7) / 8;  // 1+-bit thresholds
    if (!LS.kthr.empty()) words += (LS.t.rank_base.back() + 1) / 2;
  }
  for (const Member& mb : b->members) words += mb.fin.nW;
  return words * 64;
}

int burr_set_error(int code) { return set_error(code); }

uint64_t burr_workspace_bytes(uint64_t n, uint32_t rmax, uint32_t count, const burr_params* p,
                              int staged) {
  if (!p) return 0;
  uint64_t m0 = 64, R0;
  if (p->layers > 0) plan_layer(*p, n, &m0, &R0);
  uint64_t nf = 0;
  estimate_table(n, rmax, *p, &nf);
  const uint64_t mf = nf ? plan_final(*p, nf, 0) : 64;
  // every structure has at least one bucket per layer
  const uint64_t m = std::max(m0, mf) + 64ull * count;
  const uint64_t B = m / 64;
  uint64_t bytes = 0;
  bytes += 44 * std::max<uint64_t>(n, 1);              // next keys/values, sort intermediates
  bytes += 16 * (n + B + 1);                           // item stream
  bytes += 12 * m + 8 * (B + 1);                       // rows and occupancy
  bytes += 10 * (B + 1) + 4 * ((B + 2047) / 2048) * 2048 + 4 * (B + 64);  // codes (2 sets), counts, scans
  bytes += 8 * (7ull * (count + 1) + 8);               // per-structure tables
  bytes += 36ull * 64 * (mf / 64 / 4 + count);         // final-layer segments
  if (staged) bytes += (8 + (rmax <= 8 ? 1 : rmax <= 16 ? 2 : 4)) * n;
  return bytes + (1u << 20);
}

extern "C" {

int burr_estimate_build_bytes(uint64_t n, uint32_t r, const burr_params* p,
                              uint64_t* table_bytes, uint64_t* workspace_bytes) {
  if (!params_ok(p) || r < 1 || r > 32) return set_error(BURR_E_INVALID);
  if (table_bytes) *table_bytes = estimate_table(n, r, *p, nullptr);
  if (workspace_bytes) *workspace_bytes = burr_workspace_bytes(n, r, 1, p, 0);
  return BURR_OK;
}

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
  if (!params_ok(p) || r < 1 || r > 32 || (n > 0 && !keys) ||
      (!p->filter_mode && !values && n > 0) || n >= kMaxKeys) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  burr_batch* b = new_batch(p, 1);
  if (!b) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  b->members[0].n = n;
  b->members[0].r = r;
  b->views[0].owner = true;
  const std::vector<uint64_t> off = {0, n};
  const int rc = build_batch(b, keys, values, off);
  if (rc != BURR_OK) {
    free_batch(b);
    set_error(rc);
    return nullptr;
  }
  set_error(BURR_OK);
  return &b->views[0];
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Builds that allocate nothing (burr_build_noalloc)
// ---------------------------------------------------------------------------
// The build's temporary buffers come from one fixed device array per GPU.
// In host code `scratch` names a host-side stand-in, not device memory: the
// array is only ever used through the device address hipGetSymbolAddress
// returns for the current device (kept per device in g_scratch).
namespace {
constexpr uint64_t kScratchBytes = 128ull << 20;
}
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

struct ScratchState {
  std::mutex mu;                  // one scratch build per device at a time
  uint8_t* ptr = nullptr;         // device address of this device's array
  std::vector<hipEvent_t> evs;    // a build's events, created by the first call
};
ScratchState g_scratch[kMaxDevices];

// Workspace bytes the build of n keys may carve from the array: the
// workspace estimate with a quarter added for what it leaves out (the second
// row set of the deeper layers, buffers outgrown by a final-layer retry) and
// 4 MiB of fixed-size buffers.
uint64_t scratch_need(uint64_t n, uint32_t r, const burr_params* p) {
  return burr_workspace_bytes(n, r, 1, p, 0) / 4 * 5 + (4ull << 20);
}

}  // namespace

extern "C" {

burr_handle* burr_build_noalloc(const uint64_t* keys, const void* values, uint64_t n,
                                uint32_t r, const burr_params* p, void* table_mem,
                                size_t table_cap) {
  if (!params_ok(p) || r < 1 || r > 32 || (n > 0 && !keys) ||
      (!p->filter_mode && !values && n > 0) || n >= kMaxKeys || !table_mem ||
      reinterpret_cast<uintptr_t>(table_mem) % 256 != 0 ||
      (p->flags & BURR_FLAG_KEEP_LAYER_KEYS)) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  const uint64_t need = scratch_need(n, r, p);
  if (need > kScratchBytes) {
    fprintf(stderr,
            "burr_build_noalloc: %llu keys need about %llu bytes of scratch, more than its "
            "%llu bytes\n",
            (unsigned long long)n, (unsigned long long)need, (unsigned long long)kScratchBytes);
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(BURR_E_DEVICE);
    return nullptr;
  }
  ScratchState& st = g_scratch[dev];
  std::lock_guard<std::mutex> lk(st.mu);
  if (!st.ptr) {  // set-up, once per device, with the device current
    void* addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !addr) {
      fprintf(stderr, "burr_build_noalloc: hipGetSymbolAddress failed: %s\n",
              hipGetErrorString(e));
      set_error(BURR_E_DEVICE);
      return nullptr;
    }
    st.ptr = static_cast<uint8_t*>(addr);
  }
  burr_batch* b = new_batch(p, 1, true);
  if (!b) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  b->members[0].n = n;
  b->members[0].r = r;
  b->views[0].owner = true;
  b->arena = static_cast<uint8_t*>(table_mem);
  b->arena_cap = table_cap;
  b->table_bytes = table_cap;
  Workspace ws(st.ptr, kScratchBytes);
  ws.evs.swap(st.evs);  // events are made by the first call and kept
  const std::vector<uint64_t> off = {0, n};
  const int rc = build_batch(b, keys, values, off, &ws);
  (void)hipStreamSynchronize(b->stream);  // the array is free for the next call
  ws.evs.swap(st.evs);
  if (rc != BURR_OK) {
    free_batch(b);
    set_error(rc);
    return nullptr;
  }
  set_error(BURR_OK);
  return &b->views[0];
}

namespace {

// minimum buckets per range of a structure with n keys: the first class of
// the table that holds n, the last one for larger structures (classes
// ascend). A short table is counted through without branches: a binary
// search's data-dependent branches over the log-normal mix of sizes cost
// about a millisecond per 200,000 structures.
uint32_t tuned_minbpt(const burr_tune_entry* table, uint32_t entries, uint64_t n) {
  if (entries <= 32) {
    uint32_t k = 0;
    for (uint32_t e = 0; e + 1 < entries; ++e) k += table[e].n_max < n ? 1u : 0u;
    return table[k].minbpt;
  }
  uint32_t lo = 0, hi = entries - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (table[mid].n_max >= n)
      hi = mid;
    else
      lo = mid + 1;
  }
  return table[lo].minbpt;
}

// Batched build; with a table, each member's minimum buckets per range comes
// from its size class (else the parameter block's applies).
burr_batch* batch_entry(const uint64_t* keys, const void* values, const uint64_t* host_offsets,
                        const uint32_t* host_r, uint32_t count, const burr_params* p,
                        const burr_tune_entry* table, uint32_t entries) {
  if (!params_ok(p) || !host_offsets || !host_r || count == 0) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  const std::vector<uint64_t> off(host_offsets, host_offsets + count + 1);
  for (uint32_t i = 0; i < count; ++i)
    if (off[i + 1] < off[i] || host_r[i] < 1 || host_r[i] > 32) {
      set_error(BURR_E_INVALID);
      return nullptr;
    }
  const uint64_t total = off.back();
  if (off[0] != 0 || total >= kMaxKeys || (total > 0 && !keys) ||
      (!p->filter_mode && !values && total > 0)) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  burr_batch* b = new_batch(p, count);
  if (!b) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  for (uint32_t i = 0; i < count; ++i) {
    Member& mb = b->members[i];
    mb.n = off[i + 1] - off[i];
    mb.r = host_r[i];
    mb.minbpt = table ? tuned_minbpt(table, entries, mb.n) : 0u;
  }
  const int rc = build_batch(b, keys, values, off);
  if (rc != BURR_OK) {
    free_batch(b);
    set_error(rc);
    return nullptr;
  }
  set_error(BURR_OK);
  return b;
}

}  // namespace

burr_batch* burr_build_batch(const uint64_t* keys, const void* values,
                             const uint64_t* host_offsets, const uint32_t* host_r,
                             uint32_t count, const burr_params* p) {
  return batch_entry(keys, values, host_offsets, host_r, count, p, nullptr, 0);
}

burr_batch* burr_build_batch_tuned(const uint64_t* keys, const void* values,
                                   const uint64_t* host_offsets, const uint32_t* host_r,
                                   uint32_t count, const burr_params* p,
                                   const burr_tune_entry* table, uint32_t entries) {
  if (!table || entries == 0) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  for (uint32_t e = 0; e < entries; ++e)
    if (table[e].minbpt == 0 || (e > 0 && table[e].n_max <= table[e - 1].n_max)) {
      set_error(BURR_E_INVALID);
      return nullptr;
    }
  return batch_entry(keys, values, host_offsets, host_r, count, p, table, entries);
}

uint32_t burr_batch_size(const burr_batch* b) { return b ? (uint32_t)b->members.size() : 0; }

const burr_handle* burr_batch_member(const burr_batch* b, uint32_t i) {
  if (!b || i >= b->members.size()) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  return &b->views[i];
}

void burr_batch_free(burr_batch* b) { free_batch(b); }

int burr_query(const burr_handle* h, const uint64_t* keys, uint64_t n, void* out, void* stream) {
  const Member* mb = member_of(h);
  if (!mb || (n > 0 && (!keys || !out))) return set_error(BURR_E_INVALID);
  const QueryPlan plan = make_plan(h->b, *mb);
  hipStream_t s = (hipStream_t)stream;  // NULL: the null stream
  if (query(plan, keys, n, out, value_bytes(mb->r), 0, 0, s) != hipSuccess)
    return set_error(BURR_E_DEVICE);
  return BURR_OK;
}

int burr_contains(const burr_handle* h, const uint64_t* keys, uint64_t n, uint8_t* out,
                  void* stream) {
  const Member* mb = member_of(h);
  if (!mb || !h->b->p.filter_mode || (n > 0 && (!keys || !out))) return set_error(BURR_E_INVALID);
  const QueryPlan plan = make_plan(h->b, *mb);
  hipStream_t s = (hipStream_t)stream;  // NULL: the null stream
  if (query(plan, keys, n, out, 1, 1, mix64(~h->b->p.seed), s) != hipSuccess)
    return set_error(BURR_E_DEVICE);
  return BURR_OK;
}

void burr_free(burr_handle* h) {
  if (!h || !h->b) return;
  if (!h->owner) {  // a batch member: its memory belongs to the batch
    set_error(BURR_E_INVALID);
    return;
  }
  free_batch(h->b);
}

int burr_get_stats(const burr_handle* h, burr_stats* st) {
  const Member* mb = member_of(h);
  if (!mb || !st) return set_error(BURR_E_INVALID);
  const burr_batch* b = h->b;
  memset(st, 0, sizeof(*st));
  st->n = mb->n;
  st->r = mb->r;
  st->layers_built = mb->built;
  uint64_t bytes = 0;
  double ms_sort = 0, ms_solve = 0;
  for (uint32_t i = 0; i < mb->built; ++i) {
    const MemberLayer& L = layer_of(b, h->idx, i);
    const LayerStore& LS = b->layers[i];
    st->layer[i].n = L.n;
    st->layer[i].m = L.m;
    st->layer[i].nbuckets = L.m / 64;
    st->layer[i].nranges = L.R;
    st->layer[i].bumped = L.bumped;
    st->layer[i].steps = LS.steps;
    st->layer[i].ms_sort = LS.ms_sort;
    st->layer[i].ms_solve = LS.ms_solve;
    st->layer[i].ms_backsub = LS.ms_backsub;
    st->layer[i].ms_gather = LS.ms_gather;
    ms_sort += LS.ms_sort;
    ms_solve += LS.ms_solve + LS.ms_backsub;
    bytes += (L.ncode + L.nW) * 8;
    if (b->p.threshold_mode == 1) bytes += (1 + (L.K + 7) / 8) * 8 + L.nrank * 4;
  }
  st->final_n = mb->fin.n;
  st->final_m = mb->fin.m;
  st->final_attempt = mb->fin_attempt;
  st->table_bytes = bytes + mb->fin.nW * 8;
  st->ms_sort = ms_sort;
  st->ms_solve = ms_solve;
  st->ms_final = b->ms_final;
  st->ms_total = b->ms_total;
  return BURR_OK;
}

int burr_export(const burr_handle* h, void* host_buf, size_t cap, size_t* needed) {
  const Member* mb = member_of(h);
  if (!mb) return set_error(BURR_E_INVALID);
  const burr_batch* b = h->b;
  Out o{(uint8_t*)host_buf, host_buf ? cap : 0};
  const burr_params& p = b->p;
  const uint32_t mb_minbpt = mb->minbpt ? mb->minbpt : p.minbpt;
  o.put(kExportMagic, 8);
  const uint32_t hdr[20] = {kExportVersion,   kWidth,         p.bucket,       mb->r,
                            p.load_num,       p.load_den,     p.final_num,    p.final_den,
                            p.layers,         p.t_lo,         p.t_hi,         p.ranges,
                            mb_minbpt,        p.final_attempts, p.filter_mode, mb->built,
                            p.threshold_mode, p.cut_strategy, p.cut_search,   0u};
  for (uint32_t x : hdr) o.put(x, 4);
  o.put(p.seed, 8);
  o.put(mb->n, 8);
  std::vector<uint64_t> tmp;
  auto copy_words = [&](const uint64_t* d, uint64_t nw) -> bool {
    tmp.assign(nw, 0);
    if (nw && hipMemcpy(tmp.data(), d, nw * 8, hipMemcpyDeviceToHost) != hipSuccess) return false;
    return true;
  };
  const bool fill = host_buf != nullptr;
  for (uint32_t l = 0; l < mb->built; ++l) {
    const MemberLayer& L = layer_of(b, h->idx, l);
    o.put(L.n, 8);
    o.put(L.m, 8);
    o.put(L.R, 8);
    const LayerStore& LS = b->layers[l];
    const bool one_plus = p.threshold_mode == 1;
    const bool cuts = p.cut_strategy != 0;
    const uint64_t thr_words = one_plus ? 1 + (L.K + 7) / 8 : 0;  // K, then the bytes
    const uint64_t cut_words = cuts ? L.R / 2 : 0;                 // ceil((R-1)/2)
    if (fill) {
      if (!copy_words(LS.codes + L.code_off, L.ncode)) return set_error(BURR_E_DEVICE);
      o.put_words(tmp);
      if (one_plus) {
        o.put(L.K, 8);
        std::vector<uint8_t> tb(L.K);
        if (L.K && hipMemcpy(tb.data(), LS.thr + L.thr_off, L.K, hipMemcpyDeviceToHost) != hipSuccess)
          return set_error(BURR_E_DEVICE);
        for (uint8_t x : tb) o.put(x, 1);
        for (uint64_t k = L.K; k % 8; ++k) o.put(0, 1);
      }
      if (!copy_words(LS.W + L.word_off, L.nW)) return set_error(BURR_E_DEVICE);
      o.put_words(tmp);
      if (cuts) {  // last bucket of ranges 0..R-2, structure-local
        std::vector<uint32_t> rf(L.R + 1);
        if (hipMemcpy(rf.data(), LS.rfirst + L.range_off, (L.R + 1) * 4,
                      hipMemcpyDeviceToHost) != hipSuccess)
          return set_error(BURR_E_DEVICE);
        const uint64_t bb = rf[0];
        uint64_t k = 1;
        for (; k < L.R; ++k) o.put(rf[k] - bb - 1, 4);
        for (; (k - 1) % 2; ++k) o.put(0, 4);
      }
    } else {
      o.len += (L.ncode + thr_words + L.nW + cut_words) * 8;
    }
  }
  o.put(mb->fin.n, 8);
  o.put(mb->fin.m, 8);
  o.put(mb->fin_attempt, 8);
  if (fill) {
    if (!copy_words(mb->fin_W, mb->fin.nW)) return set_error(BURR_E_DEVICE);
    o.put_words(tmp);
  } else {
    o.len += mb->fin.nW * 8;
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
  uint32_t hdr[20];
  for (auto& x : hdr) x = (uint32_t)in.get(4);
  if (!in.ok || hdr[0] != kExportVersion || hdr[1] != kWidth || hdr[2] != kBucket ||
      hdr[3] < 1 || hdr[3] > 32 || hdr[15] >= kMaxLayers || hdr[19] != 0) {
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
  def.threshold_mode = hdr[16];
  def.cut_strategy = hdr[17];
  def.cut_search = hdr[18];
  def.seed = in.get(8);
  // the imported parameters must be ones a build accepts, and the layer
  // count must fit them
  if (!params_ok(&def) || hdr[15] > def.layers) {
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  burr_batch* b = new_batch(&def, 1);
  if (!b) {
    set_error(BURR_E_NOMEM);
    return nullptr;
  }
  b->views[0].owner = true;
  Member& mb = b->members[0];
  mb.r = hdr[3];
  mb.n = in.get(8);
  mb.built = hdr[15];
  // words of a layer of m slots that the rest of the buffer can hold: a
  // size read from the buffer is checked against it before any product
  // that could wrap (m / 64 words of codes or r words per 64 slots)
  auto fits = [&](uint64_t m, uint64_t per_block) -> bool {
    const uint64_t rest = (in.len - std::min<size_t>(in.off, in.len)) / 8;
    return m / 64 <= rest / per_block;
  };
  auto load_words = [&](uint64_t nw, uint64_t** dst) -> bool {
    if (in.off + nw * 8 > in.len) return false;
    *dst = (uint64_t*)b->alloc_table(nw * 8 + 8);
    if (!*dst) return false;
    if (nw && hipMemcpy(*dst, in.buf + in.off, nw * 8, hipMemcpyHostToDevice) != hipSuccess)
      return false;
    in.off += nw * 8;
    return true;
  };
  bool ok = in.ok;
  for (uint32_t l = 0; ok && l < mb.built; ++l) {
    MemberLayer L;
    L.n = in.get(8);
    L.m = in.get(8);
    L.R = in.get(8);
    if (!in.ok || L.m % 64 || L.m < 64 || !fits(L.m, mb.r) || L.R == 0 || L.R > L.m / 64) {
      ok = false;
      break;
    }
    LayerStore& LS = b->layers[l];
    LS.ids.assign(1, 0);
    LS.t = Table();
    LS.t.thr_mode = def.threshold_mode;
    LS.t.add(L.n, L.m, L.R, mb.r);
    LS.bumped.assign(1, 0);
    if (l > 0) b->layers[l - 1].bumped[0] = (uint32_t)L.n;  // keys passed on
    L.ncode = LS.t.code_base.back();
    L.nW = LS.t.word_base.back();
    const uint64_t B = L.m / 64;
    ok = load_words(L.ncode, &LS.codes);
    if (ok && def.threshold_mode == 1) {
      // bit words (already loaded), K, K bytes; the rank directory is
      // rebuilt here from the bit words
      std::vector<uint64_t> bits(L.ncode);
      memcpy(bits.data(), in.buf + in.off - L.ncode * 8, L.ncode * 8);
      const uint64_t K = in.get(8);
      uint64_t ones = 0;
      std::vector<uint32_t> rank(LS.t.rank_base.back());
      for (uint64_t w = 0; w < L.ncode; ++w) {
        if (w % 8 == 0) rank[w / 8] = (uint32_t)ones;
        ones += (uint64_t)__builtin_popcountll(bits[w]);
      }
      ok = in.ok && K == ones && K <= B && in.off + (K + 7) / 8 * 8 <= in.len;
      if (ok) {
        LS.thr = (uint8_t*)b->alloc_table(B);
        LS.rank = (uint32_t*)b->alloc_table(rank.size() * 4 + 4);
        ok = LS.thr && LS.rank &&
             (K == 0 || hipMemcpy(LS.thr, in.buf + in.off, K, hipMemcpyHostToDevice) == hipSuccess) &&
             hipMemcpy(LS.rank, rank.data(), rank.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        in.off += (K + 7) / 8 * 8;
        LS.kthr.assign(1, (uint32_t)K);
      }
    }
    ok = ok && load_words(L.nW, &LS.W);
    if (ok && def.cut_strategy != 0) {  // last bucket of ranges 0..R-2, as u32
      const uint64_t cw = L.R / 2;
      ok = in.off + cw * 8 <= in.len;
      std::vector<uint32_t> rf(L.R + 1, 0);
      for (uint64_t k = 0; ok && k + 1 < L.R; ++k) {
        uint32_t c;
        memcpy(&c, in.buf + in.off + 4 * k, 4);
        rf[k + 1] = c + 1;
        ok = rf[k + 1] > rf[k] && rf[k + 1] < B;
      }
      rf[L.R] = (uint32_t)B;
      if (ok) {
        in.off += cw * 8;
        LS.rfirst = (uint32_t*)b->alloc_table((L.R + 1) * 4);
        ok = LS.rfirst &&
             hipMemcpy(LS.rfirst, rf.data(), (L.R + 1) * 4, hipMemcpyHostToDevice) == hipSuccess;
      }
    }
  }
  if (ok) {
    mb.fin.n = in.get(8);
    mb.fin.m = in.get(8);
    mb.fin_attempt = in.get(8);
    if (mb.built > 0) b->layers[mb.built - 1].bumped[0] = (uint32_t)mb.fin.n;
    ok = in.ok && mb.fin.m % 64 == 0 && fits(mb.fin.m, mb.r) && (mb.fin.m == 0) == (mb.fin.n == 0);
    if (ok) {
      mb.fin.nW = (mb.fin.m / 64) * mb.r;
      uint64_t* w = nullptr;
      ok = load_words(mb.fin.nW, &w);
      mb.fin_W = w;
    }
  }
  if (!ok || in.off != in.len) {
    free_batch(b);
    set_error(BURR_E_INVALID);
    return nullptr;
  }
  set_error(BURR_OK);
  return &b->views[0];
}

int64_t burr_debug_layer_keys(const burr_handle* h, uint32_t layer, uint64_t* host_out,
                              uint64_t cap) {
  const Member* mb = member_of(h);
  if (!mb || layer > mb->built || !(h->b->p.flags & BURR_FLAG_KEEP_LAYER_KEYS))
    return set_error(BURR_E_INVALID);
  const uint64_t* src;
  uint64_t n;
  if (layer < mb->built) {
    const MemberLayer& L = layer_of(h->b, h->idx, layer);
    src = h->b->layers[layer].keys + L.key_off;
    n = L.n;
  } else {
    src = mb->fin_keys;
    n = mb->fin.n;
  }
  if (host_out && cap && n) {
    const uint64_t c = std::min(n, cap);
    if (hipMemcpy(host_out, src, c * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(BURR_E_DEVICE);
  }
  return (int64_t)n;
}

void burr_release_workspaces(void) {
  {
    std::lock_guard<std::mutex> lk(g_host.mu);
    g_host.layers.clear();
    g_host.layers.shrink_to_fit();
    g_host.members.clear();
    g_host.views.clear();
  }
  std::vector<Workspace*> all;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& v : g_ws_free) {
      all.insert(all.end(), v.begin(), v.end());
      v.clear();
    }
  }
  for (Workspace* w : all) delete w;
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
    case BURR_E_EVICTED: return "structure evicted or dropped";
    default: return "unknown error";
  }
}

}  // extern "C"
