// burr_server.cpp - request loop of the BuRR library (burr_server_* in
// include/burr.h): structures stay resident on the device between requests,
// and build and query requests run concurrently on the workers' HIP streams
// while their memory fits a budget.
//
// Scheduling, all under one mutex:
//   - queries run as soon as their structure is resident (in arrival order
//     among the ready ones); a query of a structure still being built waits;
//   - builds are admitted in arrival order: the head build waits until its
//     table and workspace estimate fits the budget (with EVICT_LRU, idle
//     structures are evicted, least recently used first); the builds behind
//     it that also fit are packed into the same batched build;
//   - at most workers-1 workers run builds, so queries always find a worker;
//   - a build that cannot fit even with nothing else running fails with
//     BURR_E_BUDGET instead of waiting forever.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/burr.h"
#include "burr_internal.h"
#include "burr_kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

uint32_t vbytes_of(uint32_t r) { return r <= 8 ? 1 : (r <= 16 ? 2 : 4); }

struct Req {
  uint64_t id = 0;
  uint32_t kind = 0;
  const uint64_t* keys = nullptr;
  const void* values = nullptr;
  uint64_t n = 0;
  uint32_t r = 0;
  void* out = nullptr;
  uint64_t target = 0;
  uint64_t table_est = 0;
  double t_submit = 0, t_start = 0;
};

enum StructState : uint32_t { S_BUILDING, S_RESIDENT, S_GONE };

struct StructRec {
  StructState st = S_BUILDING;
  int32_t err = BURR_OK;  // S_GONE: status of later queries
  uint64_t batch = 0;     // server batch holding it
  uint32_t member = 0;
  uint64_t pending_q = 0;
};

struct BatchRec {
  burr_batch* b = nullptr;  // null without a device
  uint64_t bytes = 0;
  uint32_t live = 0;  // members not dropped or evicted
  uint32_t busy = 0;  // running queries of its members
  uint64_t last_use = 0;
  std::vector<uint64_t> members;
};

// one unit of work handed to a worker
struct Task {
  uint32_t kind = 0;
  Req q;                    // query
  std::vector<Req> builds;  // packed builds
  uint64_t reserved = 0;    // budget bytes held while it runs
  uint64_t batch_id = 0;
  // results of a build task: batches made and the status of every request
  struct Made {
    burr_batch* b;
    uint64_t bytes;
    std::vector<size_t> reqs;  // indices into builds
  };
  std::vector<Made> made;
  std::vector<int32_t> status;
  int32_t qstatus = BURR_OK;
};

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

}  // namespace

struct burr_server {
  burr_server_config cfg{};
  burr_params p{};
  bool device = true;
  int dev = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> builds, queries;
  std::unordered_map<uint64_t, StructRec> structs;
  std::unordered_map<uint64_t, BatchRec> batches;
  std::deque<burr_completion> done;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
  uint64_t next_id = 1, next_batch = 1, use_clock = 0;
  uint64_t resident = 0, inflight = 0, peak = 0, evictions = 0, nbatches = 0, completed = 0;
  uint64_t running = 0;
  uint32_t build_workers = 0;
  bool stop = false;
  Clock::time_point t0;
};

namespace {

uint32_t max_build_workers(const burr_server* s) {
  return s->cfg.workers > 1 ? s->cfg.workers - 1 : 1;
}

void note_peak(burr_server* s) { s->peak = std::max(s->peak, s->resident + s->inflight); }

void complete(burr_server* s, const Req& r, int32_t status, uint64_t batch_id, uint64_t sid) {
  burr_completion c{};
  c.req_id = r.id;
  c.struct_id = sid;
  c.kind = r.kind;
  c.status = status;
  c.n = r.n;
  c.batch_id = batch_id;
  c.t_submit_ms = r.t_submit;
  c.t_start_ms = r.t_start;
  c.t_end_ms = ms_since(s->t0);
  s->done.push_back(c);
  ++s->completed;
}

// Releases a batch whose members are all gone and which no query uses; the
// device memory is freed by the caller after the lock is dropped.
void maybe_release(burr_server* s, uint64_t bid, std::vector<burr_batch*>& to_free) {
  auto it = s->batches.find(bid);
  if (it == s->batches.end()) return;
  if (it->second.live || it->second.busy) return;
  s->resident -= it->second.bytes;
  if (it->second.b) to_free.push_back(it->second.b);
  s->batches.erase(it);
}

void mark_gone(burr_server* s, uint64_t sid, int32_t err, std::vector<burr_batch*>& to_free) {
  auto it = s->structs.find(sid);
  if (it == s->structs.end() || it->second.st != S_RESIDENT) return;
  it->second.st = S_GONE;
  it->second.err = err;
  auto bt = s->batches.find(it->second.batch);
  if (bt != s->batches.end()) {
    --bt->second.live;
    maybe_release(s, it->second.batch, to_free);
  }
}

// Evicts idle batches, least recently used first, until `need` more bytes
// fit; returns whether they fit.
bool evict_for(burr_server* s, uint64_t need, std::vector<burr_batch*>& to_free) {
  const uint64_t budget = s->cfg.budget_bytes;
  while (s->resident + s->inflight + need > budget) {
    uint64_t best = 0, best_use = ~0ull;
    for (auto& kv : s->batches) {
      const BatchRec& br = kv.second;
      if (br.busy) continue;
      bool idle = true;
      for (uint64_t sid : br.members) {
        auto st = s->structs.find(sid);
        if (st != s->structs.end() && st->second.st == S_RESIDENT && st->second.pending_q) {
          idle = false;
          break;
        }
      }
      if (idle && br.last_use < best_use) {
        best_use = br.last_use;
        best = kv.first;
      }
    }
    if (!best) return false;
    BatchRec& br = s->batches[best];
    for (uint64_t sid : br.members) {
      auto st = s->structs.find(sid);
      if (st != s->structs.end() && st->second.st == S_RESIDENT) {
        st->second.st = S_GONE;
        st->second.err = BURR_E_EVICTED;
        --br.live;
        ++s->evictions;
      }
    }
    maybe_release(s, best, to_free);
  }
  return true;
}

uint64_t build_need(const burr_server* s, const std::vector<Req>& group) {
  uint64_t n = 0, table = 0;
  uint32_t rmax = 1;
  for (const Req& r : group) {
    n += r.n;
    table += r.table_est;
    rmax = std::max(rmax, r.r);
  }
  return table + burr_workspace_bytes(n, rmax, (uint32_t)group.size(), &s->p, group.size() > 1);
}

// Picks the next task under the lock; false if nothing can run now.
bool pick(burr_server* s, Task& t, std::vector<burr_batch*>& to_free) {
  // queries of resident structures; queries of lost structures complete now
  for (auto it = s->queries.begin(); it != s->queries.end();) {
    auto st = s->structs.find(it->target);
    if (st == s->structs.end() || st->second.st == S_GONE) {
      if (st != s->structs.end() && st->second.pending_q) --st->second.pending_q;
      it->t_start = ms_since(s->t0);
      complete(s, *it, st == s->structs.end() ? BURR_E_EVICTED : st->second.err, 0, it->target);
      it = s->queries.erase(it);
      s->cv_done.notify_all();
      continue;
    }
    if (st->second.st == S_RESIDENT) {
      t.kind = BURR_REQ_QUERY;
      t.q = *it;
      t.q.t_start = ms_since(s->t0);
      --st->second.pending_q;
      BatchRec& br = s->batches[st->second.batch];
      ++br.busy;
      br.last_use = ++s->use_clock;
      s->queries.erase(it);
      ++s->running;
      return true;
    }
    ++it;
  }
  if (s->builds.empty() || s->build_workers >= max_build_workers(s)) return false;
  const uint64_t budget = s->cfg.budget_bytes;
  std::vector<Req> group;
  uint64_t keys = 0;
  while (!s->builds.empty() && group.size() < s->cfg.max_batch) {
    const Req& r = s->builds.front();
    if (!group.empty() && keys + r.n > s->cfg.max_batch_keys) break;
    group.push_back(r);
    const uint64_t need = build_need(s, group);
    bool fits = !budget || s->resident + s->inflight + need <= budget;
    if (!fits && group.size() == 1 && (s->cfg.flags & BURR_SERVER_EVICT_LRU))
      fits = evict_for(s, need, to_free);
    if (!fits) {
      group.pop_back();
      if (group.empty() && s->running == 0) {
        // nothing running will ever free memory for it
        Req head = s->builds.front();
        s->builds.pop_front();
        head.t_start = ms_since(s->t0);
        s->structs[head.id].st = S_GONE;
        s->structs[head.id].err = BURR_E_BUDGET;
        complete(s, head, BURR_E_BUDGET, 0, head.id);
        s->cv_done.notify_all();
        return pick(s, t, to_free);
      }
      break;
    }
    keys += r.n;
    s->builds.pop_front();
  }
  if (group.empty()) return false;
  t.kind = BURR_REQ_BUILD;
  t.reserved = build_need(s, group);
  t.batch_id = s->next_batch++;
  const double now = ms_since(s->t0);
  for (Req& r : group) r.t_start = now;
  t.builds = std::move(group);
  s->inflight += t.reserved;
  note_peak(s);
  ++s->build_workers;
  ++s->running;
  return true;
}

// ---- execution (no lock held) ----

void run_query(burr_server* s, uint32_t w, Task& t, const burr_handle* h) {
  if (!s->device) {
    std::this_thread::sleep_for(std::chrono::microseconds(20 + t.q.n / 2000));
    t.qstatus = BURR_OK;
    return;
  }
  int rc = burr_query(h, t.q.keys, t.q.n, t.q.out, (void*)s->streams[w]);
  if (rc == BURR_OK && hipStreamSynchronize(s->streams[w]) != hipSuccess) rc = BURR_E_DEVICE;
  t.qstatus = rc;
}

burr_batch* build_group(burr_server* s, uint32_t w, const std::vector<Req>& g,
                        const std::vector<size_t>& idx, int* rc) {
  hipStream_t st = s->streams[w];
  burr_params p = s->p;
  p.stream = (void*)st;
  p.alloc = nullptr;
  p.free = nullptr;
  p.alloc_ctx = nullptr;
  p.flags |= BURR_FLAG_NO_WORKSPACE_CACHE;  // the budget accounts every workspace
  std::vector<uint64_t> off(idx.size() + 1, 0);
  std::vector<uint32_t> rs(idx.size());
  uint32_t rmax = 1;
  for (size_t i = 0; i < idx.size(); ++i) {
    off[i + 1] = off[i] + g[idx[i]].n;
    rs[i] = g[idx[i]].r;
    rmax = std::max(rmax, rs[i]);
  }
  burr_batch* b = nullptr;
  if (idx.size() == 1) {
    b = burr_build_batch(g[idx[0]].keys, g[idx[0]].values, off.data(), rs.data(), 1, &p);
    *rc = b ? BURR_OK : burr_last_error();
    return b;
  }
  // inputs of several requests: one contiguous copy, widened to max r
  const uint64_t n = off.back();
  const uint32_t J = (uint32_t)idx.size();
  const uint32_t vb = vbytes_of(rmax);
  const bool filt = p.filter_mode != 0;
  std::vector<uint64_t> tab(4ull * J + 1);
  for (uint32_t i = 0; i < J; ++i) {
    tab[i] = (uint64_t)(uintptr_t)g[idx[i]].keys;
    tab[J + i] = filt ? 0 : (uint64_t)(uintptr_t)g[idx[i]].values;
    tab[3ull * J + 1 + i] = vbytes_of(g[idx[i]].r);
  }
  for (uint32_t i = 0; i <= J; ++i) tab[2ull * J + i] = off[i];
  void *dk = nullptr, *dv = nullptr, *dt = nullptr;
  *rc = BURR_E_NOMEM;
  if (hipMallocAsync(&dk, std::max<uint64_t>(n, 1) * 8, st) == hipSuccess &&
      (filt || hipMallocAsync(&dv, std::max<uint64_t>(n, 1) * vb, st) == hipSuccess) &&
      hipMallocAsync(&dt, tab.size() * 8, st) == hipSuccess) {
    *rc = BURR_E_DEVICE;
    if (hipMemcpyAsync(dt, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
        burr::concat_inputs((const uint64_t*)dt, J, n, (uint64_t*)dk, dv, vb, st) ==
            hipSuccess &&
        hipStreamSynchronize(st) == hipSuccess) {
      b = burr_build_batch((const uint64_t*)dk, dv, off.data(), rs.data(), J, &p);
      *rc = b ? BURR_OK : burr_last_error();
    }
  }
  if (dk) (void)hipFreeAsync(dk, st);
  if (dv) (void)hipFreeAsync(dv, st);
  if (dt) (void)hipFreeAsync(dt, st);
  (void)hipStreamSynchronize(st);
  return b;
}

void run_build(burr_server* s, uint32_t w, Task& t) {
  const size_t G = t.builds.size();
  t.status.assign(G, BURR_OK);
  if (!s->device) {
    uint64_t n = 0, bytes = 0;
    for (const Req& r : t.builds) {
      n += r.n;
      bytes += r.table_est;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50 + n / 500));
    Task::Made m{nullptr, bytes, {}};
    for (size_t i = 0; i < G; ++i) m.reqs.push_back(i);
    t.made.push_back(m);
    return;
  }
  std::vector<size_t> all(G);
  for (size_t i = 0; i < G; ++i) all[i] = i;
  int rc = BURR_OK;
  burr_batch* b = build_group(s, w, t.builds, all, &rc);
  if (b) {
    t.made.push_back({b, burr_batch_device_bytes(b), all});
    return;
  }
  if (G == 1 || rc == BURR_E_DEVICE) {
    for (size_t i = 0; i < G; ++i) t.status[i] = rc;
    return;
  }
  // one request failed the packed build (e.g. conflicting duplicates):
  // build each alone so the others still succeed
  for (size_t i = 0; i < G; ++i) {
    std::vector<size_t> one(1, i);
    int r1 = BURR_OK;
    burr_batch* b1 = build_group(s, w, t.builds, one, &r1);
    if (b1)
      t.made.push_back({b1, burr_batch_device_bytes(b1), one});
    else
      t.status[i] = r1;
  }
}

void finish(burr_server* s, Task& t, std::vector<burr_batch*>& to_free) {
  --s->running;
  if (t.kind == BURR_REQ_QUERY) {
    auto st = s->structs.find(t.q.target);
    const uint64_t bid = st->second.batch;
    --s->batches[bid].busy;
    complete(s, t.q, t.qstatus, 0, t.q.target);
    maybe_release(s, bid, to_free);
    return;
  }
  --s->build_workers;
  s->inflight -= t.reserved;
  for (Task::Made& m : t.made) {
    const uint64_t bid = s->next_batch++;
    BatchRec br;
    br.b = m.b;
    br.bytes = m.bytes;
    br.last_use = ++s->use_clock;
    for (size_t k = 0; k < m.reqs.size(); ++k) {
      const Req& r = t.builds[m.reqs[k]];
      StructRec& sr = s->structs[r.id];
      sr.st = S_RESIDENT;
      sr.batch = bid;
      sr.member = (uint32_t)k;
      br.members.push_back(r.id);
      ++br.live;
      complete(s, r, BURR_OK, t.batch_id, r.id);
    }
    s->resident += br.bytes;
    s->batches[bid] = std::move(br);
    ++s->nbatches;
  }
  for (size_t i = 0; i < t.builds.size(); ++i) {
    if (t.status[i] == BURR_OK) continue;
    StructRec& sr = s->structs[t.builds[i].id];
    sr.st = S_GONE;
    sr.err = t.status[i];
    complete(s, t.builds[i], t.status[i], t.batch_id, t.builds[i].id);
  }
  note_peak(s);
}

void free_batches(std::vector<burr_batch*>& v) {
  for (burr_batch* b : v) burr_batch_free(b);
  v.clear();
}

void worker(burr_server* s, uint32_t w) {
  if (s->device) (void)hipSetDevice(s->dev);
  std::vector<burr_batch*> to_free;
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    Task t;
    if (pick(s, t, to_free)) {
      const burr_handle* h = nullptr;
      if (t.kind == BURR_REQ_QUERY && s->device) {
        const StructRec& sr = s->structs[t.q.target];
        h = burr_batch_member(s->batches[sr.batch].b, sr.member);
      }
      lk.unlock();
      free_batches(to_free);
      if (t.kind == BURR_REQ_QUERY)
        run_query(s, w, t, h);
      else
        run_build(s, w, t);
      lk.lock();
      finish(s, t, to_free);
      s->cv_work.notify_all();
      s->cv_done.notify_all();
      continue;
    }
    if (!to_free.empty()) {
      lk.unlock();
      free_batches(to_free);
      lk.lock();
      continue;
    }
    if (s->stop && s->builds.empty() && s->queries.empty()) break;
    s->cv_work.wait(lk);
  }
}

}  // namespace

extern "C" {

void burr_server_default_config(burr_server_config* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->abi_version = BURR_ABI_VERSION;
  c->workers = 4;
  c->budget_bytes = 0;
  c->max_batch = 1024;
  c->flags = 0;
  c->max_batch_keys = 1ull << 28;
}

burr_server* burr_server_create(const burr_server_config* c, const burr_params* p) {
  if (!c || !p || c->abi_version != BURR_ABI_VERSION || c->workers == 0 || c->workers > 64 ||
      c->max_batch == 0 || c->max_batch_keys == 0) {
    burr_set_error(BURR_E_INVALID);
    return nullptr;
  }
  uint64_t tb = 0, wb = 0;
  if (burr_estimate_build_bytes(1, 1, p, &tb, &wb) != BURR_OK) return nullptr;  // checks p
  burr_server* s = new (std::nothrow) burr_server();
  if (!s) {
    burr_set_error(BURR_E_NOMEM);
    return nullptr;
  }
  s->cfg = *c;
  s->p = *p;
  s->device = !(c->flags & BURR_SERVER_NO_DEVICE);
  s->t0 = Clock::now();
  if (s->device) {
    if (hipGetDevice(&s->dev) != hipSuccess) {
      delete s;
      burr_set_error(BURR_E_DEVICE);
      return nullptr;
    }
    s->streams.resize(c->workers, nullptr);
    for (uint32_t i = 0; i < c->workers; ++i)
      if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
        for (uint32_t k = 0; k < i; ++k) (void)hipStreamDestroy(s->streams[k]);
        delete s;
        burr_set_error(BURR_E_DEVICE);
        return nullptr;
      }
  }
  for (uint32_t i = 0; i < c->workers; ++i) s->threads.emplace_back(worker, s, i);
  return s;
}

int burr_server_submit_build(burr_server* s, const uint64_t* keys, const void* values,
                             uint64_t n, uint32_t r, uint64_t* req_id) {
  if (!s || r < 1 || r > 32 || (n > 0 && !keys) || (!s->p.filter_mode && !values && n > 0) ||
      n >= 0xf0000000ull)
    return burr_set_error(BURR_E_INVALID);
  uint64_t tb = 0, wb = 0;
  if (burr_estimate_build_bytes(n, r, &s->p, &tb, &wb) != BURR_OK)
    return burr_set_error(BURR_E_INVALID);
  if (s->cfg.budget_bytes && tb + wb > s->cfg.budget_bytes) return burr_set_error(BURR_E_BUDGET);
  std::lock_guard<std::mutex> lk(s->mu);
  Req q;
  q.id = s->next_id++;
  q.kind = BURR_REQ_BUILD;
  q.keys = keys;
  q.values = s->p.filter_mode ? nullptr : values;
  q.n = n;
  q.r = r;
  q.table_est = tb;
  q.t_submit = ms_since(s->t0);
  s->structs[q.id] = StructRec{};
  s->builds.push_back(q);
  if (req_id) *req_id = q.id;
  s->cv_work.notify_all();
  return BURR_OK;
}

int burr_server_submit_query(burr_server* s, uint64_t struct_id, const uint64_t* keys,
                             uint64_t n, void* out, uint64_t* req_id) {
  if (!s || (n > 0 && (!keys || !out))) return burr_set_error(BURR_E_INVALID);
  std::lock_guard<std::mutex> lk(s->mu);
  Req q;
  q.id = s->next_id++;
  q.kind = BURR_REQ_QUERY;
  q.keys = keys;
  q.n = n;
  q.out = out;
  q.target = struct_id;
  q.t_submit = ms_since(s->t0);
  auto it = s->structs.find(struct_id);
  if (it != s->structs.end()) ++it->second.pending_q;
  s->queries.push_back(q);
  if (req_id) *req_id = q.id;
  s->cv_work.notify_all();
  return BURR_OK;
}

int burr_server_poll(burr_server* s, burr_completion* out, uint32_t max, uint32_t* got,
                     int64_t timeout_ms) {
  if (!s || (max && !out)) return BURR_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] {
      return !s->done.empty() ||
             (s->builds.empty() && s->queries.empty() && s->running == 0);
    });
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  if (got) *got = k;
  return BURR_OK;
}

int burr_server_drain(burr_server* s) {
  if (!s) return BURR_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->builds.empty() && s->queries.empty() && s->running == 0; });
  return BURR_OK;
}

int burr_server_drop(burr_server* s, uint64_t struct_id) {
  if (!s) return BURR_E_INVALID;
  std::vector<burr_batch*> to_free;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->structs.find(struct_id);
    if (it == s->structs.end()) return BURR_E_INVALID;
    if (it->second.st == S_BUILDING) return BURR_E_INVALID;
    if (it->second.st == S_GONE) return BURR_OK;
    mark_gone(s, struct_id, BURR_E_EVICTED, to_free);
    s->cv_work.notify_all();
  }
  free_batches(to_free);
  return BURR_OK;
}

const burr_handle* burr_server_handle(burr_server* s, uint64_t struct_id) {
  if (!s || !s->device) return nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->structs.find(struct_id);
  if (it == s->structs.end() || it->second.st != S_RESIDENT) return nullptr;
  return burr_batch_member(s->batches[it->second.batch].b, it->second.member);
}

int burr_server_get_info(burr_server* s, burr_server_info* info) {
  if (!s || !info) return BURR_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  memset(info, 0, sizeof(*info));
  info->resident_bytes = s->resident;
  info->inflight_bytes = s->inflight;
  info->peak_bytes = s->peak;
  for (auto& kv : s->structs) info->resident += kv.second.st == S_RESIDENT;
  info->pending = s->builds.size() + s->queries.size();
  info->running = s->running;
  info->completed = s->completed;
  info->evictions = s->evictions;
  info->batches = s->nbatches;
  return BURR_OK;
}

void burr_server_destroy(burr_server* s) {
  if (!s) return;
  burr_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (auto& th : s->threads) th.join();
  for (auto& kv : s->batches)
    if (kv.second.b) burr_batch_free(kv.second.b);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

}  // extern "C"
