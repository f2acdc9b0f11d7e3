// kc_server.hip - the served form of the k-mer counter: count jobs queue in
// arrival order and are admitted while the device bytes of admitted jobs fit
// the server's HBM budget and a worker is free.  Each worker thread runs one
// job at a time on a stream of its own, so admitted jobs overlap on the
// device; a finished job keeps its context (tables resident) until the client
// releases it, after which the context is pooled: a later job reconfigures it
// and reuses its buffers, so steady serving allocates and frees nothing.  Host
// code only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kc.h"
#include "kc_internal.h"

namespace {

struct Job {
  kc_request req{};
  kc_response resp{};
  uint64_t bases[2] = {0, 0};
  uint64_t estimate = 0;  // device bytes of a fresh context after the job
  uint64_t reserve = 0;   // bytes counted in the server's in_use for the job
  bool done = false;
};

// A released context, kept for reuse by any later job (contexts are
// reconfigured per job and keep their buffers, which only grow).
struct Pooled {
  kc_ctx* ctx;
  uint64_t bytes;  // device bytes it holds
  uint64_t stamp;  // last use, for least-recently-used eviction
};

kc_config normalised(const kc_config& c) {
  kc_config n = c;
  n.hbm_table_budget_bytes = 0;  // a job's tables always stay resident
  return n;
}

}  // namespace

struct kc_server {
  explicit kc_server(uint64_t b) : budget(b), cache(b) {}
  int device = 0;
  uint64_t budget = 0;
  // buffers of the server's contexts: freed ones are kept for later jobs (up
  // to the budget again, beyond the admitted bytes) rather than returned to
  // the runtime while serving
  kc::BlockCache cache;
  uint32_t workers = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;  // tickets waiting for admission, in arrival order
  std::unordered_map<uint64_t, Job> jobs;
  uint64_t next_ticket = 1, stamp = 0;
  uint64_t in_use = 0;  // bytes of admitted, unreleased jobs
  std::vector<Pooled> pool;
  uint64_t pooled = 0;  // bytes of pooled contexts
  uint32_t running = 0;
  uint64_t inflight = 0;      // bases of the requests on workers now
  uint64_t max_inflight = 0;  // admission cap on inflight (0: none)
  uint64_t created = 0, reused = 0, grown = 0, evicted = 0;
  bool stop = false;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  // Pool entries as the admission rule sees them: each pooled context's
  // bytes now and after job j (0 when it cannot take it), and its last use.
  std::vector<kc_admit_pooled> pool_view(const Job& j) const {
    std::vector<kc_admit_pooled> v(pool.size());
    for (size_t i = 0; i < pool.size(); ++i)
      v[i] = {pool[i].bytes, kc::bytes_after(pool[i].ctx, &j.req.cfg, j.bases, j.req.n_parts),
              pool[i].stamp};
    return v;
  }
  kc_admit_state admit_state() const {
    kc_admit_state a{};
    a.budget = budget;
    a.in_use = in_use;
    a.pooled = pooled;
    a.max_inflight = max_inflight;
    a.inflight = inflight;
    a.running = running;
    return a;
  }
  // The head of the queue may start now (kc_server_plan_admission).
  bool admissible() const {
    if (queue.empty()) return false;
    const Job& j = jobs.at(queue.front());
    const std::vector<kc_admit_pooled> v = pool_view(j);
    const kc_admit_state a = admit_state();
    std::vector<uint32_t> ev(v.size() + 1);
    uint32_t admit = 0, nev = 0;
    int32_t choice = -1;
    uint64_t reserve = 0;
    return kc_server_plan_admission(&a, v.data(), (uint32_t)v.size(), j.bases[0] + j.bases[1],
                                    j.estimate, &admit, &choice, &reserve, ev.data(),
                                    &nev) == KC_OK &&
           admit;
  }
};

namespace {

kc_status run_job(kc_server* S, uint32_t w, const kc_request& req, kc_ctx** ctx, kc_stats* st) {
  hipStream_t s = S->streams[w];
  kc::AllocStream alloc_on(s);  // creation and growth allocate in order on the worker's stream
  kc::UseCache from(&S->cache);
  kc_status r;
  if (*ctx) {
    r = kc_reset(*ctx);
    if (r == KC_OK) r = kc::reconfigure(*ctx, &req.cfg, s);
  } else {
    r = kc_create(&req.cfg, S->device, ctx);
  }
  if (r != KC_OK) return r;
  // the reads may still be written on the caller's stream
  if (req.ready_event && hipStreamWaitEvent(s, static_cast<hipEvent_t>(req.ready_event), 0) != hipSuccess) {
    (void)hipGetLastError();
    return KC_ERR_DEVICE;
  }
  for (uint32_t p = 0; p < req.n_parts; ++p) {
    const kc_chunk& c = req.parts[p];
    r = kc_insert_reads(*ctx, c.bases_dev, c.offsets_dev, c.n_reads, c.total_bases, p, s);
    if (r != KC_OK) return r;
  }
  return kc_finalize(*ctx, s, st);
}

void worker_main(kc_server* S, uint32_t w) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_work.wait(lk, [&] { return S->stop || S->admissible(); });
    if (S->stop) break;
    const uint64_t ticket = S->queue.front();
    S->queue.pop_front();
    Job& j = S->jobs.at(ticket);  // element references survive rehashing
    const std::vector<kc_admit_pooled> view = S->pool_view(j);
    const kc_admit_state as = S->admit_state();
    std::vector<uint32_t> ev(view.size() + 1);
    uint32_t admit = 0, nev = 0;
    int32_t m = -1;
    uint64_t reserve = 0;
    (void)kc_server_plan_admission(&as, view.data(), (uint32_t)view.size(),
                                   j.bases[0] + j.bases[1], j.estimate, &admit, &m, &reserve,
                                   ev.data(), &nev);
    kc_ctx* ctx = nullptr;
    std::vector<kc_ctx*> evict;
    std::vector<char> gone(S->pool.size(), 0);
    for (uint32_t e = 0; e < nev; ++e) {
      evict.push_back(S->pool[ev[e]].ctx);
      S->pooled -= S->pool[ev[e]].bytes;
      gone[ev[e]] = 1;
      ++S->evicted;
    }
    if (m >= 0) {
      ctx = S->pool[m].ctx;
      ++(reserve > S->pool[m].bytes ? S->grown : S->reused);
      S->pooled -= S->pool[m].bytes;
      gone[m] = 1;
    } else {
      ++S->created;
    }
    {
      std::vector<Pooled> keep;
      for (size_t i = 0; i < S->pool.size(); ++i)
        if (!gone[i]) keep.push_back(S->pool[i]);
      S->pool.swap(keep);
    }
    j.reserve = reserve;  // the context's size after the job
    S->in_use += j.reserve;
    ++S->running;
    S->inflight += j.bases[0] + j.bases[1];
    j.resp.admit_ms = S->now();
    j.resp.worker = w;
    const kc_request req = j.req;
    lk.unlock();
    {
      kc::AllocStream alloc_on(S->streams[w]);  // evicted contexts are idle: free in stream order
      for (kc_ctx* e : evict) kc_destroy(e);
    }
    kc_stats st{};
    kc_status r = run_job(S, w, req, &ctx, &st);
    kc_ctx* dead = nullptr;
    if (r != KC_OK && ctx) {
      dead = ctx;
      ctx = nullptr;
    }
    const uint64_t actual = ctx ? kc::ctx_device_bytes(ctx) : 0;
    if (dead) {
      kc::AllocStream alloc_on(S->streams[w]);
      kc_destroy(dead);
    }
    lk.lock();
    --S->running;
    S->inflight -= j.bases[0] + j.bases[1];
    j.resp.status = r;
    j.resp.stats = st;
    j.resp.ctx = ctx;
    j.resp.done_ms = S->now();
    S->in_use = S->in_use - j.reserve + actual;
    j.reserve = actual;
    j.resp.footprint_bytes = actual;
    j.done = true;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

kc_status kc_server_create(int device, uint64_t hbm_budget_bytes, uint32_t workers,
                           kc_server** out) {
  if (!out || hbm_budget_bytes == 0 || workers < 1 || workers > 16) return KC_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return KC_ERR_INVALID_ARG;
  }
  if (hipSetDevice(device) != hipSuccess) return KC_ERR_DEVICE;
  kc_server* S = new (std::nothrow) kc_server(hbm_budget_bytes);
  if (!S) return KC_ERR_OUT_OF_MEMORY;
  S->device = device;
  S->workers = workers;
  S->t0 = std::chrono::steady_clock::now();
  for (uint32_t w = 0; w < workers; ++w) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      kc_server_destroy(S);
      return KC_ERR_DEVICE;
    }
    S->streams.push_back(s);
  }
  for (uint32_t w = 0; w < workers; ++w) S->threads.emplace_back(worker_main, S, w);
  *out = S;
  return KC_OK;
}

kc_status kc_server_plan_admission(const kc_admit_state* st, const kc_admit_pooled* pool,
                                   uint32_t n_pool, uint64_t job_bases, uint64_t estimate,
                                   uint32_t* admit, int32_t* choice, uint64_t* reserve,
                                   uint32_t* evict, uint32_t* n_evict) {
  if (!st || (n_pool && !pool) || !admit || !choice || !reserve || !n_evict || (n_pool && !evict))
    return KC_ERR_INVALID_ARG;
  uint64_t sum = 0;
  for (uint32_t i = 0; i < n_pool; ++i) sum += pool[i].bytes;
  if (sum != st->pooled) return KC_ERR_INVALID_ARG;
  *admit = 0;
  *choice = -1;
  *reserve = 0;
  *n_evict = 0;
  // with a cap, a request starts only alone or within the cap beside the running ones
  if (st->max_inflight && st->running && st->inflight + job_bases > st->max_inflight)
    return KC_OK;
  const uint64_t budget = st->budget, in_use = st->in_use;
  int fit = -2, grow = -2;
  uint64_t fit_bytes = ~0ull, grow_by = ~0ull, grow_after = 0;
  for (uint32_t i = 0; i < n_pool; ++i) {
    const uint64_t after = pool[i].after;
    if (after == 0 || in_use + after > budget) continue;
    if (after <= pool[i].bytes) {
      if (pool[i].bytes < fit_bytes) {
        fit = (int)i;
        fit_bytes = pool[i].bytes;
      }
    } else if (after - pool[i].bytes < grow_by) {
      grow = (int)i;
      grow_by = after - pool[i].bytes;
      grow_after = after;
    }
  }
  int c = -2;
  uint64_t r = 0;
  if (fit >= 0) {
    c = fit;
    r = fit_bytes;
  } else if (in_use + st->pooled + estimate <= budget) {
    c = -1;
    r = estimate;
  } else if (grow >= 0 && grow_by <= estimate) {
    c = grow;
    r = grow_after;
  } else if (in_use + estimate <= budget) {
    c = -1;
    r = estimate;
  } else if (grow >= 0) {
    c = grow;
    r = grow_after;
  }
  if (c == -2) return KC_OK;  // nothing fits yet: wait for releases
  *admit = 1;
  *choice = c;
  *reserve = r;
  // free pooled contexts, least recently used first, until everything fits
  uint64_t pooled = st->pooled - (c >= 0 ? pool[c].bytes : 0);
  std::vector<char> taken(n_pool, 0);
  if (c >= 0) taken[c] = 1;
  while (in_use + r + pooled > budget) {
    int lru = -1;
    for (uint32_t i = 0; i < n_pool; ++i)
      if (!taken[i] && (lru < 0 || pool[i].stamp < pool[lru].stamp)) lru = (int)i;
    if (lru < 0) break;
    taken[lru] = 1;
    evict[(*n_evict)++] = (uint32_t)lru;
    pooled -= pool[lru].bytes;
  }
  return KC_OK;
}

kc_status kc_server_set_overlap(kc_server* S, uint64_t max_inflight_bases) {
  if (!S) return KC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  S->max_inflight = max_inflight_bases;
  S->cv_work.notify_all();
  return KC_OK;
}

kc_status kc_server_submit(kc_server* S, const kc_request* req, uint64_t* ticket_out) {
  if (!S || !req || !ticket_out) return KC_ERR_INVALID_ARG;
  if (req->n_parts < 1 || req->n_parts > 2 || req->n_parts > req->cfg.n_counters ||
      req->reserved_ != 0)
    return KC_ERR_INVALID_ARG;
  Job j;
  j.req = *req;
  j.req.cfg = normalised(req->cfg);
  j.bases[0] = req->parts[0].total_bases;
  j.bases[1] = req->n_parts > 1 ? req->parts[1].total_bases : 0;
  j.estimate = kc::estimate_count_bytes(&j.req.cfg, j.bases, req->n_parts);
  if (j.estimate == 0) return KC_ERR_INVALID_ARG;  // configuration rejected
  std::lock_guard<std::mutex> lk(S->mu);
  const uint64_t t = S->next_ticket++;
  j.resp.submit_ms = S->now();
  if (j.estimate > S->budget) {
    j.resp.status = KC_ERR_OVER_BUDGET;
    j.resp.admit_ms = j.resp.done_ms = j.resp.submit_ms;
    j.resp.footprint_bytes = j.estimate;
    j.done = true;
    S->jobs.emplace(t, j);
  } else {
    S->jobs.emplace(t, j);
    S->queue.push_back(t);
    S->cv_work.notify_all();
  }
  *ticket_out = t;
  return KC_OK;
}

kc_status kc_server_wait(kc_server* S, uint64_t ticket, kc_response* out) {
  if (!S) return KC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return KC_ERR_INVALID_ARG;
  S->cv_done.wait(lk, [&] { return it->second.done || S->stop; });
  if (!it->second.done) return KC_ERR_BAD_STATE;
  if (out) *out = it->second.resp;
  return KC_OK;
}

kc_status kc_server_release(kc_server* S, uint64_t ticket) {
  if (!S) return KC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return KC_ERR_INVALID_ARG;
  if (!it->second.done) return KC_ERR_BAD_STATE;
  Job& j = it->second;
  S->in_use -= j.reserve;
  if (j.resp.ctx) {
    S->pool.push_back({j.resp.ctx, j.reserve, ++S->stamp});
    S->pooled += j.reserve;
  }
  S->jobs.erase(it);
  S->cv_work.notify_all();
  return KC_OK;
}

kc_status kc_server_usage(kc_server* S, kc_server_stats* out) {
  if (!S || !out) return KC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  out->in_use_bytes = S->in_use;
  out->pooled_bytes = S->pooled;
  out->queued = (uint32_t)S->queue.size();
  out->running = S->running;
  out->pooled_contexts = (uint32_t)S->pool.size();
  out->reserved_ = 0;
  out->created = S->created;
  out->reused = S->reused;
  out->grown = S->grown;
  out->evicted = S->evicted;
  S->cache.usage(&out->cached_bytes, &out->device_allocs, &out->device_frees);
  return KC_OK;
}

void kc_server_destroy(kc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->queue.clear();
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  for (std::thread& t : S->threads) t.join();
  (void)hipSetDevice(S->device);
  for (auto& kv : S->jobs)
    if (kv.second.resp.ctx) kc_destroy(kv.second.resp.ctx);
  for (Pooled& p : S->pool) kc_destroy(p.ctx);
  (void)hipDeviceSynchronize();
  S->cache.drain();
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
