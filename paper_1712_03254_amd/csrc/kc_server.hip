// kc_server.hip - the served form of the k-mer counter: count jobs queue in
// arrival order and are admitted while the device bytes of admitted jobs fit
// the server's HBM budget and a worker is free.  Each worker thread runs one
// job at a time on a stream of its own, so admitted jobs overlap on the
// device; a finished job keeps its context (tables resident) until the client
// releases it, after which the context is pooled for a later job of the same
// configuration.  Host code only.
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
  uint64_t estimate = 0;  // estimated device bytes of a fresh context for the job
  uint64_t reserve = 0;   // bytes counted in the server's in_use for the job
  bool done = false;
};

struct Pooled {
  kc_config cfg;
  kc_ctx* ctx;
  uint64_t bytes;
  uint64_t stamp;  // last use, for least-recently-used eviction
};

kc_config normalised(const kc_config& c) {
  kc_config n = c;
  n.hbm_table_budget_bytes = 0;  // a job's tables always stay resident
  return n;
}

bool same_cfg(const kc_config& a, const kc_config& b) {
  return a.k == b.k && a.n_counters == b.n_counters && a.min_count == b.min_count &&
         a.bloom_bits_log2 == b.bloom_bits_log2 && a.bloom_hashes == b.bloom_hashes &&
         a.bloom_block_log2 == b.bloom_block_log2 && a.seed == b.seed &&
         a.partitions_log2 == b.partitions_log2 && a.table_slots == b.table_slots &&
         a.scatter_bits == b.scatter_bits && a.group_bases_log2 == b.group_bases_log2;
}

}  // namespace

struct kc_server {
  int device = 0;
  uint64_t budget = 0;
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
  bool stop = false;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  // pooled context of the job's configuration, or -1
  int match(const Job& j) const {
    for (size_t i = 0; i < pool.size(); ++i)
      if (same_cfg(pool[i].cfg, j.req.cfg)) return (int)i;
    return -1;
  }
  // the head job fits once other pooled contexts are freed
  bool admissible() const {
    if (queue.empty()) return false;
    const Job& j = jobs.at(queue.front());
    const int m = match(j);
    return in_use + j.estimate + (m >= 0 ? pool[m].bytes : 0) <= budget;
  }
};

namespace {

kc_status run_job(kc_server* S, uint32_t w, const kc_request& req, kc_ctx** ctx, kc_stats* st) {
  hipStream_t s = S->streams[w];
  kc_status r;
  if (*ctx) {
    r = kc_reset(*ctx);
  } else {
    r = kc_create(&req.cfg, S->device, ctx);
  }
  if (r != KC_OK) return r;
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
    kc_ctx* ctx = nullptr;
    uint64_t reuse = 0;
    const int m = S->match(j);
    if (m >= 0) {
      ctx = S->pool[m].ctx;
      reuse = S->pool[m].bytes;
      S->pooled -= reuse;
      S->pool.erase(S->pool.begin() + m);
    }
    // free pooled contexts, least recently used first, until the job fits
    std::vector<kc_ctx*> evict;
    while (S->in_use + S->pooled + j.estimate + reuse > S->budget && !S->pool.empty()) {
      auto lru = std::min_element(S->pool.begin(), S->pool.end(),
                                  [](const Pooled& a, const Pooled& b) { return a.stamp < b.stamp; });
      evict.push_back(lru->ctx);
      S->pooled -= lru->bytes;
      S->pool.erase(lru);
    }
    j.reserve = j.estimate + reuse;  // a reused context keeps its buffers and may grow them
    S->in_use += j.reserve;
    ++S->running;
    j.resp.admit_ms = S->now();
    j.resp.worker = w;
    const kc_request req = j.req;
    lk.unlock();
    for (kc_ctx* e : evict) kc_destroy(e);
    kc_stats st{};
    kc_status r = run_job(S, w, req, &ctx, &st);
    kc_ctx* dead = nullptr;
    if (r != KC_OK && ctx) {
      dead = ctx;
      ctx = nullptr;
    }
    const uint64_t actual = ctx ? kc::ctx_device_bytes(ctx) : 0;
    if (dead) kc_destroy(dead);
    lk.lock();
    --S->running;
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
  kc_server* S = new (std::nothrow) kc_server();
  if (!S) return KC_ERR_OUT_OF_MEMORY;
  S->device = device;
  S->budget = hbm_budget_bytes;
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

kc_status kc_server_submit(kc_server* S, const kc_request* req, uint64_t* ticket_out) {
  if (!S || !req || !ticket_out) return KC_ERR_INVALID_ARG;
  if (req->n_parts < 1 || req->n_parts > 2 || req->n_parts > req->cfg.n_counters)
    return KC_ERR_INVALID_ARG;
  Job j;
  j.req = *req;
  j.req.cfg = normalised(req->cfg);
  uint64_t bases[2] = {req->parts[0].total_bases, req->n_parts > 1 ? req->parts[1].total_bases : 0};
  j.estimate = kc::estimate_count_bytes(&j.req.cfg, bases, req->n_parts);
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
    S->pool.push_back({j.req.cfg, j.resp.ctx, j.reserve, ++S->stamp});
    S->pooled += j.reserve;
  }
  S->jobs.erase(it);
  S->cv_work.notify_all();
  return KC_OK;
}

kc_status kc_server_usage(kc_server* S, uint64_t* in_use, uint64_t* pooled, uint32_t* queued,
                          uint32_t* running) {
  if (!S) return KC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (in_use) *in_use = S->in_use;
  if (pooled) *pooled = S->pooled;
  if (queued) *queued = (uint32_t)S->queue.size();
  if (running) *running = S->running;
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
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
