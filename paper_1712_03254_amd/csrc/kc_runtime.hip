// kc_runtime.hip - host runtime of the k-mer counter: the C ABI of kc.h.
//
// One context = one counting job on one GPU.  The runtime owns the Bloom
// levels, the per-call key segments (pass-1 output), the per-partition tables
// and the spill directory, and enqueues the kernels of kc_kernels.hip on the
// caller's stream.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "kc.h"
#include "kc_internal.h"

using namespace kc;

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t ceil_log2(uint64_t v) {
  uint32_t r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

}  // namespace

namespace kc {

// Allocation stream of the calling thread: set by the entry points that run
// on a stream.  There, buffers are allocated and freed in stream order
// (hipMallocAsync / hipFreeAsync on the device's default pool, which keeps
// freed memory for reuse), so a growing or freed buffer does not wait for the
// whole device; elsewhere hipMalloc / hipFree.
thread_local bool t_async = false;
thread_local hipStream_t t_stream = nullptr;

AllocStream::AllocStream(hipStream_t s) : prev(t_stream), prev_on(t_async) {
  t_stream = s;
  t_async = true;
}
AllocStream::~AllocStream() {
  t_stream = prev;
  t_async = prev_on;
}

thread_local BlockCache* t_cache = nullptr;
UseCache::UseCache(BlockCache* k) : prev(t_cache) { t_cache = k; }
UseCache::~UseCache() { t_cache = prev; }

uint64_t cache_round(uint64_t n) {
  if (n <= 16384) return std::max<uint64_t>(4096, (n + 4095) & ~4095ull);
  const uint64_t step = 1ull << (63 - __builtin_clzll(n) - 2);
  return (n + step - 1) & ~(step - 1);
}

hipError_t BlockCache::alloc(uint64_t want, hipStream_t s, void** p, uint64_t* got) {
  const uint64_t r = cache_round(want);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.lower_bound(r);
    if (it != free_.end() && it->first <= 2 * r) {
      const Block b = it->second;
      if (b.ev && b.s != s) {
        const hipError_t e = hipStreamWaitEvent(s, b.ev, 0);
        if (e != hipSuccess) return e;
      }
      if (b.ev) events_.push_back(b.ev);  // the wait is enqueued: the event may be recorded again
      *p = b.p;
      *got = it->first;
      cached_ -= it->first;
      free_.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, r);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(mu_);
      while (!free_.empty()) free_largest();
    }
    e = hipMalloc(p, r);
  }
  if (e == hipSuccess) {
    *got = r;
    std::lock_guard<std::mutex> lk(mu_);
    ++allocs_;
  }
  return e;
}

void BlockCache::give_back(void* p, uint64_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu_);
  hipEvent_t ev = nullptr;
  if (!events_.empty()) {
    ev = events_.back();
    events_.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    ev = nullptr;
  }
  if (!ev || hipEventRecord(ev, s) != hipSuccess) {
    // no event: wait here for the work queued on s, so no later user has to
    if (ev) events_.push_back(ev);
    ev = nullptr;
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
  }
  free_.emplace(bytes, Block{p, s, ev});
  cached_ += bytes;
  while (cached_ > limit_ && !free_.empty()) free_largest();
}

void BlockCache::free_largest() {
  auto it = std::prev(free_.end());
  if (it->second.ev) {
    (void)hipEventSynchronize(it->second.ev);
    events_.push_back(it->second.ev);
  }
  (void)hipFree(it->second.p);
  ++frees_;
  cached_ -= it->first;
  free_.erase(it);
}

void BlockCache::drain() {
  std::lock_guard<std::mutex> lk(mu_);
  while (!free_.empty()) free_largest();
  for (hipEvent_t e : events_) (void)hipEventDestroy(e);
  events_.clear();
}

void keep_pool_memory(int device) {
  static std::once_flag once[64];
  if (device < 0 || device >= 64) return;
  std::call_once(once[device], [device] {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t keep = ~0ull;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
  });
}

}  // namespace kc

namespace {

using kc::t_async;
using kc::t_stream;

constexpr size_t kPinnedBytes = 4096;  // a context's pinned staging area for small readbacks

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool async = false;               // came from hipMallocAsync
  kc::BlockCache* cache = nullptr;  // came from (and goes back to) a server's block cache
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
  void release() {
    if (p) {
      if (cache)
        cache->give_back(p, bytes, t_async ? t_stream : nullptr);
      else if (async && t_async)
        (void)hipFreeAsync(p, t_stream);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    async = false;
    cache = nullptr;
  }
  hipError_t ensure(size_t want) {
    if (want == 0) want = 8;
    if (bytes >= want) return hipSuccess;
    release();
    if (kc::t_cache) {
      uint64_t got = 0;
      const hipError_t e = kc::t_cache->alloc(want, t_async ? t_stream : nullptr, &p, &got);
      if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return e;
      }
      bytes = got;
      cache = kc::t_cache;
      return hipSuccess;
    }
    hipError_t e = t_async ? hipMallocAsync(&p, want, t_stream) : hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return e;
    }
    bytes = want;
    async = t_async;
    return hipSuccess;
  }
};

// Releases call-local device buffers when the call returns (DevBuf itself has
// no destructor: contexts and segments hold theirs by value and copy them).
struct ReleaseOnExit {
  std::vector<DevBuf*> bufs;
  ReleaseOnExit(std::initializer_list<DevBuf*> l) : bufs(l) {}
  ~ReleaseOnExit() {
    for (DevBuf* b : bufs) b->release();
  }
};

struct Segment {
  DevBuf keys, bucket_off, tile_first, meta2;
  uint64_t n = 0;
  uint32_t counter = 0;
  void release() {
    keys.release();
    bucket_off.release();
    tile_first.release();
    meta2.release();
  }
};

// One spilled partition: its table (keys and counts in slot order) in pinned
// host memory.  Mirrors the paper's swap metadata record (partition,
// stale flag, byte offset, item count; Sec. III-D).
struct SpillRec {
  uint32_t partition = 0;
  bool stale = false;
  uint64_t host_offset = 0;  // first slot of the table in the spill pool
  uint64_t entries = 0;      // keys with a count at or above min_count
};

enum State { CREATED = 0, INSERTING = 1, FINALIZED = 2 };

// kc_count_batch: consecutive chunks packed side by side into one key segment.
struct BatchGroup {
  uint32_t c0 = 0, nc = 0;  // chunk range
  uint64_t nwords = 0;      // packed words of the group stream
  uint64_t nslots = 0;      // read slots (sum of n_reads + 1)
  uint64_t ntiles = 0, nhist = 0, tiles2 = 0;
  DevBuf cdesc;             // ChunkDesc[nc]
  Segment seg;              // key segment; upper-bound sized (graph replays reuse it)
};

// The captured graph of one chunk list and everything its nodes point to.
struct BatchPlan {
  std::vector<kc_chunk> chunks;
  uint32_t counter = 0;
  std::vector<BatchGroup> groups;
  DevBuf counts;  // keys per group (u64), written by the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    for (BatchGroup& g : groups) {
      g.cdesc.release();
      g.seg.release();
    }
    groups.clear();
    chunks.clear();
    counts.release();
  }
};

thread_local std::string g_create_error;

}  // namespace

struct kc_ctx {
  kc_config cfg{};
  int device = 0;
  State state = CREATED;
  std::string err;

  // derived layout
  HashCfg hc{};
  uint32_t s_log2 = 0, p_log2 = 0, cap = 0, a1 = 0, a2 = 0, upb_log2 = 0, bsub_log2 = 0;
  uint32_t t2_log2 = 13;  // keys per second-level shuffle tile (log2)
  uint32_t nbw = 1, l2w = 2, slot_bytes = 12;
  size_t count_lds = 0, tally_lds = 0;
  uint64_t bloom_words64 = 1;

  DevBuf b1, b2;
  DevBuf dstat;   // kNst u64 stats, then ovf stats scratch
  DevBuf derr;    // u32 error flags
  DevBuf packed, flags, hist1, lstart1, off1, parts, keys1, tile_desc;
  DevBuf segdesc;
  DevBuf tkeys, tcounts, pstats, pstats2, pstats_ovf;
  DevBuf slot_of, slot_live;  // partition -> HBM table slot; slot -> holds a live table
  DevBuf okeys, ocounts, ovf_used;
  DevBuf qrows, qkeys, qcount;
  uint32_t pool_slots = 0;            // partition tables held in HBM (the budget's share)
  std::vector<uint32_t> slot_of_h;    // host mirror of slot_of
  // slot_of[u] = u - slot_first for u >= slot_first and kNoSlot below it, as
  // finalize, restore and the batched form lay tables out; -1 once a single
  // partition has been spilled (lookups then read slot_of)
  int64_t slot_first = -1;
  hipStream_t copy_stream = nullptr;  // device-to-host spill copies
  hipEvent_t ev_tally[2] = {nullptr, nullptr}, ev_copy[2] = {nullptr, nullptr};
  uint32_t ovf_log2 = 12;
  std::vector<Segment> segs, spare_segs;
  bool segs_borrowed = false;  // segs are views of the batch plan's segments
  BatchPlan batch;
  hipStream_t capture_stream = nullptr;
  hipEvent_t insert_done = nullptr;
  bool insert_done_valid = false;

  uint64_t* pinned = nullptr;  // small pinned staging area (kPinnedBytes)

  // spill directory + pool (pinned host).  The pool holds whole partition
  // tables in their HBM layout (cap slots each), so host lookups probe them
  // with the table's own slot function.
  std::vector<SpillRec> spill_dir;
  std::vector<int32_t> spill_of;  // partition -> index into spill_dir or -1
  uint64_t* spill_keys = nullptr;
  uint32_t* spill_counts = nullptr;
  uint64_t spill_cap = 0, spill_used = 0;  // in tables

  kc_stats st{};

  // timers: pending (start, stop, stage) triples
  struct Timer {
    hipEvent_t a, b;
    int id;
  };
  std::vector<Timer> pending;
  std::vector<hipEvent_t> event_pool;
};

namespace {

kc_status fail(kc_ctx* c, kc_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

kc_status hip_fail(kc_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return fail(c, KC_ERR_OUT_OF_MEMORY, m);
  }
  return fail(c, KC_ERR_DEVICE, m);
}

#define KC_HIP(ctx, expr, what)                       \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

hipEvent_t take_event(kc_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  // Timer events only time the stream (completion queries, elapsed times);
  // results reach the host through copies and stream synchronisation, so the
  // system-scope fence a default event record carries is not needed.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

struct StageTimer {
  kc_ctx* c;
  hipStream_t s;
  hipEvent_t a = nullptr;
  int id;
  StageTimer(kc_ctx* c_, hipStream_t s_, int id_, bool on = true) : c(c_), s(s_), id(id_) {
    a = on ? take_event(c) : nullptr;
    if (a) (void)hipEventRecord(a, s);
  }
  void stop() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->pending.push_back({a, b, id});
    a = nullptr;
  }
};

// Folds finished timer pairs into st.kernel_ms (call after a synchronisation).
void resolve_timers(kc_ctx* c) {
  std::vector<kc_ctx::Timer> keep;
  for (auto& t : c->pending) {
    if (hipEventQuery(t.b) != hipSuccess) {
      (void)hipGetLastError();
      keep.push_back(t);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->st.kernel_ms[t.id] += ms;
      c->st.kernel_launches[t.id] += 1;
    } else {
      (void)hipGetLastError();
    }
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->pending.swap(keep);
}

kc_status validate(const kc_config* cfg, std::string* why) {
  char buf[256];
  auto bad = [&](const char* m) {
    *why = m;
    return KC_ERR_INVALID_ARG;
  };
  if (!cfg) return bad("config is NULL");
  if (cfg->k < 1 || cfg->k > 31) return bad("k must be in 1..31");
  if (cfg->n_counters < 1 || cfg->n_counters > 2) return bad("n_counters must be 1 or 2");
  if (cfg->min_count < 2) return bad("min_count must be >= 2");
  if (cfg->bloom_hashes < 1 || cfg->bloom_hashes > 8) return bad("bloom_hashes must be in 1..8");
  if (cfg->bloom_block_log2 < 1 || cfg->bloom_block_log2 > 19)
    return bad("bloom_block_log2 must be in 1..19");
  if (cfg->bloom_bits_log2 < cfg->bloom_block_log2 || cfg->bloom_bits_log2 > 40)
    return bad("bloom_bits_log2 must be in bloom_block_log2..40");
  if (cfg->bloom_bits_log2 - cfg->bloom_block_log2 > kMaxPartLog2)
    return bad("more than 2^21 Bloom blocks (raise bloom_block_log2)");
  if (cfg->partitions_log2 > kMaxPartLog2) return bad("partitions_log2 must be <= 21");
  if (cfg->group_bases_log2 != 0 && (cfg->group_bases_log2 < 10 || cfg->group_bases_log2 > 32))
    return bad("group_bases_log2 must be 0 or in 10..32");
  if (cfg->shuffle_tile_log2 != 0 &&
      (cfg->shuffle_tile_log2 < kT2MinLog2 || (1u << cfg->shuffle_tile_log2) > (uint32_t)kT2))
    return bad("shuffle_tile_log2 must be 0 or in 10..13");
  if (cfg->reserved_ != 0) return bad("reserved_ must be 0");
  if (cfg->scatter_bits > kMaxA1) {
    snprintf(buf, sizeof buf, "scatter_bits must be <= %d", kMaxA1);
    *why = buf;
    return KC_ERR_INVALID_ARG;
  }
  return KC_OK;
}

kc_status derive(kc_ctx* c) {
  const kc_config& f = c->cfg;
  HashCfg& hc = c->hc;
  for (uint32_t i = 0; i <= f.bloom_hashes; ++i) hc.salt[i] = host_mix64(f.seed + (uint64_t)(i + 1) * kGamma);
  hc.k = f.k;
  hc.h = f.bloom_hashes;
  hc.bl = f.bloom_block_log2;
  hc.nc = f.n_counters;
  hc.min_count = f.min_count;
  c->s_log2 = f.bloom_bits_log2 - f.bloom_block_log2;
  c->p_log2 = std::max<uint32_t>(std::max<uint32_t>(f.partitions_log2, c->s_log2), 2);
  if (c->p_log2 > (uint32_t)kMaxPartLog2)
    return fail(c, KC_ERR_INVALID_ARG, "more than 2^21 partitions");
  c->upb_log2 = c->p_log2 - c->s_log2;
  hc.s_log2 = c->s_log2;
  hc.p_log2 = c->p_log2;
  c->nbw = f.bloom_block_log2 >= 5 ? (1u << (f.bloom_block_log2 - 5)) : 1u;
  c->slot_bytes = 8 + 4 * f.n_counters;
  // k_bloom: the block's two levels in LDS.  k_tally: a partition table (cap
  // slots) plus per-wave miss queues; by default three workgroups fit a CU,
  // with kLdsSlack bytes to spare each (a table sized to the last byte of a
  // third of the LDS measured as if only two fitted).
  const uint32_t cap_max = (uint32_t)(((size_t)kLdsMax - kQueueBytes) / c->slot_bytes / 64 * 64);
  const uint32_t cap_def =
      (uint32_t)(((size_t)kLdsMax / 3 - kLdsSlack - kQueueBytes) / c->slot_bytes / 64 * 64);
  if (f.table_slots) {
    const uint32_t want = f.table_slots / 64 * 64;
    if (want < 64 || want > cap_max)
      return fail(c, KC_ERR_INVALID_ARG,
                  "table_slots must be in 64.." + std::to_string(cap_max));
    c->cap = want;
  } else {
    c->cap = cap_def;
  }
  // two shuffle levels: a1 bits in the first, the rest in the second
  c->a1 = f.scatter_bits ? std::min<uint32_t>(f.scatter_bits, c->p_log2 - 1)
                         : std::min<uint32_t>(c->p_log2 / 2, kMaxA1);
  c->a2 = c->p_log2 - c->a1;
  c->t2_log2 = f.shuffle_tile_log2 ? f.shuffle_tile_log2 : 13u;
  if (c->a1 < 1 || c->a1 > (uint32_t)kMaxA1 || c->a2 < 1 || c->a2 > (uint32_t)kMaxA2)
    return fail(c, KC_ERR_INVALID_ARG, "partition count needs a wider shuffle (set scatter_bits)");
  // k_bloom takes up to four Bloom blocks smaller than 2^18 bits per
  // workgroup (the LDS and run lengths of one 2^18-bit block), as long as
  // their partitions lie in one first-level bucket
  c->bsub_log2 = 0;
  if (f.bloom_block_log2 >= 5 && f.bloom_block_log2 < 18) {
    uint32_t bs = std::min<uint32_t>(2, 18 - f.bloom_block_log2);
    bs = std::min<uint32_t>(bs, c->s_log2);
    bs = c->a2 >= c->upb_log2 ? std::min<uint32_t>(bs, c->a2 - c->upb_log2) : 0u;
    c->bsub_log2 = bs;
  }
  const uint32_t wg_words = c->nbw << c->bsub_log2;  // words per level in one k_bloom workgroup
  c->l2w = (wg_words + 1) & ~1u;
  c->count_lds = std::max((size_t)4 * (c->l2w + wg_words), (size_t)kWaves * 2 * 8);
  c->tally_lds = std::max((size_t)c->cap * c->slot_bytes + kQueueBytes,
                          (size_t)kTallyWaves * kNst * 8);
  if (c->count_lds > (size_t)kLdsMax || c->tally_lds > (size_t)kLdsMax)
    return fail(c, KC_ERR_INVALID_ARG, "LDS layout too large");
  c->bloom_words64 = f.bloom_bits_log2 >= 6 ? (1ull << (f.bloom_bits_log2 - 6)) : 1ull;
  return KC_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Forgets the spill directory; the pinned pool stays for the next finalize.
void free_spill(kc_ctx* c) {
  c->spill_used = 0;
  c->spill_dir.clear();
  c->spill_of.assign(1ull << c->p_log2, -1);
}

void release_spill_pool(kc_ctx* c) {
  if (c->spill_keys) (void)hipHostFree(c->spill_keys);
  if (c->spill_counts) (void)hipHostFree(c->spill_counts);
  c->spill_keys = nullptr;
  c->spill_counts = nullptr;
  c->spill_cap = 0;
  free_spill(c);
}

// Room for `tables` more partition tables in the pinned pool.  Growing keeps
// the tables already there (a copy); finalize sizes the pool once per run.
kc_status ensure_spill_pool(kc_ctx* c, uint64_t tables) {
  if (c->spill_used + tables <= c->spill_cap) return KC_OK;
  const uint64_t cap = c->cap, nc = c->cfg.n_counters;
  const uint64_t want = std::max<uint64_t>(c->spill_used + tables,
                                           c->spill_used ? c->spill_cap * 2 : 0);
  uint64_t* nk = nullptr;
  uint32_t* ncs = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&nk), want * cap * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ncs), want * cap * 4 * nc, hipHostMallocDefault) !=
          hipSuccess) {
    (void)hipGetLastError();
    if (nk) (void)hipHostFree(nk);
    return fail(c, KC_ERR_OUT_OF_MEMORY, "pinned spill pool allocation failed");
  }
  if (c->spill_used) {
    memcpy(nk, c->spill_keys, c->spill_used * cap * 8);
    memcpy(ncs, c->spill_counts, c->spill_used * cap * 4 * nc);
  }
  if (c->spill_keys) (void)hipHostFree(c->spill_keys);
  if (c->spill_counts) (void)hipHostFree(c->spill_counts);
  c->spill_keys = nk;
  c->spill_counts = ncs;
  c->spill_cap = want;
  return KC_OK;
}

kc_status sync_read(kc_ctx* c, hipStream_t s, const void* dev, size_t bytes, void* host) {
  if (bytes > kPinnedBytes) {  // larger than the pinned staging area: straight to the host buffer
    KC_HIP(c, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s), "readback");
    KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
    return KC_OK;
  }
  KC_HIP(c, hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  memcpy(host, c->pinned, bytes);
  return KC_OK;
}

// Directory record for the table of partition p, already copied to pool
// table t; entries come from the partition's statistics row.
void add_spill_record(kc_ctx* c, uint32_t p, uint64_t t, uint64_t entries) {
  SpillRec rec;
  rec.partition = p;
  rec.stale = false;
  rec.host_offset = t * c->cap;
  rec.entries = entries;
  c->spill_of[p] = (int32_t)c->spill_dir.size();
  c->spill_dir.push_back(rec);
  c->st.spilled_partitions += 1;
  c->st.spilled_bytes += (uint64_t)c->cap * c->slot_bytes;
}

// Moves the HBM table of a resident partition p to the pinned pool; its slot
// is then free (no longer exported or probed on the device).
kc_status spill_partition(kc_ctx* c, uint32_t p, hipStream_t s, uint64_t* bytes) {
  const uint32_t slot = c->slot_of_h[p];
  if (slot == kNoSlot) return KC_OK;
  const uint64_t cap = c->cap;
  const uint32_t nc = c->cfg.n_counters;
  kc_status r = ensure_spill_pool(c, 1);
  if (r != KC_OK) return r;
  const uint64_t t = c->spill_used;
  StageTimer tm(c, s, KC_T_SPILL);
  KC_HIP(c, hipMemcpyAsync(c->spill_keys + t * cap, c->tkeys.as<uint64_t>() + slot * cap, cap * 8,
                           hipMemcpyDeviceToHost, s),
         "spill copy");
  KC_HIP(c, hipMemcpyAsync(c->spill_counts + t * cap * nc, c->tcounts.as<uint32_t>() + slot * cap * nc,
                           cap * 4 * nc, hipMemcpyDeviceToHost, s),
         "spill copy");
  KC_HIP(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(c->slot_of.as<uint32_t>() + p),
                              kNoSlot, 1, s),
         "slot map");
  KC_HIP(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(c->slot_live.as<uint32_t>() + slot),
                              0, 1, s),
         "slot map");
  tm.stop();
  uint64_t row[kNst];
  r = sync_read(c, s, c->pstats2.as<uint64_t>() + (uint64_t)p * kNst, sizeof(row), row);
  if (r != KC_OK) return r;
  c->spill_used += 1;
  c->slot_of_h[p] = kNoSlot;
  c->slot_first = -1;
  add_spill_record(c, p, t, row[ST_ENTRIES]);
  if (bytes) *bytes += cap * c->slot_bytes;
  return KC_OK;
}

// Arguments of the count kernels over the context's current buffers (the
// launch range fields part_base / part_n / slot_base are the caller's).
CountArgs count_args(kc_ctx* c, uint32_t nsegs) {
  const uint64_t on = 1ull << c->ovf_log2;
  CountArgs a{};
  a.hc = c->hc;
  a.segs = c->segdesc.as<SegDesc>();
  a.nsegs = nsegs;
  a.upb_log2 = c->upb_log2;
  a.nbw = c->nbw;
  a.l2w = c->l2w;
  a.bsub_log2 = c->bsub_log2;
  a.cap = c->cap;
  a.probe_limit = probe_limit_of(c->cap);
  a.ovf_log2 = c->ovf_log2;
  a.ovf_limit = (uint32_t)std::min<uint64_t>(on / 2, 0xFFFFFFFFull);
  a.b1 = c->b1.as<uint32_t>();
  a.b2 = c->b2.as<uint32_t>();
  a.tkeys = c->tkeys.as<uint64_t>();
  a.tcounts = c->tcounts.as<uint32_t>();
  a.okeys = c->okeys.as<uint64_t>();
  a.ocounts = c->ocounts.as<uint32_t>();
  a.ovf_used = c->ovf_used.as<uint32_t>();
  a.err = c->derr.as<uint32_t>();
  a.pstats = c->pstats.as<uint64_t>();
  a.pstats2 = c->pstats2.as<uint64_t>();
  return a;
}

// A captured batch graph points at buffers that an eager insert or finalize
// may reallocate: those calls drop the graph (the next kc_count_batch
// captures it again).  The plan's segments stay until that rebuild, since
// the context may still be reading them.
void invalidate_batch_graph(kc_ctx* c) {
  BatchPlan& b = c->batch;
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.chunks.clear();
}

uint64_t resident_bytes(const kc_ctx* c) {
  uint64_t n = 0;
  for (uint32_t v : c->slot_of_h) n += v != kNoSlot;
  return n * c->cap * c->slot_bytes;
}

}  // namespace

namespace kc {

uint64_t ctx_device_bytes(const kc_ctx* c) {
  const DevBuf* bufs[] = {&c->b1, &c->b2, &c->dstat, &c->derr, &c->packed, &c->flags, &c->hist1,
                          &c->lstart1, &c->off1, &c->parts, &c->keys1, &c->tile_desc, &c->segdesc,
                          &c->tkeys, &c->tcounts, &c->slot_of, &c->slot_live, &c->pstats,
                          &c->pstats2, &c->pstats_ovf, &c->okeys, &c->ocounts, &c->ovf_used,
                          &c->qrows, &c->qkeys, &c->qcount};
  uint64_t n = 0;
  for (const DevBuf* b : bufs) n += b->bytes;
  auto seg = [](const Segment& g) {
    return (uint64_t)g.keys.bytes + g.bucket_off.bytes + g.tile_first.bytes + g.meta2.bytes;
  };
  if (!c->segs_borrowed)
    for (const Segment& g : c->segs) n += seg(g);
  for (const Segment& g : c->spare_segs) n += seg(g);
  for (const BatchGroup& g : c->batch.groups) n += seg(g.seg) + g.cdesc.bytes;
  return n + c->batch.counts.bytes;
}

uint64_t bytes_after(const kc_ctx* c, const kc_config* cfg, const uint64_t* part_bases,
                     uint32_t n_parts) {
  std::string why;
  if (validate(cfg, &why) != KC_OK) return 0;
  kc_ctx d;
  d.cfg = *cfg;
  if (derive(&d) != KC_OK) return 0;
  const uint64_t nb1 = 1ull << d.a1, nb2 = 1ull << d.a2;
  const uint64_t nparts = 1ull << d.p_log2, nc = cfg->n_counters;
  // the server's contexts allocate from its block cache: sizes as the cache rounds them
  auto mx = [&](const DevBuf kc_ctx::*buf, uint64_t need) {
    return std::max<uint64_t>(c ? (c->*buf).bytes : 0, cache_round(std::max<uint64_t>(need, 8)));
  };
  // first-level scratch (largest insert) and the per-insert segments
  uint64_t packed = 0, hist = 0, lstart = 0, off = 0, parts = 0, keys1 = 0, runs = 0, keys = 0;
  std::vector<std::array<uint64_t, 2>> seg;  // keys bytes, other bytes of each new segment
  for (uint32_t i = 0; i < n_parts; ++i) {
    const uint64_t nwords = (part_bases[i] + 31) / 32;
    const uint64_t ntiles = (nwords + kTileWords - 1) / kTileWords;
    const uint64_t nhist = nb1 * ntiles;
    const uint64_t kmax = nwords * 32;  // keys <= window positions
    const uint64_t tiles2 = ((kmax + (1ull << d.t2_log2) - 1) >> d.t2_log2) + nb1;
    packed = std::max(packed, nwords * 8);
    hist = std::max(hist, nhist * 4);
    lstart = std::max(lstart, ntiles * (nb1 + 1) * 4);
    off = std::max(off, (nhist + 1) * 8);
    parts = std::max<uint64_t>(parts, scan_parts(nhist) * 8);
    keys1 = std::max<uint64_t>(keys1, ntiles * kTilePos * 8);
    runs = std::max(runs, tile_desc_bytes(tiles2));
    if (kmax)
      seg.push_back({cache_round(kmax * 8), cache_round((nb1 + 1) * 8) + cache_round((nb1 + 1) * 4) +
                                                cache_round(tiles2 * (nb2 + 1) * 4)});
    keys += kmax;
  }
  uint64_t n = mx(&kc_ctx::b1, d.bloom_words64 * 8) + mx(&kc_ctx::b2, d.bloom_words64 * 8) +
               mx(&kc_ctx::packed, packed) + mx(&kc_ctx::flags, packed) + mx(&kc_ctx::hist1, hist) +
               mx(&kc_ctx::lstart1, lstart) + mx(&kc_ctx::off1, off) + mx(&kc_ctx::parts, parts) +
               mx(&kc_ctx::keys1, keys1) + mx(&kc_ctx::tile_desc, runs);
  const uint32_t ovf_log2 = std::max<uint32_t>(12, std::min<uint32_t>(30, ceil_log2(keys / 256 + 1)));
  const uint64_t on = 1ull << ovf_log2;
  const uint64_t oblocks = std::min<uint64_t>(1024, (on + 255) / 256);
  n += mx(&kc_ctx::tkeys, nparts * d.cap * 8) + mx(&kc_ctx::tcounts, nparts * d.cap * 4 * nc) +
       mx(&kc_ctx::slot_of, nparts * 4) + mx(&kc_ctx::slot_live, nparts * 4) +
       mx(&kc_ctx::pstats, (1ull << d.s_log2) * kNst * 8) +
       mx(&kc_ctx::pstats2, nparts * kNst * 8) + mx(&kc_ctx::okeys, on * 8) +
       mx(&kc_ctx::ocounts, on * 4 * nc) + mx(&kc_ctx::pstats_ovf, oblocks * kNst * 8) +
       mx(&kc_ctx::segdesc, std::max<uint64_t>(1, n_parts) * sizeof(SegDesc)) +
       mx(&kc_ctx::dstat, kNst * 8 * 3) + mx(&kc_ctx::derr, 8) + mx(&kc_ctx::ovf_used, 8) +
       mx(&kc_ctx::qcount, 8) + (c ? c->qrows.bytes + c->qkeys.bytes : 0);
  // segments: after a reset the context keeps at most four spare ones, largest
  // first; an insert reuses the first spare whose key buffer is large enough
  std::vector<const Segment*> spare;
  if (c) {
    if (!c->segs_borrowed)
      for (const Segment& g : c->segs) spare.push_back(&g);
    for (const Segment& g : c->spare_segs) spare.push_back(&g);
    std::sort(spare.begin(), spare.end(),
              [](const Segment* a, const Segment* b) { return a->keys.bytes > b->keys.bytes; });
    if (spare.size() > 4) spare.resize(4);
    for (const BatchGroup& g : c->batch.groups)
      n += g.seg.keys.bytes + g.seg.bucket_off.bytes + g.seg.tile_first.bytes + g.seg.meta2.bytes +
           g.cdesc.bytes;
    n += c->batch.counts.bytes;
  }
  for (const auto& need : seg) {
    size_t k = 0;
    while (k < spare.size() && spare[k]->keys.bytes < need[0]) ++k;
    if (k < spare.size()) {
      const Segment* g = spare[k];
      n += g->keys.bytes + std::max<uint64_t>(g->bucket_off.bytes + g->tile_first.bytes + g->meta2.bytes,
                                              need[1]);
      spare.erase(spare.begin() + k);
    } else {
      n += need[0] + need[1];
    }
  }
  for (const Segment* g : spare)
    n += g->keys.bytes + g->bucket_off.bytes + g->tile_first.bytes + g->meta2.bytes;
  return n;
}

uint64_t estimate_count_bytes(const kc_config* cfg, const uint64_t* part_bases, uint32_t n_parts) {
  return bytes_after(nullptr, cfg, part_bases, n_parts);
}

kc_status reconfigure(kc_ctx* c, const kc_config* cfg, hipStream_t s) {
  if (!c) return KC_ERR_INVALID_ARG;
  AllocStream alloc_on(s);
  if (c->state != CREATED) return fail(c, KC_ERR_BAD_STATE, "reconfigure needs a reset context");
  std::string why;
  if (validate(cfg, &why) != KC_OK) return fail(c, KC_ERR_INVALID_ARG, why);
  const kc_config old = c->cfg;
  c->cfg = *cfg;
  kc_status r = derive(c);
  if (r != KC_OK) {
    c->cfg = old;
    (void)derive(c);
    return r;
  }
  invalidate_batch_graph(c);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  KC_HIP(c, c->b1.ensure(c->bloom_words64 * 8), "Bloom level allocation");
  KC_HIP(c, c->b2.ensure(c->bloom_words64 * 8), "Bloom level allocation");
  c->spill_of.assign(1ull << c->p_log2, -1);
  c->slot_of_h.clear();
  c->st.partitions_log2 = c->p_log2;
  c->st.table_slots = c->cap;
  return KC_OK;
}

}  // namespace kc

// Filter-unit lookup: the reads are packed and their read starts marked as
// for an insert, then every window is looked up in the final tables (bitmap
// of selected windows) and each read's selected windows are counted.  The
// packed words, flag words and window bitmap are scratch: every word of them
// that a kernel reads is written earlier in the same call.
namespace {

kc_status filter_checks(kc_ctx* c, const uint8_t* bases, const uint64_t* offsets, uint64_t n_reads,
                        uint64_t total_bases, uint32_t* out) {
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "filter before finalize");
  if (!c->spill_dir.empty())
    return fail(c, KC_ERR_BAD_STATE, "filter needs every partition table in HBM (tables were spilled)");
  if (n_reads == 0) return KC_OK;
  if (!offsets || !out || (total_bases && !bases))
    return fail(c, KC_ERR_INVALID_ARG, "NULL read or output buffer");
  if (total_bases > 0xFFFFFFFFull) return fail(c, KC_ERR_INVALID_ARG, "more than 2^32 - 1 bases in one call");
  return KC_OK;
}

// With fkeys (room for every resident slot) the lookups read the table keys
// marked with the selection (launch_filter_keys) instead of keys and counts.
kc_status filter_run(kc_ctx* c, const uint8_t* bases, const uint64_t* offsets, uint64_t n_reads,
                     uint64_t total_bases, uint32_t tumour_min, uint32_t normal_max, uint32_t* out,
                     hipStream_t s, uint64_t* packed, uint64_t* flags, uint32_t* hit, bool timed,
                     uint64_t* fkeys) {
  const uint64_t nwords = (total_bases + 31) / 32;
  KC_HIP(c, launch_fill32(c->derr.as<uint32_t>(), 1, 0, s), "fill");
  QueryArgs a{};
  a.hc = c->hc;
  a.cap = c->cap;
  a.probe_limit = probe_limit_of(c->cap);
  a.tkeys = c->tkeys.as<uint64_t>();
  a.tcounts = c->tcounts.as<uint32_t>();
  a.slot_of = c->slot_of.as<uint32_t>();
  a.slot_first = c->slot_first;
  a.okeys = c->okeys.as<uint64_t>();
  a.ocounts = c->ocounts.as<uint32_t>();
  a.ovf_used = c->ovf_used.as<uint32_t>();
  a.ovf_log2 = c->ovf_log2;
  a.err = c->derr.as<uint32_t>();
  a.fkeys = fkeys;
  {
    StageTimer t(c, s, KC_T_FILTER, timed);
    if (fkeys)
      KC_HIP(c, launch_filter_keys(c->tkeys.as<uint64_t>(), c->tcounts.as<uint32_t>(),
                                   (uint64_t)c->pool_slots * c->cap, c->cfg.n_counters, tumour_min,
                                   normal_max, fkeys, s),
             "filter keys");
    KC_HIP(c, launch_pack(bases, total_bases, nwords, packed, flags, s), "pack");
    KC_HIP(c, launch_rstart(offsets, n_reads, total_bases, flags, c->derr.as<uint32_t>(), s),
           "read starts");
    KC_HIP(c, launch_filter(a, packed, flags, nwords, offsets, n_reads, total_bases, tumour_min,
                            normal_max, hit, out, s),
           "filter");
    t.stop();
  }
  uint32_t errf = 0;
  kc_status r = sync_read(c, s, c->derr.p, 4, &errf);
  if (r != KC_OK) return r;
  if (errf & ERR_OFFSETS)
    return fail(c, KC_ERR_INVALID_ARG,
                "offsets must start at 0, be non-decreasing and end at total_bases");
  return KC_OK;
}

// Scratch of kc_filter_reads_noalloc: packed words, flag words and the
// window bitmap of up to KC_FILTER_NOALLOC_MAX_BASES bases, one copy per
// GPU for the life of the process.  Host code never uses the array's name
// as an address: its device address comes from hipGetSymbolAddress, once per
// device (noalloc_scratch), and that address is what the kernels receive.
constexpr uint64_t kNaWords = KC_FILTER_NOALLOC_MAX_BASES / 32;
constexpr size_t kNaPackedOff = 0;
constexpr size_t kNaFlagsOff = kNaWords * 8;
constexpr size_t kNaHitOff = kNaWords * 16;
constexpr size_t kNaBytes = kNaWords * 20;
static_assert(KC_FILTER_NOALLOC_MAX_BASES % 32 == 0 && kNaFlagsOff % 256 == 0 && kNaHitOff % 256 == 0,
              "scratch layout");
__device__ __align__(256) uint8_t scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up once per device.
kc_status noalloc_scratch(int device, void** out, std::string* why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device index too large for the scratch table";
    return KC_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      *why = std::string("hipGetSymbolAddress of the filter scratch: ") + hipGetErrorString(e);
      return KC_ERR_DEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return KC_OK;
}

}  // namespace

extern "C" {

uint32_t kc_abi_version(void) { return KC_ABI_VERSION; }

const char* kc_status_str(kc_status s) {
  switch (s) {
    case KC_OK: return "KC_OK";
    case KC_ERR_INVALID_ARG: return "KC_ERR_INVALID_ARG";
    case KC_ERR_OUT_OF_MEMORY: return "KC_ERR_OUT_OF_MEMORY";
    case KC_ERR_BAD_STATE: return "KC_ERR_BAD_STATE";
    case KC_ERR_DEVICE: return "KC_ERR_DEVICE";
    case KC_ERR_OVER_BUDGET: return "KC_ERR_OVER_BUDGET";
  }
  return "KC_UNKNOWN";
}

const char* kc_last_error(const kc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

kc_status kc_create(const kc_config* cfg, int device, kc_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return KC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  std::string why;
  if (validate(cfg, &why) != KC_OK) {
    g_create_error = why;
    return KC_ERR_INVALID_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    g_create_error = "no such HIP device";
    return KC_ERR_INVALID_ARG;
  }
  kc_ctx* c = new (std::nothrow) kc_ctx();
  if (!c) {
    g_create_error = "host allocation failed";
    return KC_ERR_OUT_OF_MEMORY;
  }
  c->cfg = *cfg;
  c->device = device;
  kc_status r = derive(c);
  if (r != KC_OK) {
    g_create_error = c->err;
    delete c;
    return r;
  }
  auto bail = [&](kc_status s, const std::string& m) {
    g_create_error = m;
    kc_destroy(c);
    return s;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(KC_ERR_DEVICE, "hipSetDevice failed");
  kc::keep_pool_memory(device);
  {
    void* scratch_ptr = nullptr;
    std::string why;
    if (noalloc_scratch(device, &scratch_ptr, &why) != KC_OK) return bail(KC_ERR_DEVICE, why);
  }
  const size_t bloom_bytes = c->bloom_words64 * 8;
  if (c->b1.ensure(bloom_bytes) != hipSuccess || c->b2.ensure(bloom_bytes) != hipSuccess)
    return bail(KC_ERR_OUT_OF_MEMORY, "Bloom level allocation failed");
  if (c->dstat.ensure(kNst * 8 * 3) != hipSuccess || c->derr.ensure(8) != hipSuccess ||
      c->ovf_used.ensure(8) != hipSuccess || c->qcount.ensure(8) != hipSuccess)
    return bail(KC_ERR_OUT_OF_MEMORY, "device allocation failed");
  if (hipHostMalloc(reinterpret_cast<void**>(&c->pinned), kPinnedBytes, hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    c->pinned = nullptr;
    return bail(KC_ERR_OUT_OF_MEMORY, "pinned allocation failed");
  }
  if (hipEventCreateWithFlags(&c->insert_done, hipEventDisableTiming) != hipSuccess)
    return bail(KC_ERR_DEVICE, "event creation failed");
  c->spill_of.assign(1ull << c->p_log2, -1);
  c->st.partitions_log2 = c->p_log2;
  c->st.table_slots = c->cap;
  *out = c;
  return KC_OK;
}

kc_status kc_insert_reads(kc_ctx* c, const uint8_t* bases, const uint64_t* offsets,
                          uint64_t n_reads, uint64_t total_bases, uint32_t counter,
                          void* hip_stream) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state == FINALIZED) return fail(c, KC_ERR_BAD_STATE, "insert after finalize (reset first)");
  if (counter >= c->cfg.n_counters) return fail(c, KC_ERR_INVALID_ARG, "counter >= n_counters");
  if (!offsets) return fail(c, KC_ERR_INVALID_ARG, "offsets is NULL");
  if (total_bases && !bases) return fail(c, KC_ERR_INVALID_ARG, "bases is NULL");
  if (total_bases >= (1ull << 32))
    return fail(c, KC_ERR_INVALID_ARG, "more than 2^32 - 1 bases in one call (split the reads)");
  hipStream_t s = as_stream(hip_stream);
  kc::AllocStream alloc_on(s);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  if (c->insert_done_valid) KC_HIP(c, hipStreamWaitEvent(s, c->insert_done, 0), "stream wait");
  invalidate_batch_graph(c);
  c->state = INSERTING;

  const uint64_t nwords = (total_bases + 31) / 32;
  const uint64_t ntiles = (nwords + kTileWords - 1) / kTileWords;
  const uint32_t nb1 = 1u << c->a1;
  const uint64_t nhist = (uint64_t)nb1 * ntiles;
  KC_HIP(c, c->packed.ensure(nwords * 8), "packed buffer");
  KC_HIP(c, c->flags.ensure(nwords * 8), "flag buffer");
  KC_HIP(c, c->hist1.ensure(nhist * 4), "histogram buffer");
  KC_HIP(c, c->lstart1.ensure(ntiles * (nb1 + 1) * 4), "tile start buffer");
  KC_HIP(c, c->off1.ensure((nhist + 1) * 8), "offset buffer");
  KC_HIP(c, c->parts.ensure(scan_parts(nhist) * 8), "scan buffer");
  KC_HIP(c, c->keys1.ensure(ntiles * kTilePos * 8), "first-level key buffer");
  KC_HIP(c, hipMemsetAsync(c->derr.p, 0, 4, s), "memset");

  const uint64_t s0 = c->hc.salt[0];
  const uint64_t tag = (uint64_t)counter << 62;
  {
    StageTimer t(c, s, KC_T_PACK);
    KC_HIP(c, launch_pack(bases, total_bases, nwords, c->packed.as<uint64_t>(),
                          c->flags.as<uint64_t>(), s),
           "pack");
    KC_HIP(c, launch_rstart(offsets, n_reads, total_bases, c->flags.as<uint64_t>(),
                            c->derr.as<uint32_t>(), s),
           "read starts");
    t.stop();
  }
  {
    StageTimer t(c, s, KC_T_LEVEL1);
    KC_HIP(c, launch_level1(c->packed.as<uint64_t>(), c->flags.as<uint64_t>(), nwords, c->cfg.k,
                            s0, c->a1, tag, c->hist1.as<uint32_t>(), c->lstart1.as<uint32_t>(),
                            ntiles, c->keys1.as<uint64_t>(), s),
           "first-level shuffle");
    t.stop();
  }
  {
    StageTimer t(c, s, KC_T_SCAN);
    KC_HIP(c, launch_scan(c->hist1.as<uint32_t>(), nhist, c->off1.as<uint64_t>(),
                          c->parts.as<uint64_t>(), s),
           "scan");
    t.stop();
  }
  KC_HIP(c, hipMemcpyAsync(c->pinned, c->off1.as<uint64_t>() + nhist, 8, hipMemcpyDeviceToHost, s),
         "readback");
  KC_HIP(c, hipMemcpyAsync(c->pinned + 1, c->derr.p, 4, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  const uint64_t n = c->pinned[0];
  const uint32_t errf = (uint32_t)c->pinned[1];
  if (errf & ERR_OFFSETS)
    return fail(c, KC_ERR_INVALID_ARG,
                "offsets must start at 0, be non-decreasing and end at total_bases");
  if (n == 0) return KC_OK;

  Segment seg;
  // reuse a kept segment allocation when it is large enough
  for (size_t i = 0; i < c->spare_segs.size(); ++i) {
    if (c->spare_segs[i].keys.bytes >= n * 8) {
      seg = c->spare_segs[i];
      c->spare_segs.erase(c->spare_segs.begin() + i);
      break;
    }
  }
  seg.n = n;
  seg.counter = counter;
  const uint32_t nb2 = 1u << c->a2;
  const uint64_t tiles2 = ((n + (1ull << c->t2_log2) - 1) >> c->t2_log2) + nb1;
  hipError_t e;
  if ((e = seg.keys.ensure(n * 8)) != hipSuccess || (e = seg.bucket_off.ensure((nb1 + 1) * 8)) != hipSuccess ||
      (e = seg.tile_first.ensure((nb1 + 1) * 4)) != hipSuccess ||
      (e = seg.meta2.ensure(tiles2 * (nb2 + 1) * 4)) != hipSuccess) {
    seg.release();
    return hip_fail(c, e, "segment allocation");
  }
  KC_HIP(c, c->tile_desc.ensure(tile_desc_bytes(tiles2)), "tile descriptor buffer");
  {
    StageTimer t(c, s, KC_T_LEVEL2);
    KC_HIP(c, launch_bucket_off(c->off1.as<uint64_t>(), ntiles, nb1, seg.bucket_off.as<uint64_t>(), s),
           "bucket offsets");
    KC_HIP(c, launch_tiles2(seg.bucket_off.as<uint64_t>(), nb1, c->t2_log2,
                            seg.tile_first.as<uint32_t>(), s),
           "tiles");
    KC_HIP(c, launch_level2(c->keys1.as<uint64_t>(), c->off1.as<uint64_t>(),
                            c->lstart1.as<uint32_t>(), ntiles, seg.bucket_off.as<uint64_t>(),
                            seg.tile_first.as<uint32_t>(), c->tile_desc.as<uint64_t>(), c->a1,
                            c->a2, c->t2_log2, s0, seg.keys.as<uint64_t>(), seg.meta2.as<uint32_t>(), tiles2,
                            s),
           "second-level shuffle");
    t.stop();
  }
  KC_HIP(c, hipEventRecord(c->insert_done, s), "event record");
  c->insert_done_valid = true;
  c->segs.push_back(seg);
  c->st.n_valid += n;
  c->st.n_segments += 1;
  return KC_OK;
}

kc_status kc_finalize(kc_ctx* c, void* hip_stream, kc_stats* out) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state == FINALIZED) return fail(c, KC_ERR_BAD_STATE, "already finalized");
  hipStream_t s = as_stream(hip_stream);
  kc::AllocStream alloc_on(s);
  invalidate_batch_graph(c);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  if (c->insert_done_valid) KC_HIP(c, hipStreamWaitEvent(s, c->insert_done, 0), "stream wait");
  const uint32_t nc = c->cfg.n_counters;
  const uint64_t nparts = 1ull << c->p_log2;
  const uint64_t cap = c->cap;
  const uint64_t budget = c->cfg.hbm_table_budget_bytes;
  const uint64_t per_table = cap * c->slot_bytes;
  if (budget && budget < per_table)
    return fail(c, KC_ERR_OVER_BUDGET, "table budget smaller than one partition table");
  // HBM holds R partition tables (all of them, or what the budget pays for).
  // The last R partitions are counted straight into their slots; the others
  // are counted in waves through two staging halves of the same slots, and
  // each wave's tables are copied to the pinned pool while the next wave runs.
  // Table memory in HBM never exceeds R tables.
  const uint64_t R = budget ? std::min<uint64_t>(nparts, budget / per_table) : nparts;
  const uint64_t n_spill = nparts - R;
  c->pool_slots = (uint32_t)R;
  KC_HIP(c, c->tkeys.ensure(R * cap * 8), "table allocation");
  KC_HIP(c, c->tcounts.ensure(R * cap * 4 * nc), "table allocation");
  KC_HIP(c, c->slot_of.ensure(nparts * 4), "slot map");
  KC_HIP(c, c->slot_live.ensure(R * 4), "slot map");
  KC_HIP(c, c->pstats.ensure((1ull << c->s_log2) * kNst * 8), "stats rows");
  KC_HIP(c, c->pstats2.ensure(nparts * kNst * 8), "stats rows");
  free_spill(c);
  c->st.spilled_partitions = 0;
  c->st.spilled_bytes = 0;
  uint64_t wave = 0, nbuf = 1;
  if (n_spill) {
    kc_status r = ensure_spill_pool(c, n_spill);
    if (r != KC_OK) return r;
    if (!c->copy_stream) KC_HIP(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking),
                                "copy stream");
    for (int b = 0; b < 2; ++b) {
      if (!c->ev_tally[b])
        KC_HIP(c, hipEventCreateWithFlags(&c->ev_tally[b], hipEventDisableTiming), "event");
      if (!c->ev_copy[b])
        KC_HIP(c, hipEventCreateWithFlags(&c->ev_copy[b], hipEventDisableTiming), "event");
    }
    nbuf = R >= 2 ? 2 : 1;
    wave = R / nbuf;
    // whole groups of 8 Bloom blocks keep the XCD-aware partition order
    const uint64_t group = 8ull << c->upb_log2;
    if (wave >= group) wave -= wave % group;
  }

  std::vector<SegDesc> hd(c->segs.size());
  for (size_t i = 0; i < c->segs.size(); ++i) {
    const Segment& g = c->segs[i];
    hd[i].keys = g.keys.as<uint64_t>();
    hd[i].bucket_off = g.bucket_off.as<uint64_t>();
    hd[i].tile_first = g.tile_first.as<uint32_t>();
    hd[i].meta2 = g.meta2.as<uint32_t>();
    hd[i].a1 = c->a1;
    hd[i].a2 = c->a2;
    hd[i].t2_log2 = c->t2_log2;
  }
  KC_HIP(c, c->segdesc.ensure(std::max<size_t>(1, hd.size()) * sizeof(SegDesc)), "segment table");
  if (!hd.empty())
    KC_HIP(c, hipMemcpyAsync(c->segdesc.p, hd.data(), hd.size() * sizeof(SegDesc),
                             hipMemcpyHostToDevice, s),
           "segment table copy");

  // overflow table: sized from the occurrence count, grown on a fill
  c->ovf_log2 = std::max<uint32_t>(12, std::min<uint32_t>(30, ceil_log2(c->st.n_valid / 256 + 1)));
  c->st.retries = 0;
  uint64_t sv[kNst];
  uint32_t errf = 0;
  for (;;) {
    const uint64_t on = 1ull << c->ovf_log2;
    KC_HIP(c, c->okeys.ensure(on * 8), "overflow table");
    KC_HIP(c, c->ocounts.ensure(on * 4 * nc), "overflow table");
    const uint32_t oblocks = (uint32_t)std::min<uint64_t>(1024, (on + 255) / 256);
    KC_HIP(c, c->pstats_ovf.ensure((uint64_t)oblocks * kNst * 8), "stats rows");
    KC_HIP(c, hipMemsetAsync(c->okeys.p, 0xFF, on * 8, s), "memset");
    KC_HIP(c, hipMemsetAsync(c->ocounts.p, 0, on * 4 * nc, s), "memset");
    KC_HIP(c, hipMemsetAsync(c->ovf_used.p, 0, 4, s), "memset");
    KC_HIP(c, hipMemsetAsync(c->derr.p, 0, 4, s), "memset");
    if (c->cfg.bloom_block_log2 < 5) {
      KC_HIP(c, hipMemsetAsync(c->b1.p, 0, c->bloom_words64 * 8, s), "memset");
      KC_HIP(c, hipMemsetAsync(c->b2.p, 0, c->bloom_words64 * 8, s), "memset");
    }
    CountArgs a = count_args(c, (uint32_t)hd.size());
    {
      StageTimer t(c, s, KC_T_BLOOM);
      KC_HIP(c, launch_bloom(a, 1u << c->s_log2, c->count_lds, s), "Bloom kernel");
      t.stop();
    }
    // waves of spilled partitions
    for (uint64_t first = 0, w = 0; first < n_spill; first += wave, ++w) {
      const uint64_t n = std::min<uint64_t>(wave, n_spill - first);
      const int b = (int)(w % nbuf);
      const uint64_t slot0 = (uint64_t)b * wave;
      if (w >= nbuf) KC_HIP(c, hipStreamWaitEvent(s, c->ev_copy[b], 0), "stream wait");
      a.part_base = (uint32_t)first;
      a.part_n = (uint32_t)n;
      a.slot_base = (uint32_t)slot0;
      {
        StageTimer t(c, s, KC_T_TALLY);
        KC_HIP(c, launch_tally(a, (uint32_t)n, c->tally_lds, s), "count kernel");
        t.stop();
      }
      KC_HIP(c, hipEventRecord(c->ev_tally[b], s), "event");
      KC_HIP(c, hipStreamWaitEvent(c->copy_stream, c->ev_tally[b], 0), "stream wait");
      {
        StageTimer t(c, c->copy_stream, KC_T_SPILL);
        KC_HIP(c, hipMemcpyAsync(c->spill_keys + first * cap, c->tkeys.as<uint64_t>() + slot0 * cap,
                                 n * cap * 8, hipMemcpyDeviceToHost, c->copy_stream),
               "spill copy");
        KC_HIP(c, hipMemcpyAsync(c->spill_counts + first * cap * nc,
                                 c->tcounts.as<uint32_t>() + slot0 * cap * nc, n * cap * 4 * nc,
                                 hipMemcpyDeviceToHost, c->copy_stream),
               "spill copy");
        t.stop();
      }
      KC_HIP(c, hipEventRecord(c->ev_copy[b], c->copy_stream), "event");
    }
    if (n_spill) {
      for (uint64_t b = 0; b < nbuf; ++b) KC_HIP(c, hipStreamWaitEvent(s, c->ev_copy[b], 0), "stream wait");
    }
    // resident partitions, straight into their slots
    a.part_base = (uint32_t)n_spill;
    a.part_n = (uint32_t)R;
    a.slot_base = 0;
    {
      StageTimer t(c, s, KC_T_TALLY);
      KC_HIP(c, launch_tally(a, (uint32_t)R, c->tally_lds, s), "count kernel");
      t.stop();
    }
    {
      StageTimer t(c, s, KC_T_UNIFY);
      KC_HIP(c, launch_ovf_emit(a, c->pstats_ovf.as<uint64_t>(), oblocks, s), "overflow pass");
      KC_HIP(c, launch_reduce(c->pstats.as<uint64_t>(), (1ull << c->s_log2) >> c->bsub_log2,
                              c->dstat.as<uint64_t>(), s),
             "reduce");
      KC_HIP(c, launch_reduce(c->pstats_ovf.as<uint64_t>(), oblocks, c->dstat.as<uint64_t>() + kNst, s),
             "reduce");
      KC_HIP(c, launch_reduce(c->pstats2.as<uint64_t>(), nparts, c->dstat.as<uint64_t>() + 2 * kNst, s),
             "reduce");
      t.stop();
    }
    KC_HIP(c, hipMemcpyAsync(c->pinned, c->dstat.p, 3 * kNst * 8, hipMemcpyDeviceToHost, s), "readback");
    KC_HIP(c, hipMemcpyAsync(c->pinned + 3 * kNst, c->derr.p, 4, hipMemcpyDeviceToHost, s), "readback");
    KC_HIP(c, hipMemcpyAsync(c->pinned + 3 * kNst + 1, c->ovf_used.p, 4, hipMemcpyDeviceToHost, s),
           "readback");
    KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
    errf = (uint32_t)c->pinned[3 * kNst];
    for (int i = 0; i < kNst; ++i) sv[i] = c->pinned[i] + c->pinned[kNst + i] + c->pinned[2 * kNst + i];
    if (!(errf & (ERR_OVF_FULL | ERR_OVF_LOAD))) break;
    if (c->st.retries >= 6 || c->ovf_log2 + 3 > 34)
      return fail(c, KC_ERR_OUT_OF_MEMORY, "overflow table kept filling up");
    c->ovf_log2 += 3;
    c->st.retries += 1;
  }
  c->st.n_pass = sv[ST_NPASS];
  c->st.entries = sv[ST_ENTRIES];
  c->st.sum_counts = sv[ST_SUM];
  c->st.fp_singletons = sv[ST_FP];
  c->st.b1_popcount = sv[ST_B1POP];
  c->st.b2_popcount = sv[ST_B2POP];
  c->st.passed_distinct = sv[ST_PASSED];
  {
    uint32_t used = 0;
    memcpy(&used, reinterpret_cast<uint8_t*>(c->pinned + 3 * kNst + 1), 4);
    c->st.overflow_keys = used;
  }
  // slot map: partitions below n_spill live in the pool, the rest in slots 0..R
  KC_HIP(c, launch_slot_map(c->slot_of.as<uint32_t>(), (uint32_t)nparts, (uint32_t)n_spill, s), "slot map");
  KC_HIP(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(c->slot_live.p), 1, R, s), "slot map");
  c->slot_of_h.resize(nparts);
  for (uint64_t u = 0; u < nparts; ++u) c->slot_of_h[u] = u < n_spill ? kNoSlot : (uint32_t)(u - n_spill);
  c->slot_first = (int64_t)n_spill;
  if (n_spill) {
    std::vector<uint64_t> rows(n_spill * kNst);
    KC_HIP(c, hipMemcpyAsync(rows.data(), c->pstats2.p, rows.size() * 8, hipMemcpyDeviceToHost, s),
           "readback");
    KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
    for (uint64_t u = 0; u < n_spill; ++u) add_spill_record(c, (uint32_t)u, u, rows[u * kNst + ST_ENTRIES]);
    c->spill_used = n_spill;
  }
  KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  c->state = FINALIZED;
  resolve_timers(c);
  if (out) *out = c->st;
  return KC_OK;
}

// Host lookup of a canonical key in the pinned copy of its partition table:
// the same home slot and linear probing as on the device.
void host_probe(const kc_ctx* c, const SpillRec& rec, uint64_t x, uint32_t* out) {
  const uint64_t cap = c->cap;
  const uint32_t nc = c->cfg.n_counters;
  const uint64_t th = (x ^ c->hc.salt[0]) * kTableMul;
  uint64_t slot = home_slot_of(th, cap);
  const uint64_t* keys = c->spill_keys + rec.host_offset;
  const uint32_t* counts = c->spill_counts + rec.host_offset * nc;
  for (uint64_t n = 0, limit = probe_limit_of(cap); n < limit; ++n) {
    const uint64_t k = keys[slot];
    if (k == x) {
      for (uint32_t t = 0; t < nc; ++t) out[t] = counts[slot * nc + t];
      return;
    }
    if (k == kEmpty) return;
    slot = slot + 1 == cap ? 0 : slot + 1;
  }
}

kc_status kc_query(kc_ctx* c, const uint64_t* kmers, uint64_t n, uint32_t* counts, void* hip_stream) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "query before finalize");
  if (n == 0) return KC_OK;
  if (!kmers || !counts) return fail(c, KC_ERR_INVALID_ARG, "NULL query buffer");
  if (n > 0xFFFFFFFFull) return fail(c, KC_ERR_INVALID_ARG, "more than 2^32 queries in one call");
  hipStream_t s = as_stream(hip_stream);
  kc::AllocStream alloc_on(s);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  const bool any_spill = !c->spill_dir.empty();
  if (any_spill) {
    KC_HIP(c, c->qrows.ensure(n * 4), "query rows");
    KC_HIP(c, c->qkeys.ensure(n * 8), "query keys");
  }
  KC_HIP(c, hipMemsetAsync(c->derr.p, 0, 4, s), "memset");
  KC_HIP(c, hipMemsetAsync(c->qcount.p, 0, 4, s), "memset");
  QueryArgs a{};
  a.hc = c->hc;
  a.cap = c->cap;
  a.probe_limit = probe_limit_of(c->cap);
  a.tkeys = c->tkeys.as<uint64_t>();
  a.tcounts = c->tcounts.as<uint32_t>();
  a.slot_of = c->slot_of.as<uint32_t>();
  a.slot_first = c->slot_first;
  a.okeys = c->okeys.as<uint64_t>();
  a.ocounts = c->ocounts.as<uint32_t>();
  a.ovf_used = c->ovf_used.as<uint32_t>();
  a.ovf_log2 = c->ovf_log2;
  a.err = c->derr.as<uint32_t>();
  a.host_rows = any_spill ? c->qrows.as<uint32_t>() : nullptr;
  a.host_keys = any_spill ? c->qkeys.as<uint64_t>() : nullptr;
  a.host_count = c->qcount.as<uint32_t>();
  {
    StageTimer t(c, s, KC_T_QUERY);
    KC_HIP(c, launch_query(a, kmers, n, counts, s), "query");
    t.stop();
  }
  KC_HIP(c, hipMemcpyAsync(c->pinned, c->derr.p, 4, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipMemcpyAsync(c->pinned + 1, c->qcount.p, 4, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  const uint32_t errf = (uint32_t)c->pinned[0];
  const uint32_t nhost = (uint32_t)c->pinned[1];
  if (errf & ERR_QUERY_RANGE) {
    resolve_timers(c);
    return fail(c, KC_ERR_INVALID_ARG, "query k-mer code >= 4^k");
  }
  if (nhost) {
    // keys on spilled partitions: probed in the pinned table copies, results
    // scattered back to their rows by one kernel
    const uint32_t nc = c->cfg.n_counters;
    std::vector<uint64_t> q(nhost);
    KC_HIP(c, hipMemcpyAsync(q.data(), c->qkeys.p, nhost * 8ull, hipMemcpyDeviceToHost, s), "readback");
    KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
    std::vector<uint32_t> res((size_t)nhost * nc, 0);
    for (uint32_t i = 0; i < nhost; ++i) {
      const uint64_t x = q[i];
      const uint32_t p = (uint32_t)(host_mix64(x ^ c->hc.salt[0]) >> (64 - c->p_log2));
      const int32_t d = c->spill_of[p];
      if (d >= 0) host_probe(c, c->spill_dir[d], x, &res[(size_t)i * nc]);
    }
    DevBuf vals;
    ReleaseOnExit free_vals{&vals};
    KC_HIP(c, vals.ensure(res.size() * 4), "query results");
    KC_HIP(c, hipMemcpyAsync(vals.p, res.data(), res.size() * 4, hipMemcpyHostToDevice, s), "results");
    KC_HIP(c, launch_scatter_rows(c->qrows.as<uint32_t>(), vals.as<uint32_t>(), nhost, nc, counts, s),
           "scatter");
    KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  }
  resolve_timers(c);
  return KC_OK;
}


kc_status kc_filter_reads(kc_ctx* c, const uint8_t* bases, const uint64_t* offsets,
                          uint64_t n_reads, uint64_t total_bases, uint32_t tumour_min,
                          uint32_t normal_max, uint32_t* out, void* hip_stream) {
  if (!c) return KC_ERR_INVALID_ARG;
  kc_status r = filter_checks(c, bases, offsets, n_reads, total_bases, out);
  if (r != KC_OK || n_reads == 0) return r;
  hipStream_t s = as_stream(hip_stream);
  kc::AllocStream alloc_on(s);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  const uint64_t nwords = (total_bases + 31) / 32;
  DevBuf packed, flags, hit, fkeys;
  ReleaseOnExit free_bufs{&packed, &flags, &hit, &fkeys};
  KC_HIP(c, packed.ensure(nwords * 8), "packed buffer");
  KC_HIP(c, flags.ensure(nwords * 8), "flag buffer");
  KC_HIP(c, hit.ensure(nwords * 4), "window bitmap");
  // marking the slots reads every table once (8 + 4 n_counters bytes a slot,
  // 8 written); it pays when the windows outnumber half the slots, since a
  // marked lookup skips a random count line
  // a marked copy that does not fit leaves the direct probe (same results)
  const uint64_t nslots = (uint64_t)c->pool_slots * c->cap;
  if (total_bases >= nslots / 2) (void)fkeys.ensure(nslots * 8);
  return filter_run(c, bases, offsets, n_reads, total_bases, tumour_min, normal_max, out, s,
                    packed.as<uint64_t>(), flags.as<uint64_t>(), hit.as<uint32_t>(), true,
                    fkeys.as<uint64_t>());
}

kc_status kc_filter_reads_noalloc(kc_ctx* c, const uint8_t* bases, const uint64_t* offsets,
                                  uint64_t n_reads, uint64_t total_bases, uint32_t tumour_min,
                                  uint32_t normal_max, uint32_t* out, void* hip_stream) {
  if (!c) return KC_ERR_INVALID_ARG;
  kc_status r = filter_checks(c, bases, offsets, n_reads, total_bases, out);
  if (r != KC_OK || n_reads == 0) return r;
  if (total_bases > KC_FILTER_NOALLOC_MAX_BASES)
    return fail(c, KC_ERR_INVALID_ARG,
                "more bases than the allocation-free filter's scratch holds (" +
                    std::to_string((unsigned long long)KC_FILTER_NOALLOC_MAX_BASES) + ")");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  void* base = nullptr;
  std::string why;
  r = noalloc_scratch(c->device, &base, &why);
  if (r != KC_OK) return fail(c, r, why);
  uint8_t* p = static_cast<uint8_t*>(base);
  return filter_run(c, bases, offsets, n_reads, total_bases, tumour_min, normal_max, out,
                    as_stream(hip_stream), reinterpret_cast<uint64_t*>(p + kNaPackedOff),
                    reinterpret_cast<uint64_t*>(p + kNaFlagsOff),
                    reinterpret_cast<uint32_t*>(p + kNaHitOff), false, nullptr);
}

// ------------------------------------------------------------ checkpoints
//
// File layout (little endian): a reserved area at the start holding the
// header and one record per partition table {partition, stale, byte offset,
// entries}, then every partition table in partition order (cap keys, then
// cap * n_counters counts), the two Bloom levels and the overflow table.

namespace {

constexpr char kCkptMagic[8] = {'K', 'C', 'C', 'K', 'P', 'T', 0, 1};

struct CkptHeader {
  char magic[8];
  uint32_t abi_version;
  uint32_t reserved_;
  uint64_t header_bytes;  // the reserved area: this header and the records
  kc_config cfg;
  uint32_t p_log2, cap, n_counters, ovf_log2;
  uint64_t n_parts, bloom_words64;
  uint64_t records_offset, b1_offset, b2_offset, ovf_keys_offset, ovf_counts_offset, file_bytes;
  kc_stats stats;
};

struct CkptRecord {
  uint32_t partition;
  uint32_t stale;
  uint64_t offset;   // bytes from the start of the file
  uint64_t entries;  // keys with a count at or above min_count
};

struct FileCloser {
  FILE* f = nullptr;
  ~FileCloser() {
    if (f) fclose(f);
  }
};

bool write_all(FILE* f, const void* p, size_t n) { return n == 0 || fwrite(p, 1, n, f) == n; }
bool read_all(FILE* f, void* p, size_t n) { return n == 0 || fread(p, 1, n, f) == n; }

}  // namespace

kc_status kc_checkpoint(kc_ctx* c, const char* path) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "checkpoint before finalize");
  if (!path || !*path) return fail(c, KC_ERR_INVALID_ARG, "path is empty");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  KC_HIP(c, hipDeviceSynchronize(), "synchronise");
  const uint32_t nc = c->cfg.n_counters;
  const uint64_t cap = c->cap, P = 1ull << c->p_log2, R = c->pool_slots;
  const uint64_t on = 1ull << c->ovf_log2, words = c->bloom_words64;
  // HBM copies: the resident tables, the overflow table, both Bloom levels
  std::vector<uint64_t> tk(R * cap), ok(on), b1(words), b2(words);
  std::vector<uint32_t> tc(R * cap * nc), oc(on * nc);
  KC_HIP(c, hipMemcpy(tk.data(), c->tkeys.p, tk.size() * 8, hipMemcpyDeviceToHost), "checkpoint copy");
  KC_HIP(c, hipMemcpy(tc.data(), c->tcounts.p, tc.size() * 4, hipMemcpyDeviceToHost), "checkpoint copy");
  KC_HIP(c, hipMemcpy(ok.data(), c->okeys.p, on * 8, hipMemcpyDeviceToHost), "checkpoint copy");
  KC_HIP(c, hipMemcpy(oc.data(), c->ocounts.p, on * 4 * nc, hipMemcpyDeviceToHost), "checkpoint copy");
  KC_HIP(c, hipMemcpy(b1.data(), c->b1.p, words * 8, hipMemcpyDeviceToHost), "checkpoint copy");
  KC_HIP(c, hipMemcpy(b2.data(), c->b2.p, words * 8, hipMemcpyDeviceToHost), "checkpoint copy");
  resolve_timers(c);
  CkptHeader h{};
  memcpy(h.magic, kCkptMagic, 8);
  h.abi_version = KC_ABI_VERSION;
  h.cfg = c->cfg;
  h.p_log2 = c->p_log2;
  h.cap = (uint32_t)cap;
  h.n_counters = nc;
  h.ovf_log2 = c->ovf_log2;
  h.n_parts = P;
  h.bloom_words64 = words;
  h.records_offset = sizeof(CkptHeader);
  h.header_bytes = (sizeof(CkptHeader) + P * sizeof(CkptRecord) + 4095) / 4096 * 4096;
  h.stats = c->st;
  const uint64_t table_bytes = cap * 8 + cap * 4 * nc;
  h.b1_offset = h.header_bytes + P * table_bytes;
  h.b2_offset = h.b1_offset + words * 8;
  h.ovf_keys_offset = h.b2_offset + words * 8;
  h.ovf_counts_offset = h.ovf_keys_offset + on * 8;
  h.file_bytes = h.ovf_counts_offset + on * 4 * nc;
  const std::string tmp = std::string(path) + ".tmp";
  FileCloser fc;
  fc.f = fopen(tmp.c_str(), "wb");
  if (!fc.f) return fail(c, KC_ERR_INVALID_ARG, "cannot open " + tmp + " for writing");
  std::vector<CkptRecord> recs(P);
  std::vector<char> pad(h.header_bytes, 0);
  bool ok_io = write_all(fc.f, pad.data(), pad.size());
  for (uint64_t u = 0; u < P && ok_io; ++u) {
    const uint64_t* keys;
    const uint32_t* counts;
    if (c->slot_of_h[u] != kNoSlot) {
      keys = tk.data() + (uint64_t)c->slot_of_h[u] * cap;
      counts = tc.data() + (uint64_t)c->slot_of_h[u] * cap * nc;
    } else {
      const SpillRec& rec = c->spill_dir[c->spill_of[u]];
      keys = c->spill_keys + rec.host_offset;
      counts = c->spill_counts + rec.host_offset * nc;
    }
    uint64_t entries = 0;
    for (uint64_t i = 0; i < cap; ++i) {
      uint32_t any = 0;
      for (uint32_t t = 0; t < nc; ++t) any |= counts[i * nc + t];
      entries += keys[i] != kEmpty && any;
    }
    recs[u] = CkptRecord{(uint32_t)u, 0u, h.header_bytes + u * table_bytes, entries};
    ok_io = write_all(fc.f, keys, cap * 8) && write_all(fc.f, counts, cap * 4 * nc);
  }
  ok_io = ok_io && write_all(fc.f, b1.data(), words * 8) && write_all(fc.f, b2.data(), words * 8) &&
          write_all(fc.f, ok.data(), on * 8) && write_all(fc.f, oc.data(), on * 4 * nc) &&
          fseek(fc.f, 0, SEEK_SET) == 0 && write_all(fc.f, &h, sizeof(h)) &&
          write_all(fc.f, recs.data(), P * sizeof(CkptRecord)) && fflush(fc.f) == 0;
  const bool closed = fclose(fc.f) == 0;
  fc.f = nullptr;
  if (!ok_io || !closed || rename(tmp.c_str(), path) != 0) {
    (void)remove(tmp.c_str());
    return fail(c, KC_ERR_INVALID_ARG, std::string("writing the checkpoint ") + path + " failed");
  }
  return KC_OK;
}

// kc_restore's body.  `made` tracks the context it created and has neither
// destroyed nor handed out, so that kc_restore can free it when a host
// allocation throws.
static kc_status restore_file(const char* path, int device, kc_ctx** out, kc_ctx** made) {
  *out = nullptr;
  if (!path) {
    g_create_error = "path is NULL";
    return KC_ERR_INVALID_ARG;
  }
  FileCloser fc;
  fc.f = fopen(path, "rb");
  if (!fc.f) {
    g_create_error = std::string("cannot open ") + path;
    return KC_ERR_INVALID_ARG;
  }
  CkptHeader h{};
  auto bad = [](const std::string& why) {
    g_create_error = "not a usable checkpoint: " + why;
    return KC_ERR_INVALID_ARG;
  };
  if (!read_all(fc.f, &h, sizeof(h))) return bad("short header");
  if (memcmp(h.magic, kCkptMagic, 8) != 0) return bad("bad magic");
  if (h.abi_version != KC_ABI_VERSION) return bad("written by another ABI version");
  if (h.n_counters < 1 || h.n_counters > 2 || h.p_log2 > (uint32_t)kMaxPartLog2 ||
      h.n_parts != (1ull << h.p_log2) || h.cap < 64 || h.ovf_log2 < 12 || h.ovf_log2 > 34)
    return bad("inconsistent sizes");
  const uint32_t nc = h.n_counters;
  const uint64_t cap = h.cap, P = h.n_parts, on = 1ull << h.ovf_log2;
  const uint64_t table_bytes = cap * 8 + cap * 4 * nc;
  if (h.records_offset != sizeof(CkptHeader) ||
      h.header_bytes < sizeof(CkptHeader) + P * sizeof(CkptRecord) ||
      h.b1_offset != h.header_bytes + P * table_bytes ||
      h.file_bytes != h.b1_offset + 2 * h.bloom_words64 * 8 + on * 8 + on * 4 * nc)
    return bad("inconsistent offsets");
  // every size below comes from the header: check it against the file first
  struct stat fst;
  if (fstat(fileno(fc.f), &fst) != 0 || (uint64_t)fst.st_size != h.file_bytes)
    return bad("file size differs from its header");
  std::vector<CkptRecord> recs(P);
  if (!read_all(fc.f, recs.data(), P * sizeof(CkptRecord))) return bad("short record area");
  for (uint64_t u = 0; u < P; ++u)
    if (recs[u].partition != u || recs[u].stale || recs[u].offset != h.header_bytes + u * table_bytes)
      return bad("inconsistent record");
  // the tables start after the reserved area
  if (fseek(fc.f, (long)h.header_bytes, SEEK_SET) != 0) return bad("short reserved area");
  kc_config cfg = h.cfg;
  cfg.partitions_log2 = h.p_log2;
  cfg.table_slots = h.cap;
  kc_ctx* c = nullptr;
  kc_status r = kc_create(&cfg, device, &c);
  if (r != KC_OK) return r;
  *made = c;
  auto give_up = [&](kc_status st, const std::string& why) {
    g_create_error = why;
    *made = nullptr;
    kc_destroy(c);
    return st;
  };
  if (c->p_log2 != h.p_log2 || c->cap != cap || c->bloom_words64 != h.bloom_words64)
    return give_up(KC_ERR_INVALID_ARG, "not a usable checkpoint: layout differs from its configuration");
  const uint64_t budget = c->cfg.hbm_table_budget_bytes, per_table = cap * c->slot_bytes;
  const uint64_t R = budget ? std::min<uint64_t>(P, budget / per_table) : P;
  const uint64_t n_spill = P - R;
  if (R == 0) return give_up(KC_ERR_OVER_BUDGET, "table budget smaller than one partition table");
  hipError_t e;
  auto hip_ok = [&](hipError_t x) { return (e = x) == hipSuccess; };
  c->pool_slots = (uint32_t)R;
  c->ovf_log2 = h.ovf_log2;
  if (!hip_ok(c->tkeys.ensure(R * cap * 8)) || !hip_ok(c->tcounts.ensure(R * cap * 4 * nc)) ||
      !hip_ok(c->slot_of.ensure(P * 4)) || !hip_ok(c->slot_live.ensure(R * 4)) ||
      !hip_ok(c->okeys.ensure(on * 8)) || !hip_ok(c->ocounts.ensure(on * 4 * nc)))
    return give_up(KC_ERR_OUT_OF_MEMORY, "restore allocation failed");
  free_spill(c);
  if (n_spill && ensure_spill_pool(c, n_spill) != KC_OK)
    return give_up(KC_ERR_OUT_OF_MEMORY, "pinned spill pool allocation failed");
  // tables: the lowest n_spill partitions into the pinned pool, the others to
  // HBM slots u - n_spill, as finalize lays them out under the same budget
  std::vector<char> buf;
  std::vector<uint64_t> hk;
  std::vector<uint32_t> hc;
  const uint64_t batch = std::max<uint64_t>(1, std::min<uint64_t>(R, (256ull << 20) / table_bytes));
  for (uint64_t u = 0; u < P;) {
    if (u < n_spill) {
      if (!read_all(fc.f, c->spill_keys + u * cap, cap * 8) ||
          !read_all(fc.f, c->spill_counts + u * cap * nc, cap * 4 * nc))
        return give_up(KC_ERR_INVALID_ARG, "not a usable checkpoint: short table area");
      add_spill_record(c, (uint32_t)u, u, recs[u].entries);
      ++u;
      continue;
    }
    const uint64_t n = std::min<uint64_t>(batch, P - u);
    buf.resize(n * table_bytes);
    if (!read_all(fc.f, buf.data(), buf.size()))
      return give_up(KC_ERR_INVALID_ARG, "not a usable checkpoint: short table area");
    // slots u - n_spill .. are consecutive: keys and counts of the batch go
    // to HBM in one copy each
    hk.resize(n * cap);
    hc.resize(n * cap * nc);
    for (uint64_t i = 0; i < n; ++i) {
      const char* t = buf.data() + i * table_bytes;
      memcpy(hk.data() + i * cap, t, cap * 8);
      memcpy(hc.data() + i * cap * nc, t + cap * 8, cap * 4 * nc);
    }
    const uint64_t slot = u - n_spill;
    if (!hip_ok(hipMemcpy(c->tkeys.as<uint64_t>() + slot * cap, hk.data(), n * cap * 8,
                          hipMemcpyHostToDevice)) ||
        !hip_ok(hipMemcpy(c->tcounts.as<uint32_t>() + slot * cap * nc, hc.data(), n * cap * 4 * nc,
                          hipMemcpyHostToDevice)))
      return give_up(KC_ERR_DEVICE, "restore copy failed");
    u += n;
  }
  c->spill_used = n_spill;
  // B1, B2 and the overflow table pass through a host buffer of at most 64 MiB
  std::vector<char> stage((size_t)std::min<uint64_t>(64ull << 20, std::max<uint64_t>(h.bloom_words64, on) * 8));
  e = hipSuccess;
  auto section = [&](void* dev, uint64_t bytes) {
    for (uint64_t done = 0; done < bytes;) {
      const uint64_t n = std::min<uint64_t>(bytes - done, stage.size());
      if (!read_all(fc.f, stage.data(), n) ||
          !hip_ok(hipMemcpy(static_cast<char*>(dev) + done, stage.data(), n, hipMemcpyHostToDevice)))
        return false;
      done += n;
    }
    return true;
  };
  const bool ok_io = section(c->b1.p, h.bloom_words64 * 8) && section(c->b2.p, h.bloom_words64 * 8) &&
                     section(c->okeys.p, on * 8) && section(c->ocounts.p, on * 4 * nc);
  if (!ok_io)
    return e != hipSuccess ? give_up(KC_ERR_DEVICE, "restore copy failed")
                           : give_up(KC_ERR_INVALID_ARG, "not a usable checkpoint: short Bloom or overflow area");
  const uint32_t used = (uint32_t)h.stats.overflow_keys;
  if (!hip_ok(hipMemcpy(c->ovf_used.p, &used, 4, hipMemcpyHostToDevice)) ||
      !hip_ok(launch_slot_map(c->slot_of.as<uint32_t>(), (uint32_t)P, (uint32_t)n_spill, nullptr)) ||
      !hip_ok(launch_fill32(c->slot_live.as<uint32_t>(), R, 1, nullptr)) ||
      !hip_ok(hipDeviceSynchronize()))
    return give_up(KC_ERR_DEVICE, "restore setup failed");
  c->slot_of_h.resize(P);
  for (uint64_t u = 0; u < P; ++u) c->slot_of_h[u] = u < n_spill ? kNoSlot : (uint32_t)(u - n_spill);
  c->slot_first = (int64_t)n_spill;
  const uint64_t sp = c->st.spilled_partitions, sb = c->st.spilled_bytes;
  c->st = h.stats;
  c->st.spilled_partitions = sp;
  c->st.spilled_bytes = sb;
  for (int i = 0; i < KC_T_COUNT_OF; ++i) {
    c->st.kernel_ms[i] = 0;
    c->st.kernel_launches[i] = 0;
  }
  c->state = FINALIZED;
  *made = nullptr;
  *out = c;
  return KC_OK;
}

kc_status kc_restore(const char* path, int device, kc_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return KC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  kc_ctx* made = nullptr;
  // host buffers are sized from the file: their failure is an error status,
  // never an exception through the C boundary
  try {
    return restore_file(path, device, out, &made);
  } catch (const std::bad_alloc&) {
    if (made) kc_destroy(made);
    *out = nullptr;
    g_create_error = "host allocation failed while restoring";
    return KC_ERR_OUT_OF_MEMORY;
  }
}

kc_status kc_spill(kc_ctx* c, int64_t partition, uint64_t* bytes_out) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (bytes_out) *bytes_out = 0;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "spill before finalize");
  const uint64_t nparts = 1ull << c->p_log2;
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  hipStream_t s = nullptr;
  if (partition >= 0) {
    if ((uint64_t)partition >= nparts) return fail(c, KC_ERR_INVALID_ARG, "no such partition");
    return spill_partition(c, (uint32_t)partition, s, bytes_out);
  }
  if (partition != -1) return fail(c, KC_ERR_INVALID_ARG, "partition must be >= -1");
  const uint64_t budget = c->cfg.hbm_table_budget_bytes;
  if (!budget) return KC_OK;
  uint64_t held = resident_bytes(c);
  const uint64_t per_table = (uint64_t)c->cap * c->slot_bytes;
  for (int64_t p = (int64_t)nparts - 1; p >= 0 && held > budget; --p) {
    if (c->slot_of_h[p] == kNoSlot) continue;
    kc_status r = spill_partition(c, (uint32_t)p, s, bytes_out);
    if (r != KC_OK) return r;
    held -= per_table;
  }
  return KC_OK;
}

kc_status kc_export(kc_ctx* c, uint64_t* keys, uint32_t* counts, uint64_t cap, uint64_t* n_out) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "export before finalize");
  if (n_out) *n_out = c->st.entries;
  if (!keys) return KC_OK;
  if (!counts) return fail(c, KC_ERR_INVALID_ARG, "counts is NULL");
  if (cap < c->st.entries) return fail(c, KC_ERR_INVALID_ARG, "cap smaller than the entry count");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  const uint32_t nc = c->cfg.n_counters;
  const uint64_t E = c->st.entries;
  DevBuf ok, oc, cur;
  ReleaseOnExit free_bufs{&ok, &oc, &cur};
  KC_HIP(c, ok.ensure(E * 8), "export buffer");
  KC_HIP(c, oc.ensure(E * 4 * nc), "export buffer");
  KC_HIP(c, cur.ensure(8), "export cursor");
  hipStream_t s = nullptr;
  KC_HIP(c, hipMemsetAsync(cur.p, 0, 8, s), "memset");
  const uint64_t nslots = (uint64_t)c->pool_slots * c->cap;
  KC_HIP(c, launch_export(c->tkeys.as<uint64_t>(), c->tcounts.as<uint32_t>(), nslots,
                          c->slot_live.as<uint32_t>(), c->cap, nc, ok.as<uint64_t>(),
                          oc.as<uint32_t>(), E, cur.as<uint64_t>(), s),
         "export");
  KC_HIP(c, launch_export(c->okeys.as<uint64_t>(), c->ocounts.as<uint32_t>(), 1ull << c->ovf_log2,
                          nullptr, 0, nc, ok.as<uint64_t>(), oc.as<uint32_t>(), E,
                          cur.as<uint64_t>(), s),
         "export");
  uint64_t got = 0;
  kc_status r = sync_read(c, s, cur.p, 8, &got);
  if (r != KC_OK) return r;
  uint64_t spilled = 0;
  for (const SpillRec& rec : c->spill_dir) spilled += rec.entries;
  if (got + spilled != E) return fail(c, KC_ERR_DEVICE, "export count mismatch");
  KC_HIP(c, hipMemcpy(keys, ok.p, got * 8, hipMemcpyDeviceToHost), "export copy");
  KC_HIP(c, hipMemcpy(counts, oc.p, got * 4 * nc, hipMemcpyDeviceToHost), "export copy");
  uint64_t at = got;
  for (const SpillRec& rec : c->spill_dir) {
    const uint64_t* tk = c->spill_keys + rec.host_offset;
    const uint32_t* tc = c->spill_counts + rec.host_offset * nc;
    uint64_t taken = 0;
    for (uint64_t i = 0; i < c->cap; ++i) {
      uint32_t any = 0;
      for (uint32_t t = 0; t < nc; ++t) any |= tc[i * nc + t];
      if (tk[i] == kEmpty || !any) continue;
      keys[at] = tk[i];
      for (uint32_t t = 0; t < nc; ++t) counts[at * nc + t] = tc[i * nc + t];
      ++at;
      ++taken;
    }
    if (taken != rec.entries) return fail(c, KC_ERR_DEVICE, "spilled partition entry count mismatch");
  }
  return KC_OK;
}

// Stem items of the final table in three passes over its live slots (resident
// tables, the overflow table, and spilled tables staged back in batches):
// claim each k-mer's canonical stem in a device hash table, number the
// claimed slots by a prefix sum (writing the stems out), then store every
// k-mer's counts in its stem's item.
kc_status kc_export_stems(kc_ctx* c, uint64_t* stems, uint16_t* items, uint64_t capacity,
                          uint64_t* n_out, void* hip_stream) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "stem export before finalize");
  if (!n_out) return fail(c, KC_ERR_INVALID_ARG, "n_out is NULL");
  if (c->cfg.k < 3) return fail(c, KC_ERR_INVALID_ARG, "stems need k >= 3");
  if (reinterpret_cast<uintptr_t>(items) & 3u)
    return fail(c, KC_ERR_INVALID_ARG, "counts_dev must be 4-byte aligned");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  AllocStream alloc_on(s);
  StageTimer tm(c, s, KC_T_STEMS);
  const uint32_t nc = c->cfg.n_counters, k = c->cfg.k;
  const uint64_t E = c->st.entries, cap = c->cap;
  DevBuf pcount, poff, parts, cursor, rstem, rcnt, err, icur, stage_k, stage_c;
  ReleaseOnExit free_bufs{&pcount, &poff, &parts, &cursor, &rstem, &rcnt, &err, &icur,
                          &stage_k, &stage_c};
  KC_HIP(c, err.ensure(4), "error flag");
  KC_HIP(c, icur.ensure(8), "item cursor");
  KC_HIP(c, launch_fill32(err.as<uint32_t>(), 1, 0, s), "fill");
  // spilled tables come back to HBM in batches of up to kStage tables
  const uint64_t kStage = std::max<uint64_t>(1, std::min<uint64_t>(c->spill_used, 2048));
  if (c->spill_used) {
    KC_HIP(c, stage_k.ensure(kStage * cap * 8), "staging buffer");
    KC_HIP(c, stage_c.ensure(kStage * cap * 4 * nc), "staging buffer");
  }
  // fn(keys, counts, slots, live) over every table: resident, overflow, spilled
  auto sources = [&](auto&& fn) -> kc_status {
    hipError_t e;
    if ((e = fn(c->tkeys.as<uint64_t>(), c->tcounts.as<uint32_t>(), (uint64_t)c->pool_slots * cap,
                c->slot_live.as<uint32_t>())) != hipSuccess)
      return hip_fail(c, e, "stem pass");
    if ((e = fn(c->okeys.as<uint64_t>(), c->ocounts.as<uint32_t>(), 1ull << c->ovf_log2,
                nullptr)) != hipSuccess)
      return hip_fail(c, e, "stem pass");
    for (uint64_t t0 = 0; t0 < c->spill_used; t0 += kStage) {
      const uint64_t nt = std::min<uint64_t>(kStage, c->spill_used - t0);
      KC_HIP(c, hipMemcpyAsync(stage_k.p, c->spill_keys + t0 * cap, nt * cap * 8,
                               hipMemcpyHostToDevice, s),
             "stage copy");
      KC_HIP(c, hipMemcpyAsync(stage_c.p, c->spill_counts + t0 * cap * nc, nt * cap * 4 * nc,
                               hipMemcpyHostToDevice, s),
             "stage copy");
      if ((e = fn(stage_k.as<uint64_t>(), stage_c.as<uint32_t>(), nt * cap, nullptr)) != hipSuccess)
        return hip_fail(c, e, "stem pass");
    }
    return KC_OK;
  };
  // stem partitions of at most stem_part_max() entries: about 1536 on average,
  // doubled until the largest one fits
  uint32_t p_log2 = 0;
  while (p_log2 < 24 && (E >> p_log2) > 1536) ++p_log2;
  kc_status r;
  uint64_t P;
  std::vector<uint32_t> hc;
  for (;;) {
    P = 1ull << p_log2;
    KC_HIP(c, pcount.ensure(P * 4), "stem partition counts");
    KC_HIP(c, launch_fill32(pcount.as<uint32_t>(), P, 0, s), "fill");
    r = sources([&](const uint64_t* tk, const uint32_t* tcn, uint64_t n, const uint32_t* live) {
      return launch_stem_count(tk, tcn, n, live, (uint32_t)cap, nc, k, p_log2,
                               pcount.as<uint32_t>(), s);
    });
    if (r != KC_OK) return r;
    hc.resize(P);
    if ((r = sync_read(c, s, pcount.p, P * 4, hc.data())) != KC_OK) return r;
    const uint32_t most = *std::max_element(hc.begin(), hc.end());
    if (most <= stem_part_max()) break;
    if (p_log2 >= 24) return fail(c, KC_ERR_DEVICE, "stem partitions stay too large");
    ++p_log2;
  }
  KC_HIP(c, poff.ensure((P + 1) * 8), "stem partition offsets");
  KC_HIP(c, parts.ensure(scan_parts(P) * 8), "scan buffer");
  KC_HIP(c, launch_scan(pcount.as<uint32_t>(), P, poff.as<uint64_t>(), parts.as<uint64_t>(), s),
         "stem scan");
  uint64_t R = 0;
  if ((r = sync_read(c, s, poff.as<uint64_t>() + P, 8, &R)) != KC_OK) return r;
  KC_HIP(c, cursor.ensure(P * 8), "stem cursors");
  KC_HIP(c, hipMemcpyAsync(cursor.p, poff.p, P * 8, hipMemcpyDeviceToDevice, s), "cursor copy");
  KC_HIP(c, rstem.ensure(std::max<uint64_t>(1, R) * 8), "stem records");
  KC_HIP(c, rcnt.ensure(std::max<uint64_t>(1, R) * 4), "stem records");
  r = sources([&](const uint64_t* tk, const uint32_t* tcn, uint64_t n, const uint32_t* live) {
    return launch_stem_scatter(tk, tcn, n, live, (uint32_t)cap, nc, k, p_log2,
                               cursor.as<uint64_t>(), rstem.as<uint64_t>(), rcnt.as<uint32_t>(), s);
  });
  if (r != KC_OK) return r;
  // the item count first when the caller's capacity might not hold it
  uint64_t n = 0;
  if (capacity < E || !stems || !items) {
    KC_HIP(c, launch_fill64(icur.as<uint64_t>(), 1, 0, s), "fill");
    KC_HIP(c, launch_stem_group(poff.as<uint64_t>(), P, rstem.as<uint64_t>(), rcnt.as<uint32_t>(),
                                true, icur.as<uint64_t>(), 0, nullptr, nullptr,
                                err.as<uint32_t>(), s),
           "stem count");
    if ((r = sync_read(c, s, icur.p, 8, &n)) != KC_OK) return r;
    *n_out = n;
    if (n > E) return fail(c, KC_ERR_DEVICE, "more stems than table entries");
    if (n > capacity) return fail(c, KC_ERR_INVALID_ARG, "capacity smaller than the stem count");
    if (n && (!stems || !items)) return fail(c, KC_ERR_INVALID_ARG, "stems_dev or counts_dev is NULL");
    if (n == 0) {
      tm.stop();
      return KC_OK;
    }
  }
  KC_HIP(c, launch_fill64(icur.as<uint64_t>(), 1, 0, s), "fill");
  KC_HIP(c, launch_stem_group(poff.as<uint64_t>(), P, rstem.as<uint64_t>(), rcnt.as<uint32_t>(),
                              false, icur.as<uint64_t>(), capacity, stems, items,
                              err.as<uint32_t>(), s),
         "stem items");
  if ((r = sync_read(c, s, icur.p, 8, &n)) != KC_OK) return r;
  *n_out = n;
  uint32_t e = 0;
  if ((r = sync_read(c, s, err.p, 4, &e)) != KC_OK) return r;
  tm.stop();
  if (e) return fail(c, KC_ERR_DEVICE, "stem partition table overflow");
  if (n > E) return fail(c, KC_ERR_DEVICE, "more stems than table entries");
  return KC_OK;
}

kc_status kc_export_bloom(kc_ctx* c, uint64_t* b1, uint64_t* b2, uint64_t words) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "Bloom export before finalize");
  if (words != c->bloom_words64) return fail(c, KC_ERR_INVALID_ARG, "words must equal the Bloom size / 64");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  if (b1) KC_HIP(c, hipMemcpy(b1, c->b1.p, words * 8, hipMemcpyDeviceToHost), "Bloom copy");
  if (b2) KC_HIP(c, hipMemcpy(b2, c->b2.p, words * 8, hipMemcpyDeviceToHost), "Bloom copy");
  return KC_OK;
}

kc_status kc_export_bloom_words(kc_ctx* c, const uint64_t* word_idx, uint64_t n, uint64_t* b1,
                                uint64_t* b2) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != FINALIZED) return fail(c, KC_ERR_BAD_STATE, "Bloom export before finalize");
  if (n == 0) return KC_OK;
  if (!word_idx || !b1 || !b2) return fail(c, KC_ERR_INVALID_ARG, "NULL index or output buffer");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  DevBuf idx, out;
  ReleaseOnExit free_bufs{&idx, &out};
  KC_HIP(c, idx.ensure(n * 8), "index buffer");
  KC_HIP(c, out.ensure(n * 16), "gather buffer");
  KC_HIP(c, hipMemcpy(idx.p, word_idx, n * 8, hipMemcpyHostToDevice), "index copy");
  KC_HIP(c, hipMemset(c->derr.p, 0, 4), "memset");
  KC_HIP(c, launch_gather2(c->b1.as<uint64_t>(), c->b2.as<uint64_t>(), idx.as<uint64_t>(), n,
                           c->bloom_words64, out.as<uint64_t>(), out.as<uint64_t>() + n,
                           c->derr.as<uint32_t>(), nullptr),
         "gather");
  uint32_t errf = 0;
  KC_HIP(c, hipMemcpy(&errf, c->derr.p, 4, hipMemcpyDeviceToHost), "readback");
  if (errf & ERR_QUERY_RANGE) return fail(c, KC_ERR_INVALID_ARG, "word index past the Bloom size");
  KC_HIP(c, hipMemcpy(b1, out.p, n * 8, hipMemcpyDeviceToHost), "Bloom copy");
  KC_HIP(c, hipMemcpy(b2, out.as<uint64_t>() + n, n * 8, hipMemcpyDeviceToHost), "Bloom copy");
  return KC_OK;
}

kc_status kc_debug_keys(kc_ctx* c, uint64_t* keys, uint32_t* part, uint64_t cap, uint64_t* n_out) {
  if (!c) return KC_ERR_INVALID_ARG;
  uint64_t n = 0;
  for (const Segment& g : c->segs) n += g.n;
  if (n_out) *n_out = n;
  if (!keys) return KC_OK;
  if (cap < n) return fail(c, KC_ERR_INVALID_ARG, "cap smaller than the stored key count");
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  KC_HIP(c, hipDeviceSynchronize(), "synchronise");
  uint64_t at = 0;
  for (const Segment& g : c->segs) {
    KC_HIP(c, hipMemcpy(keys + at, g.keys.p, g.n * 8, hipMemcpyDeviceToHost), "key copy");
    if (part) {
      DevBuf pb;
      ReleaseOnExit free_pb{&pb};
      KC_HIP(c, pb.ensure(g.n * 4), "partition buffer");
      SegDesc sd{g.keys.as<uint64_t>(), g.bucket_off.as<uint64_t>(), g.tile_first.as<uint32_t>(),
                 g.meta2.as<uint32_t>(), c->a1, c->a2, c->t2_log2, 0};
      KC_HIP(c, launch_debug_part(sd, g.n, pb.as<uint32_t>(), nullptr), "partition view");
      KC_HIP(c, hipMemcpy(part + at, pb.p, g.n * 4, hipMemcpyDeviceToHost), "partition copy");
    }
    at += g.n;
  }
  return KC_OK;
}

kc_status kc_get_stats(const kc_ctx* cc, kc_stats* out) {
  if (!cc || !out) return KC_ERR_INVALID_ARG;
  kc_ctx* c = const_cast<kc_ctx*>(cc);
  resolve_timers(c);
  *out = c->st;
  return KC_OK;
}

kc_status kc_reset(kc_ctx* c) {
  if (!c) return KC_ERR_INVALID_ARG;
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  // every other call has finished its device work before returning; only the
  // last insert's shuffle may still be queued
  if (c->insert_done_valid) KC_HIP(c, hipEventSynchronize(c->insert_done), "synchronise");
  if (!c->segs_borrowed)
    for (Segment& g : c->segs) c->spare_segs.push_back(g);
  c->segs.clear();
  c->segs_borrowed = false;
  // keep at most a few spare segment allocations
  std::sort(c->spare_segs.begin(), c->spare_segs.end(),
            [](const Segment& a, const Segment& b) { return a.keys.bytes > b.keys.bytes; });
  while (c->spare_segs.size() > 4) {
    c->spare_segs.back().release();
    c->spare_segs.pop_back();
  }
  free_spill(c);
  resolve_timers(c);
  const uint32_t pl = c->p_log2, tl = c->cap;
  c->st = kc_stats{};
  c->st.partitions_log2 = pl;
  c->st.table_slots = tl;
  c->insert_done_valid = false;
  c->state = CREATED;
  c->err.clear();
  return KC_OK;
}

void kc_destroy(kc_ctx* c) {
  if (!c) return;
  if (!kc::t_async) {
    // buffers from stream-ordered calls are freed in order on the null stream
    kc::AllocStream alloc_on(nullptr);
    kc_destroy(c);
    return;
  }
  (void)hipSetDevice(c->device);
  // only the last insert may still be queued (every other call has finished)
  if (c->insert_done_valid) (void)hipEventSynchronize(c->insert_done);
  if (!c->segs_borrowed)
    for (Segment& g : c->segs) g.release();
  for (Segment& g : c->spare_segs) g.release();
  c->batch.release();
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  DevBuf* bufs[] = {&c->b1, &c->b2, &c->dstat, &c->derr, &c->packed, &c->flags, &c->hist1,
                    &c->lstart1, &c->off1, &c->parts, &c->keys1, &c->tile_desc, &c->segdesc,
                    &c->tkeys, &c->tcounts, &c->slot_of, &c->slot_live, &c->pstats, &c->pstats2,
                    &c->pstats_ovf, &c->okeys, &c->ocounts, &c->ovf_used, &c->qrows, &c->qkeys,
                    &c->qcount};
  for (DevBuf* b : bufs) b->release();
  release_spill_pool(c);
  for (int b = 0; b < 2; ++b) {
    if (c->ev_tally[b]) (void)hipEventDestroy(c->ev_tally[b]);
    if (c->ev_copy[b]) (void)hipEventDestroy(c->ev_copy[b]);
  }
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  for (auto& t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->insert_done) (void)hipEventDestroy(c->insert_done);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}


// ------------------------------------------------------------ batched form

namespace {

bool same_batch(const BatchPlan& b, const kc_chunk* ch, uint32_t n, uint32_t counter) {
  if (!b.exec || b.counter != counter || b.chunks.size() != n) return false;
  for (uint32_t i = 0; i < n; ++i) {
    const kc_chunk& a = b.chunks[i];
    if (a.bases_dev != ch[i].bases_dev || a.offsets_dev != ch[i].offsets_dev ||
        a.n_reads != ch[i].n_reads || a.total_bases != ch[i].total_bases)
      return false;
  }
  return true;
}

// Groups the chunks into segments, sizes every buffer for the largest
// possible key count (every position a key), and captures the graph: per
// segment pack, read starts, first level, scan, second level; then the Bloom
// levels, the count, Unify and the slot map.  Fills replace memsets.
kc_status build_batch(kc_ctx* c, const kc_chunk* ch, uint32_t n, uint32_t counter) {
  c->batch.release();
  BatchPlan& b = c->batch;
  const uint64_t limit = c->cfg.group_bases_log2 ? (1ull << c->cfg.group_bases_log2)
                                                 : (1ull << 32) - 64;
  std::vector<std::vector<ChunkDesc>> descs;
  {
    std::vector<ChunkDesc> d;
    uint64_t words = 0, slots = 0;
    uint32_t c0 = 0;
    auto close = [&](uint32_t end) {
      BatchGroup g;
      g.c0 = c0;
      g.nc = end - c0;
      g.nwords = words;
      g.nslots = slots;
      b.groups.push_back(g);
      descs.push_back(d);
      d.clear();
      words = slots = 0;
      c0 = end;
    };
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t w = (ch[i].total_bases + 31) / 32;
      if (w * 32 > limit) return fail(c, KC_ERR_INVALID_ARG, "a chunk holds more bases than a segment");
      if (!d.empty() && (words + w) * 32 > limit) close(i);
      ChunkDesc cd{ch[i].bases_dev, ch[i].offsets_dev, ch[i].total_bases, ch[i].n_reads, words, slots};
      d.push_back(cd);
      words += w;
      slots += ch[i].n_reads + 1;
    }
    if (!d.empty()) close(n);
  }
  const uint32_t nb1 = 1u << c->a1, nb2 = 1u << c->a2;
  uint64_t max_words = 0, max_tiles = 0, max_hist = 0, max_tiles2 = 0, bound_total = 0;
  for (BatchGroup& g : b.groups) {
    g.ntiles = (g.nwords + kTileWords - 1) / kTileWords;
    g.nhist = (uint64_t)nb1 * g.ntiles;
    const uint64_t bound = g.nwords * 32;  // keys <= positions
    g.tiles2 = ((bound + (1ull << c->t2_log2) - 1) >> c->t2_log2) + nb1;
    max_words = std::max(max_words, g.nwords);
    max_tiles = std::max(max_tiles, g.ntiles);
    max_hist = std::max(max_hist, g.nhist);
    max_tiles2 = std::max(max_tiles2, g.tiles2);
    bound_total += bound;
  }
  // shared first-level scratch, per-segment outputs, chunk tables
  KC_HIP(c, c->packed.ensure(max_words * 8), "packed buffer");
  KC_HIP(c, c->flags.ensure(max_words * 8), "flag buffer");
  KC_HIP(c, c->hist1.ensure(max_hist * 4), "histogram buffer");
  KC_HIP(c, c->lstart1.ensure(max_tiles * (nb1 + 1) * 4), "tile start buffer");
  KC_HIP(c, c->off1.ensure((max_hist + 1) * 8), "offset buffer");
  KC_HIP(c, c->parts.ensure(scan_parts(max_hist) * 8), "scan buffer");
  KC_HIP(c, c->keys1.ensure(max_tiles * kTilePos * 8), "first-level key buffer");
  KC_HIP(c, c->tile_desc.ensure(tile_desc_bytes(max_tiles2)), "tile descriptor buffer");
  KC_HIP(c, b.counts.ensure(std::max<size_t>(1, b.groups.size()) * 8), "segment counts");
  std::vector<SegDesc> hd;
  for (size_t gi = 0; gi < b.groups.size(); ++gi) {
    BatchGroup& g = b.groups[gi];
    KC_HIP(c, g.cdesc.ensure(std::max<size_t>(1, g.nc) * sizeof(ChunkDesc)), "chunk table");
    if (g.nc)
      KC_HIP(c, hipMemcpy(g.cdesc.p, descs[gi].data(), g.nc * sizeof(ChunkDesc), hipMemcpyHostToDevice),
             "chunk table copy");
    if (!g.nwords) continue;
    hipError_t e;
    if ((e = g.seg.keys.ensure(g.nwords * 32 * 8)) != hipSuccess ||
        (e = g.seg.bucket_off.ensure((nb1 + 1) * 8)) != hipSuccess ||
        (e = g.seg.tile_first.ensure((nb1 + 1) * 4)) != hipSuccess ||
        (e = g.seg.meta2.ensure(g.tiles2 * (nb2 + 1) * 4)) != hipSuccess)
      return hip_fail(c, e, "segment allocation");
    g.seg.counter = counter;
    SegDesc sd;
    sd.keys = g.seg.keys.as<uint64_t>();
    sd.bucket_off = g.seg.bucket_off.as<uint64_t>();
    sd.tile_first = g.seg.tile_first.as<uint32_t>();
    sd.meta2 = g.seg.meta2.as<uint32_t>();
    sd.a1 = c->a1;
    sd.a2 = c->a2;
    sd.t2_log2 = c->t2_log2;
    hd.push_back(sd);
  }
  KC_HIP(c, c->segdesc.ensure(std::max<size_t>(1, hd.size()) * sizeof(SegDesc)), "segment table");
  if (!hd.empty())
    KC_HIP(c, hipMemcpy(c->segdesc.p, hd.data(), hd.size() * sizeof(SegDesc), hipMemcpyHostToDevice),
           "segment table copy");
  // count buffers: every table resident
  const uint64_t nparts = 1ull << c->p_log2, cap = c->cap, nc = c->cfg.n_counters;
  c->pool_slots = (uint32_t)nparts;
  KC_HIP(c, c->tkeys.ensure(nparts * cap * 8), "table allocation");
  KC_HIP(c, c->tcounts.ensure(nparts * cap * 4 * nc), "table allocation");
  KC_HIP(c, c->slot_of.ensure(nparts * 4), "slot map");
  KC_HIP(c, c->slot_live.ensure(nparts * 4), "slot map");
  KC_HIP(c, c->pstats.ensure((1ull << c->s_log2) * kNst * 8), "stats rows");
  KC_HIP(c, c->pstats2.ensure(nparts * kNst * 8), "stats rows");
  c->ovf_log2 = std::max<uint32_t>(12, std::min<uint32_t>(30, ceil_log2(bound_total / 256 + 1)));
  const uint64_t on = 1ull << c->ovf_log2;
  const uint32_t oblocks = (uint32_t)std::min<uint64_t>(1024, (on + 255) / 256);
  KC_HIP(c, c->okeys.ensure(on * 8), "overflow table");
  KC_HIP(c, c->ocounts.ensure(on * 4 * nc), "overflow table");
  KC_HIP(c, c->pstats_ovf.ensure((uint64_t)oblocks * kNst * 8), "stats rows");
  KC_HIP(c, hipDeviceSynchronize(), "synchronise");

  if (!c->capture_stream)
    KC_HIP(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking), "capture stream");
  hipStream_t cs = c->capture_stream;
  KC_HIP(c, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
  auto record = [&]() -> hipError_t {
    hipError_t e;
#define KC_REC(x) \
  if ((e = (x)) != hipSuccess) return e
    const uint64_t s0 = c->hc.salt[0];
    const uint64_t tag = (uint64_t)counter << 62;
    KC_REC(launch_fill32(c->derr.as<uint32_t>(), 1, 0, cs));
    for (size_t gi = 0; gi < b.groups.size(); ++gi) {
      BatchGroup& g = b.groups[gi];
      const ChunkDesc* cd = g.cdesc.as<ChunkDesc>();
      KC_REC(launch_pack_batch(cd, g.nc, g.nwords, c->packed.as<uint64_t>(), c->flags.as<uint64_t>(), cs));
      KC_REC(launch_rstart_batch(cd, g.nc, g.nslots, c->flags.as<uint64_t>(), c->derr.as<uint32_t>(), cs));
      if (!g.nwords) {
        KC_REC(launch_fill64(b.counts.as<uint64_t>() + gi, 1, 0, cs));
        continue;
      }
      KC_REC(launch_level1(c->packed.as<uint64_t>(), c->flags.as<uint64_t>(), g.nwords, c->cfg.k, s0,
                           c->a1, tag, c->hist1.as<uint32_t>(), c->lstart1.as<uint32_t>(), g.ntiles,
                           c->keys1.as<uint64_t>(), cs));
      KC_REC(launch_scan(c->hist1.as<uint32_t>(), g.nhist, c->off1.as<uint64_t>(),
                         c->parts.as<uint64_t>(), cs));
      KC_REC(launch_copy64(c->off1.as<uint64_t>() + g.nhist, b.counts.as<uint64_t>() + gi, cs));
      KC_REC(launch_bucket_off(c->off1.as<uint64_t>(), g.ntiles, nb1, g.seg.bucket_off.as<uint64_t>(), cs));
      KC_REC(launch_tiles2(g.seg.bucket_off.as<uint64_t>(), nb1, c->t2_log2,
                           g.seg.tile_first.as<uint32_t>(), cs));
      KC_REC(launch_level2(c->keys1.as<uint64_t>(), c->off1.as<uint64_t>(), c->lstart1.as<uint32_t>(),
                           g.ntiles, g.seg.bucket_off.as<uint64_t>(), g.seg.tile_first.as<uint32_t>(),
                           c->tile_desc.as<uint64_t>(), c->a1, c->a2, c->t2_log2, s0, g.seg.keys.as<uint64_t>(),
                           g.seg.meta2.as<uint32_t>(), g.tiles2, cs));
    }
    KC_REC(launch_fill64(c->okeys.as<uint64_t>(), on, kEmpty, cs));
    KC_REC(launch_fill32(c->ocounts.as<uint32_t>(), on * nc, 0, cs));
    KC_REC(launch_fill32(c->ovf_used.as<uint32_t>(), 1, 0, cs));
    if (c->cfg.bloom_block_log2 < 5) {
      KC_REC(launch_fill64(c->b1.as<uint64_t>(), c->bloom_words64, 0, cs));
      KC_REC(launch_fill64(c->b2.as<uint64_t>(), c->bloom_words64, 0, cs));
    }
    CountArgs a = count_args(c, (uint32_t)hd.size());
    a.part_base = 0;
    a.part_n = (uint32_t)nparts;
    a.slot_base = 0;
    KC_REC(launch_bloom(a, 1u << c->s_log2, c->count_lds, cs));
    KC_REC(launch_tally(a, (uint32_t)nparts, c->tally_lds, cs));
    KC_REC(launch_ovf_emit(a, c->pstats_ovf.as<uint64_t>(), oblocks, cs));
    KC_REC(launch_reduce(c->pstats.as<uint64_t>(), (1ull << c->s_log2) >> c->bsub_log2,
                         c->dstat.as<uint64_t>(), cs));
    KC_REC(launch_reduce(c->pstats_ovf.as<uint64_t>(), oblocks, c->dstat.as<uint64_t>() + kNst, cs));
    KC_REC(launch_reduce(c->pstats2.as<uint64_t>(), nparts, c->dstat.as<uint64_t>() + 2 * kNst, cs));
    KC_REC(launch_slot_map(c->slot_of.as<uint32_t>(), (uint32_t)nparts, 0, cs));
    KC_REC(launch_fill32(c->slot_live.as<uint32_t>(), nparts, 1, cs));
#undef KC_REC
    return hipSuccess;
  };
  const hipError_t rec = record();
  const hipError_t end = hipStreamEndCapture(cs, &b.graph);
  if (rec != hipSuccess) return hip_fail(c, rec, "graph capture");
  if (end != hipSuccess) return hip_fail(c, end, "end capture");
  KC_HIP(c, hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "graph instantiate");
  b.chunks.assign(ch, ch + n);
  b.counter = counter;
  return KC_OK;
}

}  // namespace

kc_status kc_count_batch(kc_ctx* c, const kc_chunk* chunks, uint32_t n_chunks, uint32_t counter,
                         void* hip_stream, kc_stats* out) {
  if (!c) return KC_ERR_INVALID_ARG;
  if (c->state != CREATED) return fail(c, KC_ERR_BAD_STATE, "batch count needs a fresh or reset context");
  if (counter >= c->cfg.n_counters) return fail(c, KC_ERR_INVALID_ARG, "counter >= n_counters");
  if (n_chunks && !chunks) return fail(c, KC_ERR_INVALID_ARG, "chunks is NULL");
  for (uint32_t i = 0; i < n_chunks; ++i) {
    if (!chunks[i].offsets_dev) return fail(c, KC_ERR_INVALID_ARG, "a chunk's offsets are NULL");
    if (chunks[i].total_bases && !chunks[i].bases_dev)
      return fail(c, KC_ERR_INVALID_ARG, "a chunk's bases are NULL");
  }
  const uint64_t nparts = 1ull << c->p_log2;
  const uint64_t per_table = (uint64_t)c->cap * c->slot_bytes;
  if (c->cfg.hbm_table_budget_bytes && c->cfg.hbm_table_budget_bytes < nparts * per_table)
    return fail(c, KC_ERR_OVER_BUDGET, "batch counting keeps every partition table in HBM");
  hipStream_t s = as_stream(hip_stream);
  kc::AllocStream alloc_on(s);
  KC_HIP(c, hipSetDevice(c->device), "hipSetDevice");
  if (!same_batch(c->batch, chunks, n_chunks, counter)) {
    kc_status r = build_batch(c, chunks, n_chunks, counter);
    if (r != KC_OK) {
      c->batch.release();
      return r;
    }
  }
  BatchPlan& b = c->batch;
  free_spill(c);
  {
    StageTimer t(c, s, KC_T_GRAPH);
    KC_HIP(c, hipGraphLaunch(b.exec, s), "graph launch");
    t.stop();
  }
  const size_t ng = b.groups.size();
  std::vector<uint64_t> counts(std::max<size_t>(1, ng), 0);
  if (ng)
    KC_HIP(c, hipMemcpyAsync(counts.data(), b.counts.p, ng * 8, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipMemcpyAsync(c->pinned, c->dstat.p, 3 * kNst * 8, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipMemcpyAsync(c->pinned + 3 * kNst, c->derr.p, 4, hipMemcpyDeviceToHost, s), "readback");
  KC_HIP(c, hipMemcpyAsync(c->pinned + 3 * kNst + 1, c->ovf_used.p, 4, hipMemcpyDeviceToHost, s),
         "readback");
  KC_HIP(c, hipStreamSynchronize(s), "stream synchronise");
  const uint32_t errf = (uint32_t)c->pinned[3 * kNst];
  if (errf & ERR_OFFSETS) {
    resolve_timers(c);
    return fail(c, KC_ERR_INVALID_ARG,
                "offsets must start at 0, be non-decreasing and end at total_bases");
  }
  uint64_t nv = 0;
  c->segs.clear();
  c->segs_borrowed = true;
  for (size_t gi = 0; gi < ng; ++gi) {
    nv += counts[gi];
    if (!b.groups[gi].nwords) continue;
    Segment view = b.groups[gi].seg;  // shallow: the plan owns the memory
    view.n = counts[gi];
    c->segs.push_back(view);
  }
  c->st.n_valid = nv;
  c->st.n_segments = (uint32_t)c->segs.size();
  if (errf & (ERR_OVF_FULL | ERR_OVF_LOAD)) {
    // the overflow table filled up: count again with the eager path, which
    // grows it (and drops this graph, whose buffers it may reallocate)
    c->state = INSERTING;
    return kc_finalize(c, hip_stream, out);
  }
  uint64_t sv[kNst];
  for (int i = 0; i < kNst; ++i) sv[i] = c->pinned[i] + c->pinned[kNst + i] + c->pinned[2 * kNst + i];
  c->st.n_pass = sv[ST_NPASS];
  c->st.entries = sv[ST_ENTRIES];
  c->st.sum_counts = sv[ST_SUM];
  c->st.fp_singletons = sv[ST_FP];
  c->st.b1_popcount = sv[ST_B1POP];
  c->st.b2_popcount = sv[ST_B2POP];
  c->st.passed_distinct = sv[ST_PASSED];
  {
    uint32_t used = 0;
    memcpy(&used, reinterpret_cast<uint8_t*>(c->pinned + 3 * kNst + 1), 4);
    c->st.overflow_keys = used;
  }
  c->st.spilled_partitions = 0;
  c->st.spilled_bytes = 0;
  c->pool_slots = (uint32_t)nparts;
  c->slot_of_h.resize(nparts);
  for (uint64_t u = 0; u < nparts; ++u) c->slot_of_h[u] = (uint32_t)u;
  c->slot_first = 0;
  c->state = FINALIZED;
  resolve_timers(c);
  if (out) *out = c->st;
  return KC_OK;
}

kc_status kc_autotune_batch(const kc_config* base, int device, const kc_chunk* chunks,
                            uint32_t n_chunks, uint32_t counter, void* hip_stream,
                            kc_config* best_out, kc_tune_trial* trials, uint32_t max_trials,
                            uint32_t* n_trials_out) {
  if (n_trials_out) *n_trials_out = 0;
  if (!base || !best_out) {
    g_create_error = "base or best_out is NULL";
    return KC_ERR_INVALID_ARG;
  }
  std::string why;
  if (validate(base, &why) != KC_OK) {
    g_create_error = why;
    return KC_ERR_INVALID_ARG;
  }
  uint64_t positions = 0;
  for (uint32_t i = 0; i < n_chunks; ++i) positions += chunks[i].total_bases;
  const uint32_t s_log2 = base->bloom_bits_log2 - base->bloom_block_log2;
  const uint32_t lo = std::max<uint32_t>(s_log2, 2);  // fewest partitions allowed
  // Coordinate search from about one partition per 2^13 key positions, the
  // default table and the automatic shuffle split: along each dimension in
  // turn, step to a neighbour while that is faster.
  const int64_t pc = (int64_t)std::llround(std::log2((double)std::max<uint64_t>(positions, 1)) - 13.0);
  const uint32_t slot_bytes = 8 + 4 * base->n_counters;
  const uint32_t cap_def =
      (uint32_t)(((size_t)kLdsMax / 3 - kLdsSlack - kQueueBytes) / slot_bytes / 64 * 64);
  // table sizes: the default (three workgroups per CU) and smaller ones in 64-slot steps
  std::vector<uint32_t> slist;
  for (uint32_t f = 10; f >= 5; --f) slist.push_back(std::max<uint32_t>(64, cap_def * f / 10 / 64 * 64));
  std::vector<kc_tune_trial> got;
  // second-level tile sizes (log2 keys), the largest first
  const uint32_t tlist[] = {13, 12, 11};
  struct Key {
    uint32_t p, si, a1, ti;
    bool operator==(const Key& o) const {
      return p == o.p && si == o.si && a1 == o.a1 && ti == o.ti;
    }
  };
  std::vector<std::pair<Key, double>> seen;
  kc_config best = *base;
  double best_ms = 1e300;
  auto run = [&](Key key) -> double {
    for (auto& kv : seen)
      if (kv.first == key) return kv.second;
    kc_config cfg = *base;
    cfg.partitions_log2 = key.p;
    cfg.table_slots = slist[key.si];
    cfg.scatter_bits = key.a1;
    cfg.shuffle_tile_log2 = tlist[key.ti];
    kc_tune_trial t{};
    t.partitions_log2 = key.p;
    t.table_slots = slist[key.si];
    t.scatter_bits = key.a1;
    t.shuffle_tile_log2 = tlist[key.ti];
    t.ms = -1.0;
    kc_ctx* c = nullptr;
    kc_status r = kc_create(&cfg, device, &c);
    double ms = 1e300;
    if (r == KC_OK) {
      kc_stats st{};
      for (int rep = 0; rep < 3 && r == KC_OK; ++rep) {
        if (rep) r = kc_reset(c);
        if (r != KC_OK) break;
        r = kc_count_batch(c, chunks, n_chunks, counter, hip_stream, &st);
        if (r == KC_OK && rep) ms = std::min(ms, st.kernel_ms[KC_T_GRAPH]);
      }
      if (r == KC_OK) {
        t.ms = ms;
        t.overflow_keys = st.overflow_keys;
      }
      kc_destroy(c);
    }
    if (r != KC_OK) ms = 1e300;
    t.status = r;
    got.push_back(t);
    seen.push_back({key, ms});
    if (ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
    return ms;
  };
  const uint32_t p0 = std::min<uint32_t>(kMaxPartLog2, (uint32_t)std::max<int64_t>(lo, pc));
  auto split = [&](uint32_t p) { return std::min<uint32_t>(p / 2, kMaxA1); };
  auto valid = [&](const Key& k) {
    if (k.p < lo || k.p > (uint32_t)kMaxPartLog2 || k.si >= slist.size() || k.ti >= 3) return false;
    const int64_t a2 = (int64_t)k.p - k.a1;
    return k.a1 >= 1 && k.a1 <= (uint32_t)kMaxA1 && a2 >= 1 && a2 <= kMaxA2;
  };
  Key cur{p0, 0, split(p0), 0};
  double cur_ms = run(cur);
  const int kMaxTrials = 28;
  bool moved = true;
  while (moved && (int)got.size() < kMaxTrials) {
    moved = false;
    for (int dim = 0; dim < 4 && (int)got.size() < kMaxTrials; ++dim) {
      for (int dir : {-1, 1}) {
        for (;;) {
          Key nk = cur;
          if (dim == 0) {
            nk.p = (uint32_t)((int64_t)cur.p + dir);
            nk.a1 = split(nk.p);
          } else if (dim == 1) {
            nk.a1 = (uint32_t)((int64_t)cur.a1 + dir);
          } else if (dim == 2) {
            nk.si = (uint32_t)((int64_t)cur.si + dir);
          } else {
            nk.ti = (uint32_t)((int64_t)cur.ti + dir);
          }
          if (!valid(nk) || (int)got.size() >= kMaxTrials) break;
          const double ms = run(nk);
          if (ms >= cur_ms) break;
          cur = nk;
          cur_ms = ms;
          moved = true;
        }
      }
    }
  }
  if (trials)
    for (uint32_t i = 0; i < std::min<uint32_t>(max_trials, (uint32_t)got.size()); ++i) trials[i] = got[i];
  if (n_trials_out) *n_trials_out = (uint32_t)got.size();
  if (best_ms >= 1e300) {
    g_create_error = "no candidate configuration ran";
    return got.empty() ? KC_ERR_INVALID_ARG : (kc_status)got.back().status;
  }
  *best_out = best;
  return KC_OK;
}

}  // extern "C"
