// kc_internal.h - shared declarations between the kernels and the host runtime
// of the k-mer counter (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <vector>

#include "kc.h"

namespace kc {

constexpr uint64_t kEmpty = ~0ull;              // empty table slot (no key reaches it: x < 2^62)
constexpr uint64_t kKeyMask = (1ull << 62) - 1; // key bits; bit 62 carries the counter tag
constexpr uint64_t kTableMul = 0xD6E8FEB86659FD93ull; // odd multiplier of the table slot hash
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;          // partition table not in HBM (spilled)
constexpr uint32_t kProbeLimit = 128;              // probes before a key goes to the overflow table
// A key is stored less than this many slots past its home slot in a table of
// cap slots (further along it goes to the overflow table), so a lookup stops
// after as many probes.
inline __host__ __device__ uint32_t probe_limit_of(uint64_t cap) {
  return cap < kProbeLimit ? (uint32_t)cap : kProbeLimit;
}
// Partition tables are cut into aligned buckets of kBucket slots (cap is a
// multiple of 64).  A key's home slot is the first slot of one bucket, picked
// by the top 32 bits of th = (x ^ s_0) * kTableMul; probing is linear from
// there, so a key inserted while its bucket has room lies in that bucket, and
// a count probe reads the bucket's keys at once.
constexpr uint32_t kBucket = 4;
inline __host__ __device__ uint32_t home_slot_of(uint64_t th, uint64_t cap) {
  return (uint32_t)((((th >> 32) * (cap / kBucket)) >> 32) * kBucket);
}
constexpr int kThreads = 1024;                  // block size of the tile kernels
constexpr int kWaves = kThreads / 64;
constexpr int kTileWords = 256;                 // first-level tile: 256 packed words
constexpr int kTilePos = kTileWords * 32;       // = 8192 window positions
constexpr int kT2 = 8192;                       // second-level tile: most keys per workgroup
constexpr uint32_t kT2MinLog2 = 10;             // smallest second-level tile (log2 keys)
constexpr int kMaxA1 = 10;                      // first-level fan-out limit (bits)
constexpr int kMaxA2 = 11;                      // second-level fan-out limit (bits)
constexpr int kMaxPartLog2 = kMaxA1 + kMaxA2;    // partitions (log2) two levels can reach
constexpr int kLdsMax = 163840;                 // gfx950 LDS per workgroup
constexpr int kLdsSlack = 2048;                 // LDS left unused per k_tally workgroup
constexpr int kNst = 8;                         // statistics slots
constexpr int kTallyWaves = 8;                  // waves per k_tally workgroup
constexpr int kQueueBytes = kTallyWaves * 64 * 12;  // per-wave miss queues of k_tally
constexpr uint32_t kXcds = 8;                   // XCDs; workgroup b is dispatched to XCD b mod 8

// Second-level launch with an upper bound of `tiles2` tiles: the grid, a
// multiple of kXcds.
inline uint64_t level2_grid(uint64_t tiles2) { return (tiles2 + kXcds - 1) / kXcds * kXcds; }
// Bytes of the second-level descriptor buffer: one 64-bit descriptor per
// workgroup of the second-level grid.
inline uint64_t tile_desc_bytes(uint64_t tiles2) { return 8 * level2_grid(tiles2); }

enum Stat { ST_NPASS = 0, ST_ENTRIES, ST_SUM, ST_FP, ST_B1POP, ST_B2POP, ST_PASSED, ST_OVF };
enum Err : uint32_t { ERR_OFFSETS = 1, ERR_OVF_FULL = 2, ERR_OVF_LOAD = 4, ERR_QUERY_RANGE = 8 };

// One kc_insert_reads call: its keys grouped by partition.  Partition
// u = c * 2^a2 + sub: first-level bucket c holds keys[bucket_off[c] ..
// bucket_off[c+1]); with a2 > 0 that range is cut into tiles of 2^t2_log2 keys
// (tile_first[c] .. tile_first[c+1]), and inside tile t the keys of sub-bucket
// sub sit at [meta2[t*(2^a2+1)+sub], meta2[t*(2^a2+1)+sub+1]) of the tile.
struct SegDesc {
  const uint64_t* keys;
  const uint64_t* bucket_off;
  const uint32_t* tile_first;
  const uint32_t* meta2;
  uint32_t a1, a2;
  uint32_t t2_log2;  // keys per second-level tile (log2)
  uint32_t pad_;
};

// One read chunk of a batch, placed in its group's position stream at
// packed word word0 (chunks start on 32-base boundaries; the gap before the
// next chunk holds invalid bases).  read0: exclusive prefix of (n_reads + 1)
// over the group's chunks (one check slot per chunk end).
struct ChunkDesc {
  const uint8_t* bases;
  const uint64_t* offsets;
  uint64_t total;
  uint64_t n_reads;
  uint64_t word0;
  uint64_t read0;
};

struct HashCfg {
  uint64_t salt[9];   // s_0 .. s_h
  uint32_t k, h, bl, s_log2, p_log2, nc, min_count, pad;
};

struct CountArgs {
  HashCfg hc;
  const SegDesc* segs;
  uint32_t nsegs;
  uint32_t upb_log2;     // partitions per Bloom block (log2)
  uint32_t bsub_log2;    // Bloom blocks per k_bloom workgroup (log2)
  uint32_t part_base;    // k_tally: first partition of this launch
  uint32_t part_n;       // k_tally: partitions in this launch (= grid size)
  uint32_t slot_base;    // k_tally: table slot of partition part_base
  uint32_t nbw;          // u32 words per Bloom block and level
  uint32_t l2w;          // LDS words reserved for level 2 (even)
  uint32_t cap;          // slots per partition table (multiple of 64)
  uint32_t probe_limit;
  uint32_t ovf_log2;
  uint32_t ovf_limit;
  uint32_t* b1;
  uint32_t* b2;
  uint64_t* tkeys;
  uint32_t* tcounts;
  uint64_t* okeys;
  uint32_t* ocounts;
  uint32_t* ovf_used;
  uint32_t* err;
  uint64_t* pstats;      // [Bloom blocks * kNst]: level popcounts
  uint64_t* pstats2;     // [partitions * kNst]: count statistics
};

struct QueryArgs {
  HashCfg hc;
  uint64_t cap;            // slots per partition table
  uint32_t probe_limit;    // probes of a partition-table lookup (probe_limit_of(cap))
  const uint64_t* tkeys;
  const uint32_t* tcounts;
  const uint32_t* slot_of;  // partition -> its table slot in HBM, or kNoSlot if spilled
  int64_t slot_first;       // >= 0: slot_of[u] is u - slot_first, kNoSlot below it
  const uint64_t* okeys;
  const uint32_t* ocounts;
  const uint32_t* ovf_used;
  uint32_t ovf_log2;
  uint32_t* err;
  uint32_t* host_rows;     // indices of queries on spilled partitions
  uint64_t* host_keys;     // their canonical keys (same order)
  uint32_t* host_count;
  const uint64_t* fkeys;   // filter: the table keys with bit 63 set where the slot's counts
                           // pass the filter's thresholds (NULL: probe keys, then counts)
};

// ---- launchers (kc_kernels.hip) ----
hipError_t launch_pack(const uint8_t* bases, uint64_t total, uint64_t nwords, uint64_t* packed,
                       uint64_t* flags, hipStream_t s);
hipError_t launch_rstart(const uint64_t* offsets, uint64_t n_reads, uint64_t total,
                         uint64_t* flags, uint32_t* err, hipStream_t s);
hipError_t launch_scan(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* parts,
                       hipStream_t s);
size_t scan_parts(uint64_t n);
hipError_t launch_bucket_off(const uint64_t* off1, uint64_t ntiles, uint32_t nb1,
                             uint64_t* bucket_off, hipStream_t s);
size_t level1_lds(uint32_t a1);
size_t level2_lds(uint32_t a2, uint32_t t2_log2);
hipError_t launch_level1(const uint64_t* packed, const uint64_t* flags, uint64_t nwords,
                         uint32_t k, uint64_t s0, uint32_t a1, uint64_t tag, uint32_t* hist,
                         uint32_t* lstart, uint64_t ntiles, uint64_t* out, hipStream_t s);
hipError_t launch_tiles2(const uint64_t* bucket_off, uint32_t nb1, uint32_t t2_log2,
                         uint32_t* tile_first, hipStream_t s);
hipError_t launch_level2(const uint64_t* keys1, const uint64_t* off1, const uint32_t* lstart,
                         uint64_t ntiles1, const uint64_t* bucket_off, const uint32_t* tile_first,
                         uint64_t* tile_desc, uint32_t a1, uint32_t a2, uint32_t t2_log2,
                         uint64_t s0, uint64_t* keys2, uint32_t* meta2, uint64_t grid,
                         hipStream_t s);
hipError_t launch_bloom(const CountArgs& a, uint32_t blocks, size_t lds, hipStream_t s);
hipError_t launch_tally(const CountArgs& a, uint32_t parts, size_t lds, hipStream_t s);
int tally_threads();
hipError_t launch_ovf_emit(const CountArgs& a, uint64_t* pstats_ovf, uint32_t blocks,
                           hipStream_t s);
hipError_t launch_reduce(const uint64_t* rows, uint64_t nrows, uint64_t* out, hipStream_t s);
// Stem relayout by stem partitions (the top p_log2 bits of a stem's hash):
// count the entries of each partition over a table pass (pcount[2^p_log2]),
// scatter them as records (cursor[p] starts at partition p's offset), then
// one workgroup per partition numbers its distinct stems and writes their
// items (poff: 2^p_log2 + 1 offsets; cursor: the item count so far).
hipError_t launch_stem_count(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                             const uint32_t* live, uint32_t cap, uint32_t nc, uint32_t k,
                             uint32_t p_log2, uint32_t* pcount, hipStream_t s);
hipError_t launch_stem_scatter(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                               const uint32_t* live, uint32_t cap, uint32_t nc, uint32_t k,
                               uint32_t p_log2, uint64_t* cursor, uint64_t* rstem, uint32_t* rcnt,
                               hipStream_t s);
// Most records a partition may hold (its distinct stems fit the LDS table).
uint32_t stem_part_max();
hipError_t launch_stem_group(const uint64_t* poff, uint64_t nparts, const uint64_t* rstem,
                             const uint32_t* rcnt, bool count_only, uint64_t* cursor,
                             uint64_t capacity, uint64_t* stems, uint16_t* items, uint32_t* err,
                             hipStream_t s);
// fkeys[i] = tkeys[i] with bit 63 set when slot i's counts pass (tumour >=
// tmin, normal <= nmax), for the nslots slots of the resident tables.
hipError_t launch_filter_keys(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                              uint32_t nc, uint32_t tmin, uint32_t nmax, uint64_t* fkeys,
                              hipStream_t s);
hipError_t launch_filter(const QueryArgs& a, const uint64_t* packed, const uint64_t* flags,
                         uint64_t nwords, const uint64_t* offsets, uint64_t n_reads, uint64_t total,
                         uint32_t tmin, uint32_t nmax, uint32_t* hit, uint32_t* out, hipStream_t s);
hipError_t launch_query(const QueryArgs& a, const uint64_t* kmers, uint64_t n, uint32_t* out,
                        hipStream_t s);
hipError_t launch_export(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                         const uint32_t* live, uint32_t cap, uint32_t nc,
                         uint64_t* out_keys, uint32_t* out_counts, uint64_t out_cap,
                         uint64_t* cursor, hipStream_t s);
hipError_t launch_debug_part(const SegDesc& sd, uint64_t n, uint32_t* part, hipStream_t s);
hipError_t launch_pack_batch(const ChunkDesc* cd, uint32_t nchunks, uint64_t nwords,
                             uint64_t* packed, uint64_t* flags, hipStream_t s);
hipError_t launch_rstart_batch(const ChunkDesc* cd, uint32_t nchunks, uint64_t nslots,
                               uint64_t* flags, uint32_t* err, hipStream_t s);
hipError_t launch_fill64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_copy64(const uint64_t* src, uint64_t* dst, hipStream_t s);
hipError_t launch_gather2(const uint64_t* a, const uint64_t* b, const uint64_t* idx, uint64_t n,
                          uint64_t nwords, uint64_t* out_a, uint64_t* out_b, uint32_t* err,
                          hipStream_t s);
hipError_t launch_slot_map(uint32_t* slot_of, uint32_t n, uint32_t first, hipStream_t s);
hipError_t launch_scatter_rows(const uint32_t* rows, const uint32_t* vals, uint32_t n,
                               uint32_t nc, uint32_t* out, hipStream_t s);

// ---- runtime helpers for the request server (kc_runtime.hip) ----
// Device bytes a context holds now (every buffer it has allocated).
uint64_t ctx_device_bytes(const kc_ctx* c);
// Device bytes context c (NULL: a new one) holds after counting, with
// configuration cfg, n_parts inserts of part_bases[i] bases each: its buffers
// only grow, so each is the larger of what it holds and what the job needs
// (keys bounded by window positions).  0 when cfg is invalid.
uint64_t bytes_after(const kc_ctx* c, const kc_config* cfg, const uint64_t* part_bases,
                     uint32_t n_parts);
uint64_t estimate_count_bytes(const kc_config* cfg, const uint64_t* part_bases, uint32_t n_parts);
// Gives a reset (CREATED) context a new configuration, keeping its buffers
// (new ones are allocated in order on stream s).
kc_status reconfigure(kc_ctx* c, const kc_config* cfg, hipStream_t s);
// While one lives, the calling thread's library allocations and frees are
// stream-ordered on s.
struct AllocStream {
  explicit AllocStream(hipStream_t s);
  ~AllocStream();
  AllocStream(const AllocStream&) = delete;
  AllocStream& operator=(const AllocStream&) = delete;
  hipStream_t prev;
  bool prev_on;
};
// Keeps memory freed to the device's default pool cached there (once per device).
void keep_pool_memory(int device);

// ---- device block cache of the request server (kc_runtime.hip) ----
// Size of the block that serves a request of n bytes: a multiple of 4 KiB up
// to 16 KiB, then four sizes per octave (at most a quarter above n).
uint64_t cache_round(uint64_t n);
// Device blocks that the request server's contexts free, kept for the
// server's later allocations instead of going back to the runtime (under
// context churn the runtime's stream-ordered pool hands memory back and maps
// it again, and the workers then wait tens of milliseconds).  A block is
// reused for a request of at most half its size or more; one freed on another
// stream is handed over behind an event wait, so reuse keeps stream order.
// Blocks come from hipMalloc and go back with hipFree only past the cache
// limit (largest first) or when the cache is drained.  Thread-safe.
class BlockCache {
 public:
  explicit BlockCache(uint64_t limit) : limit_(limit) {}
  hipError_t alloc(uint64_t want, hipStream_t s, void** p, uint64_t* got);
  void give_back(void* p, uint64_t bytes, hipStream_t s);
  // Frees every cached block; call with the device idle.
  void drain();
  // bytes cached now, blocks taken from and given back to the runtime so far
  void usage(uint64_t* cached, uint64_t* allocs, uint64_t* frees) {
    std::lock_guard<std::mutex> lk(mu_);
    *cached = cached_;
    *allocs = allocs_;
    *frees = frees_;
  }

 private:
  struct Block {
    void* p;
    hipStream_t s;   // stream of its last use
    hipEvent_t ev;   // recorded there when it was given back (NULL: no wait needed)
  };
  void free_largest();
  std::mutex mu_;
  std::multimap<uint64_t, Block> free_;
  std::vector<hipEvent_t> events_;
  uint64_t cached_ = 0, allocs_ = 0, frees_ = 0;
  const uint64_t limit_;
};
// While one lives, the calling thread's new library buffers come from cache k
// (each buffer remembers where it came from and goes back there).
struct UseCache {
  explicit UseCache(BlockCache* k);
  ~UseCache();
  UseCache(const UseCache&) = delete;
  UseCache& operator=(const UseCache&) = delete;
  BlockCache* prev;
};

}  // namespace kc
