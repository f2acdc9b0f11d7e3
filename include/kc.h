/*
 * kc.h - C ABI of the MI355X k-mer frequency counter.
 *
 * The library counts canonical k-mers of DNA reads on one GPU, screens out
 * k-mers seen once with a two-level Bloom filter and keeps exact counts of the
 * k-mers seen at least min_count times in per-partition hash tables.  It
 * follows the counting unit of Cadenelli, Polo, Carrera, "Accelerating K-mer
 * Frequency Counting with GPU and Non-Volatile Memory": Sec. II-A (k-mers,
 * 2-bit 64-bit codes), Sec. II-B (Count unit: unique k-mers are discarded),
 * Sec. III (Prune: chained Bloom filters; Count: exact table; Unify: merge of
 * swapped tables and removal of Bloom false positives), Sec. III-B (GPU
 * shuffle of k-mers by consumer: histogram, exclusive prefix sum, broker
 * scatter), Sec. III-D (swap of full tables to a slower memory tier with a hot
 * spare and per-table metadata).
 *
 * Conventions that hold for every entry point:
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller owns them and keeps them valid until the call has returned (for
 *    kc_insert_reads: until the stream has passed the call).  Pointers named
 *    *_host are ordinary host memory owned by the caller.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream).  Work is
 *    ordered on that stream.  Calls marked "synchronises" return only after
 *    their device work has finished.
 *  - Every entry point returns a kc_status.  On failure the context's error
 *    text (kc_last_error) says what went wrong; the context stays usable
 *    unless the status is KC_ERR_DEVICE.  No exception crosses the ABI.
 *  - One host thread at a time per context; distinct contexts are
 *    independent and may be used from different threads.
 *  - Life cycle: CREATED -> (kc_insert_reads)* -> kc_finalize -> FINALIZED
 *    (kc_query, kc_export, kc_export_bloom, kc_spill).  kc_reset returns to
 *    CREATED.  Calls out of this order return KC_ERR_BAD_STATE.
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KC_ABI_VERSION 9u

typedef struct kc_ctx kc_ctx;

typedef enum kc_status {
  KC_OK = 0,
  KC_ERR_INVALID_ARG = -1,   /* a parameter, pointer or input value is out of range */
  KC_ERR_OUT_OF_MEMORY = -2, /* a device or pinned host allocation failed */
  KC_ERR_BAD_STATE = -3,     /* call not allowed in the context's current state */
  KC_ERR_DEVICE = -4,        /* a HIP runtime call failed; the context must be destroyed */
  KC_ERR_OVER_BUDGET = -5    /* the table budget cannot hold what the call needs */
} kc_status;

/*
 * Counting parameters.  The result-defining fields fix every output bit
 * (table, Bloom levels, statistics); the result-neutral fields change only
 * speed and memory, never a result.
 *
 * Definitions (the paper's k-mer is a 2-bit-per-base 64-bit code, Sec. II-A;
 * the screen is Prune's two Bloom levels, Sec. III):
 *   code A=0 C=1 G=2 T=3; enc(w) = sum_j code(w_j) 4^(k-1-j); only the bytes
 *   A, C, G, T are bases, any other byte breaks the windows covering it;
 *   x = min(enc(w), enc(revcomp(w))); mix64 = SplitMix64 output function;
 *   s_i = mix64(seed + (i+1) * 0x9E3779B97F4A7C15) for i = 0, 1;
 *   g = mix64(x ^ s_0); block(x) = top (bloom_bits_log2 - bloom_block_log2)
 *   bits of g; with B = 2^bloom_block_log2 and u = mix64(x ^ s_1), a = the
 *   top bloom_block_log2 bits of u and b = the next bloom_block_log2 bits,
 *   S(x) = { block * B + ((a + i*b) mod B) : i = 0..h-1 } (double hashing);
 *   hits(b) = number of occurrences of keys with b in S(x);
 *   B1[b] = hits(b) >= 1, B2[b] = hits(b) >= 2;
 *   a key passes the screen iff S(x) is a subset of B2.
 */
typedef struct kc_config {
  /* result-defining */
  uint32_t k;                /* k-mer length, 1..31 */
  uint32_t n_counters;       /* 1 = one count per k-mer; 2 = normal/tumour counts */
  uint32_t min_count;        /* keep k-mers whose total count is >= this; >= 2 */
  uint32_t bloom_bits_log2;  /* each Bloom level holds 2^this bits; bloom_block_log2..40 */
  uint32_t bloom_hashes;     /* h, 1..8 */
  uint32_t bloom_block_log2; /* Bloom block size in bits (log2), 1..19 */
  uint64_t seed;             /* derives s_0 .. s_h */
  /* result-neutral */
  uint32_t partitions_log2;  /* hash partitions = top bits of g; raised to
                                bloom_bits_log2 - bloom_block_log2 when lower; <= 21 */
  uint32_t table_slots;      /* slots per partition table, rounded down to a multiple of
                                64 (>= 64, at most what one count workgroup's LDS holds);
                                0 = the largest with which three count workgroups share a
                                CU (3840 with one counter, 2880 with two) */
  uint32_t scatter_bits;     /* first-level shuffle fan-out bits; 0 = automatic */
  uint32_t group_bases_log2; /* kc_count_batch: at most 2^this bases (with padding) per key
                                segment; 0 = 2^32 - 64, else 10..32 */
  uint64_t hbm_table_budget_bytes; /* device bytes the partition tables may use; 0 = unlimited */
  uint32_t shuffle_tile_log2; /* keys per second-level shuffle tile (log2), 10..13; 0 = 13 */
  uint32_t reserved_;        /* 0 */
} kc_config;

/* Per-stage timers (kernel_ms indexes): sums of HIP-event durations. */
enum {
  KC_T_PACK = 0,   /* ASCII -> 2-bit stream, invalid and read-start bits */
  KC_T_LEVEL1 = 1, /* extraction + first-level shuffle (one pass per tile) */
  KC_T_SCAN = 2,   /* exclusive prefix sum of the first-level histogram */
  KC_T_LEVEL2 = 3, /* second-level shuffle into partition-sorted tiles */
  KC_T_BLOOM = 4,  /* per Bloom block: B1/B2 built from every occurrence */
  KC_T_TALLY = 5,  /* per partition: screen against B2 and exact count */
  KC_T_UNIFY = 6,  /* overflow table pass, statistics reduction */
  KC_T_QUERY = 7,
  KC_T_SPILL = 8,  /* device -> pinned host copies of spilled partitions */
  KC_T_GRAPH = 9,  /* kc_count_batch: the whole batch as one graph launch */
  KC_T_STEMS = 10, /* kc_export_stems: the stem layout of the final table */
  KC_T_FILTER = 11, /* kc_filter_reads: lookups of every window of a read batch */
  KC_T_COUNT_OF = 16
};

typedef struct kc_stats {
  uint64_t n_valid;            /* valid windows (k-mer occurrences) inserted */
  uint64_t n_pass;             /* occurrences whose key passes the Bloom screen */
  uint64_t entries;            /* k-mers with total count >= min_count */
  uint64_t sum_counts;         /* sum of their total counts */
  uint64_t fp_singletons;      /* k-mers seen once that passed the screen (removed) */
  uint64_t b1_popcount;        /* set bits of Bloom level 1 */
  uint64_t b2_popcount;        /* set bits of Bloom level 2 */
  uint64_t spilled_partitions; /* partitions whose table lives in pinned host memory */
  uint64_t spilled_bytes;      /* bytes of those tables (keys + counts, no padding) */
  uint64_t overflow_keys;      /* distinct keys counted in the device overflow table */
  uint64_t passed_distinct;    /* distinct keys that passed the screen */
  uint32_t partitions_log2;    /* effective partition count (log2) */
  uint32_t table_slots;        /* effective slots per partition table */
  uint32_t n_segments;         /* kc_insert_reads calls since the last reset */
  uint32_t retries;            /* finalize re-runs after an overflow-table fill */
  double kernel_ms[KC_T_COUNT_OF]; /* per-stage device time, milliseconds */
  uint64_t kernel_launches[KC_T_COUNT_OF];
} kc_stats;

/* ABI version of the loaded library (KC_ABI_VERSION). */
uint32_t kc_abi_version(void);

/* Human-readable name of a status code (static string). */
const char* kc_status_str(kc_status s);

/* Creates one counting unit on HIP device `device`: the state SMUFIN's
 * counting unit holds across its pipeline cycles (Sec. II-B, Count unit;
 * Sec. III: Prune's two chained Bloom filters and Count's frequency table),
 * here a context that owns the two Bloom levels (allocated now, 2 *
 * 2^bloom_bits_log2 bits, the configuration's k, counters, min_count, hash
 * and partition parameters fixed for its life), the inserted keys and the
 * partition tables.  Validates cfg and returns KC_ERR_INVALID_ARG for any
 * field out of range, KC_ERR_OUT_OF_MEMORY when the levels do not fit.
 * *out receives the context, which the caller frees with kc_destroy, or NULL
 * on failure (then kc_last_error(NULL) holds the reason). */
kc_status kc_create(const kc_config* cfg, int device, kc_ctx** out);

/*
 * Adds reads (pass 1: k-mer extraction, canonical form and the hash-partition
 * shuffle of Sec. III-B).  Reads are bases_dev[offsets_dev[i] ..
 * offsets_dev[i+1]) for i < n_reads, ASCII, back to back; offsets_dev has
 * n_reads + 1 entries with offsets_dev[0] = 0 and offsets_dev[n_reads] =
 * total_bases, non-decreasing (empty reads allowed).  counter (0 or 1, <
 * n_counters) is the sample the reads belong to (0 normal, 1 tumour).
 * Windows never span two reads.  Synchronises once on hip_stream (to size the
 * key buffer); the shuffle itself stays queued on the stream.  Offsets that
 * break the rules above are detected on the device: the call then returns
 * KC_ERR_INVALID_ARG and inserts nothing.
 */
kc_status kc_insert_reads(kc_ctx* ctx, const uint8_t* bases_dev, const uint64_t* offsets_dev,
                          uint64_t n_reads, uint64_t total_bases, uint32_t counter,
                          void* hip_stream);

/*
 * Pass 2 and Unify (Sec. III): builds the Bloom levels, screens every
 * occurrence against level 2, counts the passing keys exactly per partition,
 * drops keys below min_count (false-positive singletons are counted in
 * fp_singletons) and leaves one open-addressing table per partition.  With a
 * table budget smaller than all tables, HBM holds only the tables the budget
 * pays for (the highest partitions); the others are counted in waves and
 * their tables copied to pinned host memory as each wave finishes (Sec.
 * III-D's swap of full tables), so table memory in HBM never exceeds the
 * budget.  Synchronises.  out_host (may be NULL) receives the statistics.
 */
kc_status kc_finalize(kc_ctx* ctx, void* hip_stream, kc_stats* out_host);

/*
 * Frequency-table lookups after Count and Unify (Sec. II-B: the Filter unit
 * looks k-mers up in the final frequency table; Sec. III, Unify: the table
 * holds the k-mers seen at least min_count times, false-positive singletons
 * removed).  Looks up n k-mers given as 2-bit codes < 4^k in either
 * orientation (kmers_dev[n], device, caller-owned): counts_dev[i * n_counters
 * + c] (device, caller-owned, n * n_counters uint32) receives counter c of
 * canonical(kmers_dev[i]) when its total count is >= min_count, else 0.
 * Partitions spilled to pinned host memory are answered from their host
 * copies.  After kc_finalize (else KC_ERR_BAD_STATE).  Synchronises.  A code
 * >= 4^k makes the call return KC_ERR_INVALID_ARG (its output row is 0).
 */
kc_status kc_query(kc_ctx* ctx, const uint64_t* kmers_dev, uint64_t n, uint32_t* counts_dev,
                   void* hip_stream);

/*
 * Moves a partition's finished table from HBM to pinned host memory (the
 * stand-in for the paper's swap of full tables to NVM, Sec. III-D) and records
 * it in the spill directory (partition, entries, host offset, stale flag).
 * partition = -1 spills resident partitions, highest index first, until the
 * resident tables fit hbm_table_budget_bytes.  *bytes_out (may be NULL)
 * receives the bytes moved.  Queries keep working on spilled partitions.
 */
kc_status kc_spill(kc_ctx* ctx, int64_t partition, uint64_t* bytes_out);

/*
 * Copies the final table to host memory: keys_host[cap], counts_host[cap *
 * n_counters].  With keys_host == NULL only *n_out (number of entries) is
 * set.  Entries come partition by partition (unsorted within a partition).
 * Returns KC_ERR_INVALID_ARG when cap is smaller than the number of entries.
 */
kc_status kc_export(kc_ctx* ctx, uint64_t* keys_host, uint32_t* counts_host, uint64_t cap,
                    uint64_t* n_out);

/* Copies the two Bloom levels (words = 2^bloom_bits_log2 / 64, at least 1,
 * little-endian: bit b in word b >> 6 at position b & 63).  Either pointer
 * may be NULL. */
kc_status kc_export_bloom(kc_ctx* ctx, uint64_t* b1_host, uint64_t* b2_host, uint64_t words);

/* Copies chosen words of the two Bloom levels (Sec. III, Prune: the first and
 * second filter), for filters too large to copy whole: b1_host[i] and
 * b2_host[i] receive word word_idx_host[i] of each level (same word layout as
 * kc_export_bloom).  Host arrays of n entries, owned by the caller.  After
 * kc_finalize; an index at or past 2^bloom_bits_log2 / 64 returns
 * KC_ERR_INVALID_ARG (the outputs are then unspecified). */
kc_status kc_export_bloom_words(kc_ctx* ctx, const uint64_t* word_idx_host, uint64_t n,
                                uint64_t* b1_host, uint64_t* b2_host);

/* Unify's stem layout of the final table (Sec. II-A: the stem of a k-mer is
 * its middle k-2 bases; Sec. III-D: counts grouped per stem, the 16 normal
 * and 16 tumour k-mers of a stem in one item of 2-byte counts).  After
 * kc_finalize; needs k >= 3.  Each k-mer of the table (what kc_export
 * returns) is read in the orientation of its canonical stem S, the smaller
 * code of its middle k-2 bases and their reverse complement: as a S b (a, b
 * its first and last bases) when its own middle is S, else as its reverse
 * complement (and as written when S is its own reverse complement).  Item i
 * is stems_dev[i] (the (k-2)-base code of S) and counts_dev[32 i .. 32 i + 31]:
 * entry 4a+b holds counter 0's count and 16+4a+b counter 1's, each saturated
 * to 65535; entries of k-mers not in the table are 0.  Items are in no
 * particular order.  *n_out receives the item count, at most stats.entries
 * (so a capacity of stats.entries always suffices); with a smaller capacity
 * the call fails with KC_ERR_INVALID_ARG after setting *n_out.  counts_dev
 * must be 4-byte aligned.  Spilled tables are staged back to HBM.  Scratch:
 * about 12 bytes of device memory per entry (one record per table k-mer) and
 * 12 bytes per stem partition, allocated and freed inside.  Synchronises. */
kc_status kc_export_stems(kc_ctx* ctx, uint64_t* stems_dev, uint16_t* counts_dev, uint64_t capacity,
                          uint64_t* n_out, void* hip_stream);

/* Checkpoint of a finalized context (Sec. II-B: the application's units are
 * checkpointable, dumping Bloom filters and k-mer tables at their end;
 * Sec. III-D: swapped tables are identified by metadata records - partition,
 * stale flag, byte offset, item count - kept in a reserved area at the start
 * of the device).  Writes `path` (through path + ".tmp", renamed when
 * complete): a reserved area with a header (ABI version, configuration,
 * table geometry, statistics) and one record per partition table, then
 * every partition table in partition order (resident ones copied from HBM,
 * spilled ones from the pinned pool), both Bloom levels and the overflow
 * table.  Synchronises the device. */
kc_status kc_checkpoint(kc_ctx* ctx, const char* path);

/* Creates a finalized context on `device` from a checkpoint file: the
 * configuration, tables, Bloom levels and statistics it holds.  Tables are
 * laid out as kc_finalize lays them out under the saved table budget (the
 * lowest partitions in pinned host memory when the budget is smaller than
 * all tables), so queries, exports, the stem layout and the filter answer as
 * before the checkpoint; the statistics' timers start at zero and the spill
 * counts describe the restored layout.  A file from another ABI version, or
 * truncated or inconsistent, is rejected with KC_ERR_INVALID_ARG (text in
 * kc_last_error(NULL)). */
kc_status kc_restore(const char* path, int device, kc_ctx** out);

/* Filter-unit lookup (Sec. II-B: the Filter unit reads the input sequences
 * again and looks their k-mers up in the frequency table to select k-mers
 * with imbalanced frequencies; the imbalance test is a parameter here).
 * After kc_finalize.  The reads come in the layout of kc_insert_reads
 * (bases_dev, offsets_dev[n_reads + 1], at most 2^32 - 1 bases).  Every
 * window the count enumerates is looked up: with (normal, tumour) = its
 * k-mer's counters 0 and 1 in the final table (0 and 0 when the k-mer is not
 * in it; for a one-counter table normal is 0 and tumour is the count), the
 * window is selected when tumour >= tumour_min and normal <= normal_max.
 * out_dev[r] (uint32, device) receives read r's number of selected windows.
 * Needs every partition table in HBM: after a spill it returns
 * KC_ERR_BAD_STATE (kc_query answers such tables from the host).  Scratch of
 * 2.5 bits per base, and, when the bases number at least half the table
 * slots, 8 bytes per table slot (the table keys marked with the selection,
 * so that each lookup reads one line; without room for them the lookups read
 * keys and counts, with the same results), allocated and freed inside.
 * Synchronises. */
kc_status kc_filter_reads(kc_ctx* ctx, const uint8_t* bases_dev, const uint64_t* offsets_dev,
                          uint64_t n_reads, uint64_t total_bases, uint32_t tumour_min,
                          uint32_t normal_max, uint32_t* out_dev, void* hip_stream);

/* Largest read batch (bases) of kc_filter_reads_noalloc. */
#define KC_FILTER_NOALLOC_MAX_BASES (1ull << 25)

/*
 * kc_filter_reads for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as kc_filter_reads, and the same
 * kernels; it calls no device or host allocator.  Its scratch (packed words,
 * flag words and the window bitmap of up to KC_FILTER_NOALLOC_MAX_BASES
 * bases, 20 MiB) is one array per GPU, held by the library from the first
 * kc_create on that GPU until the process ends; a batch of more bases
 * returns KC_ERR_INVALID_ARG.  Every call on a GPU uses that GPU's one
 * array, so calls that overlap in time on one GPU (from any context, stream
 * or thread) race and give undefined results; calls that follow each other
 * on one stream, or are synchronised, are safe.  Synchronises.
 */
kc_status kc_filter_reads_noalloc(kc_ctx* ctx, const uint8_t* bases_dev,
                                  const uint64_t* offsets_dev, uint64_t n_reads,
                                  uint64_t total_bases, uint32_t tumour_min, uint32_t normal_max,
                                  uint32_t* out_dev, void* hip_stream);

/*
 * Debug view of pass 1: every stored key occurrence (x | counter << 62) and the
 * partition it was shuffled to, segment by segment in storage order.  With
 * keys_host == NULL only *n_out is set.  Valid in any state after inserts.
 */
kc_status kc_debug_keys(kc_ctx* ctx, uint64_t* keys_host, uint32_t* partition_host,
                        uint64_t cap, uint64_t* n_out);

/* Statistics of the last finalize (plus inserts and timers since reset). */
kc_status kc_get_stats(const kc_ctx* ctx, kc_stats* out_host);

/* Drops inserted reads, tables and spilled partitions; keeps allocations for
 * reuse.  Back to CREATED.  Waits for the context's own queued work (the last
 * kc_insert_reads); other contexts' work on the device is not waited for. */
kc_status kc_reset(kc_ctx* ctx);

/*
 * Batched form.  A chunk is a set of reads laid out as for kc_insert_reads.
 */
typedef struct kc_chunk {
  const uint8_t* bases_dev;
  const uint64_t* offsets_dev; /* n_reads + 1 entries */
  uint64_t n_reads;
  uint64_t total_bases;
} kc_chunk;

/*
 * Counts a batch of read chunks into the shared Bloom levels and tables:
 * the same result as kc_insert_reads on every chunk (in order, all with
 * `counter`) followed by kc_finalize, produced by one hipGraph launch on
 * hip_stream.  Consecutive chunks are packed side by side into key segments
 * of at most 2^group_bases_log2 bases, each segment shuffled once; the graph
 * (every kernel of every segment, then Bloom, count and Unify) is captured on
 * the first call for a given chunk list and replayed by later calls with the
 * same chunks (pointers and sizes), after kc_reset.  The context must be in
 * CREATED state; afterwards it is FINALIZED.  Every partition table stays in
 * HBM: a budget smaller than all tables returns KC_ERR_OVER_BUDGET.  Offsets
 * that break kc_insert_reads' rules return KC_ERR_INVALID_ARG.  chunks_host
 * is read during the call only.  Synchronises.
 */
kc_status kc_count_batch(kc_ctx* ctx, const kc_chunk* chunks_host, uint32_t n_chunks,
                         uint32_t counter, void* hip_stream, kc_stats* out_host);

/* One configuration timed by kc_autotune_batch. */
typedef struct kc_tune_trial {
  uint32_t partitions_log2;
  uint32_t table_slots;
  uint32_t scatter_bits;
  int32_t status;          /* kc_status of the trial */
  double ms;               /* fastest of the timed kc_count_batch calls */
  uint64_t overflow_keys;
  uint32_t shuffle_tile_log2;
  uint32_t reserved_;
} kc_tune_trial;

/*
 * Chooses the result-neutral parameters of kc_count_batch for a batch by
 * measurement: partition count, table slots (load factor), first-level
 * fan-out (the split of the shuffle between its two tile levels) and the
 * second-level tile size (keys per shuffle workgroup, 2^13 down to 2^11).  A
 * coordinate search starts at about one partition per 2^13 key positions,
 * the default table, the automatic split and 2^13-key tiles, and steps along
 * each dimension while a neighbour is faster (at most 28 trials).  Each trial runs
 * kc_count_batch on the batch itself, on a context of its own (the fastest
 * of two timed runs after one untimed).  The fastest configuration without
 * errors is written to *best_out (base's result-defining fields unchanged).
 * trials_host (may be NULL) receives up to max_trials records and
 * *n_trials_out their number.  Needs the memory of one batched count at a
 * time.  Synchronises.
 */
kc_status kc_autotune_batch(const kc_config* base, int device, const kc_chunk* chunks_host,
                            uint32_t n_chunks, uint32_t counter, void* hip_stream,
                            kc_config* best_out, kc_tune_trial* trials_host,
                            uint32_t max_trials, uint32_t* n_trials_out);

/*
 * Served form: a request server on one device.  A request is one count job
 * (its own configuration, and up to two read chunks, chunk c counted into
 * counter c).  Requests queue in arrival order and are admitted while the
 * device bytes of admitted, unreleased requests stay within the server's
 * HBM budget and a worker is free; admitted requests run concurrently (one
 * worker thread and stream each), so their kernels overlap on the device.  A
 * finished request keeps its context (tables, Bloom levels) resident until
 * kc_server_release; released contexts are kept for reuse by later requests
 * (of any configuration: a reused context is reconfigured and keeps its
 * buffers, which only grow) and are freed when the budget needs their memory.
 * Reservations are exact: the bytes the chosen context will hold after the
 * job.  Each request's result is exactly what kc_create + kc_insert_reads (per
 * chunk) + kc_finalize would give alone: contexts share no state.
 */
typedef struct kc_server kc_server;

typedef struct kc_request {
  kc_config cfg;        /* the job's configuration (its table budget is ignored) */
  kc_chunk parts[2];    /* parts[c] is counted into counter c */
  uint32_t n_parts;     /* 1 or 2, at most cfg.n_counters */
  uint32_t reserved_;   /* 0 */
  void* ready_event;    /* hipEvent_t recorded after the work that writes the read buffers
                           (or NULL if they are ready at submission): the worker's stream
                           waits for it before the first read is counted.  Owned by the
                           caller; it must stay valid until the request is done. */
} kc_request;

typedef struct kc_response {
  int32_t status;        /* kc_status of the job */
  uint32_t worker;       /* worker that ran it */
  kc_stats stats;        /* kc_finalize's statistics */
  kc_ctx* ctx;           /* FINALIZED context with the job's tables, valid until release; may be
                            passed to kc_query / kc_export / kc_export_bloom by the waiting thread */
  double submit_ms;      /* server clock (ms since kc_server_create) at submission */
  double admit_ms;       /* ... when a worker took it */
  double done_ms;        /* ... when kc_finalize returned */
  uint64_t footprint_bytes; /* device bytes reserved for it (estimate before, actual after) */
} kc_response;

/* Starts `workers` (1..16) worker threads on `device`, admitting requests
 * within hbm_budget_bytes of device memory (> 0). */
kc_status kc_server_create(int device, uint64_t hbm_budget_bytes, uint32_t workers,
                           kc_server** out);

/* Caps the work on the device at once: a request is admitted only while no
 * request runs, or the total bases of the running requests and its own stay
 * within max_inflight_bases.  A large request then runs alone and small ones
 * overlap.  0 (the default) sets no cap: requests are admitted as memory
 * allows.  Takes effect for admissions after the call. */
kc_status kc_server_set_overlap(kc_server* srv, uint64_t max_inflight_bases);

/* Queues a request (copied; its read buffers and ready_event must stay valid
 * until the request is done) and returns at once with its ticket.  A request whose
 * estimated footprint exceeds the whole budget finishes at once with status
 * KC_ERR_OVER_BUDGET. */
kc_status kc_server_submit(kc_server* srv, const kc_request* req, uint64_t* ticket_out);

/* Blocks until the request is done; *out receives its response.  The call
 * itself fails only for an unknown or released ticket. */
kc_status kc_server_wait(kc_server* srv, uint64_t ticket, kc_response* out);

/* Ends a done request: its tables leave the budget (the context goes to the
 * reuse pool) and the ticket becomes invalid. */
kc_status kc_server_release(kc_server* srv, uint64_t ticket);

/* State and counters of a server. */
typedef struct kc_server_stats {
  uint64_t in_use_bytes;     /* reserved by admitted, unreleased requests */
  uint64_t pooled_bytes;     /* held by pooled (released) contexts */
  uint32_t queued;           /* requests waiting for admission */
  uint32_t running;          /* requests on a worker now */
  uint32_t pooled_contexts;
  uint32_t reserved_;        /* 0 */
  uint64_t created;          /* requests given a new context */
  uint64_t reused;           /* ... a pooled context that needed no new memory */
  uint64_t grown;            /* ... a pooled context whose buffers had to grow */
  uint64_t evicted;          /* pooled contexts freed to make room */
  uint64_t cached_bytes;     /* device blocks freed by the server's contexts and kept for later
                                jobs (beyond the budget's bytes, up to the budget again) */
  uint64_t device_allocs;    /* blocks the server has taken from the runtime */
  uint64_t device_frees;     /* blocks it has given back to the runtime (past the cache limit) */
} kc_server_stats;

kc_status kc_server_usage(kc_server* srv, kc_server_stats* out);

/*
 * The server's admission rule on plain numbers (the served form's memory
 * budget, Sec. III-D; exposed so that the policy can be checked without a
 * device).  A pooled context is described by its device bytes now, the bytes
 * it would hold after the request (0: it cannot take it) and its last use.
 */
typedef struct kc_admit_pooled {
  uint64_t bytes;
  uint64_t after;
  uint64_t stamp;  /* larger = used more recently */
} kc_admit_pooled;

typedef struct kc_admit_state {
  uint64_t budget;        /* device bytes the server may use */
  uint64_t in_use;        /* bytes reserved by admitted, unreleased requests */
  uint64_t pooled;        /* bytes of the pooled contexts (the sum of their bytes) */
  uint64_t max_inflight;  /* cap on the bases of requests running at once; 0 = none */
  uint64_t inflight;      /* bases of the requests running now */
  uint32_t running;       /* requests running now */
  uint32_t reserved_;     /* 0 */
} kc_admit_state;

/*
 * Plans the admission of the request at the head of the queue: job_bases
 * bases, estimate device bytes as a new context.  *admit = 1 when it may
 * start now: its memory fits, and with a cap no request runs or the running
 * ones and it stay within max_inflight.  Then *choice is the pooled context
 * it takes (index into pool) or -1 for a new one, chosen as the smallest
 * pooled context that needs no new memory; else a new context if it fits
 * beside the reservations and every pooled context; else the pooled context
 * that grows least, if it grows by no more than a new context would take;
 * else a new context that fits once pooled contexts are freed; else the
 * least-growing pooled context.  *reserve is the bytes reserved for it, and
 * evict[0 .. *n_evict) the pooled contexts (indices into pool, least recently
 * used first; never the chosen one) to free so that reservations plus pooled
 * bytes stay within the budget.  evict has room for n_pool entries.  Pure
 * host computation; KC_ERR_INVALID_ARG for NULL outputs or a pooled sum that
 * disagrees with state->pooled.
 */
kc_status kc_server_plan_admission(const kc_admit_state* state, const kc_admit_pooled* pool,
                                   uint32_t n_pool, uint64_t job_bases, uint64_t estimate,
                                   uint32_t* admit, int32_t* choice, uint64_t* reserve,
                                   uint32_t* evict, uint32_t* n_evict);

/* Waits for running requests, drops queued ones, frees every context.  NULL
 * is ignored. */
void kc_server_destroy(kc_server* srv);

/* Frees everything the context owns.  NULL is ignored. */
void kc_destroy(kc_ctx* ctx);

/* Error text of the context's last failing call ("" if none); with NULL, the
 * last kc_create failure of this thread. */
const char* kc_last_error(const kc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
