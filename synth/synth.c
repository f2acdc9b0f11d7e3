/*
 * synth.c - seeded synthetic genomes and sequencing reads.
 *
 * Input generation only: this file produces ASCII reads and read offsets and
 * holds none of the counting method's arithmetic (no k-mer encoding, no
 * canonical form, no hashing of k-mers, no Bloom filter, no counting).  Both
 * the CPU oracle and the GPU path consume what it writes.
 *
 * Randomness is counter-based: every draw is the i-th output of a SplitMix64
 * stream (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) whose starting state is derived from
 * (master seed, tag, object id).  Any read can therefore be regenerated on its
 * own, and generating a slice of reads gives the same bytes as generating all
 * of them and cutting the slice out.
 *
 * Workload model (stand-in for the simulated Illumina reads of the paper's
 * evaluation, which are not available): uniform i.i.d. genome; each read
 * starts uniformly in [0, G - L], is taken from either strand with
 * probability 1/2, gets independent per-base substitutions to one of the
 * three other bases, and optionally per-base 'N' masking applied after the
 * substitutions.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_GAMMA 0x9E3779B97F4A7C15ULL

enum { TAG_GENOME = 1, TAG_READ = 2, TAG_CHUNK = 3, TAG_SNV = 4, TAG_INV = 5, TAG_REQ = 6 };

/* i-th output (i = 0, 1, ...) of a SplitMix64 stream whose state starts at s. */
static inline uint64_t syn_draw(uint64_t s, uint64_t i) {
  uint64_t z = s + (i + 1) * SYN_GAMMA;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t syn_stream(uint64_t seed, uint64_t tag, uint64_t id) {
  return syn_draw(syn_draw(seed, tag), id);
}

/* Uniform integer in [0, n) from a 64-bit draw (high half of the product). */
static inline uint64_t syn_below(uint64_t u, uint64_t n) {
  return (uint64_t)(((unsigned __int128)u * n) >> 64);
}

/* Bernoulli(p) from a 64-bit draw, using its top 53 bits. */
static inline int syn_bern(uint64_t u, double p) {
  return (double)(u >> 11) * (1.0 / 9007199254740992.0) < p;
}

static const char SYN_ACGT[4] = {'A', 'C', 'G', 'T'};

static inline int syn_idx(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

static inline uint8_t syn_comp(uint8_t b) {
  switch (b) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return b;
  }
}

/* ---------------------------------------------------------------- threads */

typedef void (*syn_range_fn)(void* arg, uint64_t lo, uint64_t hi);
typedef struct { syn_range_fn fn; void* arg; uint64_t lo, hi; } syn_job;

static void* syn_thread_main(void* p) {
  syn_job* j = (syn_job*)p;
  j->fn(j->arg, j->lo, j->hi);
  return NULL;
}

static void syn_parallel(syn_range_fn fn, void* arg, uint64_t n, int threads) {
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((uint64_t)threads > n) threads = n ? (int)n : 1;
  if (threads == 1) { fn(arg, 0, n); return; }
  pthread_t tid[256];
  syn_job jobs[256];
  for (int t = 0; t < threads; ++t) {
    jobs[t].fn = fn; jobs[t].arg = arg;
    jobs[t].lo = n * (uint64_t)t / (uint64_t)threads;
    jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
    pthread_create(&tid[t], NULL, syn_thread_main, &jobs[t]);
  }
  for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
}

/* ----------------------------------------------------------------- genome */

typedef struct { uint64_t key; uint8_t* out; } syn_genome_arg;

static void syn_genome_range(void* a, uint64_t lo, uint64_t hi) {
  syn_genome_arg* g = (syn_genome_arg*)a;
  for (uint64_t i = lo; i < hi; ++i) g->out[i] = (uint8_t)SYN_ACGT[syn_draw(g->key, i) >> 62];
}

/* Uniform i.i.d. genome of G bases over ACGT: base i = top two bits of draw i. */
int synth_genome(uint64_t seed, uint64_t G, uint8_t* out, int threads) {
  if (!out && G) return -1;
  syn_genome_arg a = {syn_stream(seed, TAG_GENOME, 0), out};
  syn_parallel(syn_genome_range, &a, G, threads);
  return 0;
}

/* Mutated copy of a genome: n_snv distinct positions get a uniformly chosen
 * different base, then n_inv inversions (length uniform in [inv_min, inv_max],
 * start uniform) are reverse-complemented in place, one after another. */
int synth_tumour(uint64_t seed, const uint8_t* normal, uint64_t G, uint8_t* out, uint64_t n_snv,
                 uint64_t n_inv, uint64_t inv_min, uint64_t inv_max) {
  if (G == 0 || n_snv > G || inv_min > inv_max || inv_max > G) return -1;
  memcpy(out, normal, G);
  uint8_t* used = (uint8_t*)calloc((G + 7) / 8, 1);
  if (!used) return -2;
  uint64_t key = syn_stream(seed, TAG_SNV, 0), draw = 0;
  for (uint64_t s = 0; s < n_snv;) {
    uint64_t pos = syn_below(syn_draw(key, draw++), G);
    if (used[pos >> 3] & (1u << (pos & 7))) continue;
    used[pos >> 3] |= (uint8_t)(1u << (pos & 7));
    int b = syn_idx(out[pos]);
    uint64_t alt = syn_below(syn_draw(key, draw++), 3);
    out[pos] = (uint8_t)SYN_ACGT[(b + 1 + (int)alt) & 3];
    ++s;
  }
  free(used);
  uint64_t ikey = syn_stream(seed, TAG_INV, 0);
  for (uint64_t v = 0; v < n_inv; ++v) {
    uint64_t len = inv_min + syn_below(syn_draw(ikey, 2 * v), inv_max - inv_min + 1);
    uint64_t st = syn_below(syn_draw(ikey, 2 * v + 1), G - len + 1);
    uint8_t* p = out + st;
    for (uint64_t i = 0, j = len - 1; i < j; ++i, --j) {
      uint8_t t = p[i]; p[i] = syn_comp(p[j]); p[j] = syn_comp(t);
    }
    if (len & 1) p[len / 2] = syn_comp(p[len / 2]);
  }
  return 0;
}

/* ------------------------------------------------------------------ reads */

/* Length of read r: uniform integer in [lmin, lmax] (draw 0 of its stream). */
static inline uint64_t syn_read_len(uint64_t seed, uint64_t r, uint32_t lmin, uint32_t lmax) {
  if (lmin == lmax) return lmin;
  uint64_t key = syn_stream(seed, TAG_READ, r);
  return lmin + syn_below(syn_draw(key, 0), (uint64_t)(lmax - lmin) + 1);
}

/* offsets[0..n] of reads first .. first+n-1, relative to the first one. */
int synth_read_offsets(uint64_t seed, uint64_t first, uint64_t n, uint32_t lmin, uint32_t lmax,
                       uint64_t* offsets) {
  if (lmin > lmax || !offsets) return -1;
  offsets[0] = 0;
  for (uint64_t i = 0; i < n; ++i)
    offsets[i + 1] = offsets[i] + syn_read_len(seed, first + i, lmin, lmax);
  return 0;
}

typedef struct {
  uint64_t seed, first, G;
  const uint8_t* genome;
  uint32_t lmin, lmax;
  double err, nrate;
  const uint64_t* offsets;
  uint8_t* out;
} syn_reads_arg;

static void syn_reads_range(void* a, uint64_t lo, uint64_t hi) {
  const syn_reads_arg* q = (const syn_reads_arg*)a;
  for (uint64_t i = lo; i < hi; ++i) {
    uint64_t r = q->first + i;
    uint64_t key = syn_stream(q->seed, TAG_READ, r);
    uint64_t L = q->offsets[i + 1] - q->offsets[i];
    uint8_t* dst = q->out + q->offsets[i];
    uint64_t st = syn_below(syn_draw(key, 1), q->G - L + 1);
    int minus = (int)(syn_draw(key, 2) >> 63);
    for (uint64_t j = 0; j < L; ++j)
      dst[j] = minus ? syn_comp(q->genome[st + L - 1 - j]) : q->genome[st + j];
    for (uint64_t j = 0; j < L; ++j) {
      uint64_t u = syn_draw(key, 3 + 3 * j);
      if (q->err > 0 && syn_bern(u, q->err)) {
        int b = syn_idx(dst[j]);
        uint64_t alt = syn_below(syn_draw(key, 4 + 3 * j), 3);
        dst[j] = (uint8_t)SYN_ACGT[(b + 1 + (int)alt) & 3];
      }
      if (q->nrate > 0 && syn_bern(syn_draw(key, 5 + 3 * j), q->nrate)) dst[j] = 'N';
    }
  }
}

/* Reads first .. first+n-1 written back to back into out (offsets from
 * synth_read_offsets with the same seed/first/n/lmin/lmax). */
int synth_reads(uint64_t seed, const uint8_t* genome, uint64_t G, uint64_t first, uint64_t n,
                uint32_t lmin, uint32_t lmax, double err, double nrate, const uint64_t* offsets,
                uint8_t* out, int threads) {
  if (lmax > G || lmin > lmax || !genome || !offsets || (!out && n)) return -1;
  for (uint64_t i = 0; i < n; ++i)
    if (offsets[i + 1] - offsets[i] != syn_read_len(seed, first + i, lmin, lmax)) return -2;
  syn_reads_arg a = {seed, first, G, genome, lmin, lmax, err, nrate, offsets, out};
  syn_parallel(syn_reads_range, &a, n, threads);
  return 0;
}

/* Chunk sizes floor(exp(U[ln lo, ln hi])) for a batch of read chunks. */
int synth_chunk_sizes(uint64_t seed, uint64_t n_chunks, double lo, double hi, uint64_t* out) {
  if (!(lo > 0) || hi < lo) return -1;
  uint64_t key = syn_stream(seed, TAG_CHUNK, 0);
  for (uint64_t c = 0; c < n_chunks; ++c) {
    double u = (double)(syn_draw(key, c) >> 11) * (1.0 / 9007199254740992.0);
    out[c] = (uint64_t)floor(exp(log(lo) + u * (log(hi) - log(lo))));
  }
  return 0;
}

/* Generic seeded draws for request streams: out[i] = draw i of stream (seed, TAG_REQ, id). */
int synth_draws(uint64_t seed, uint64_t id, uint64_t n, uint64_t* out) {
  uint64_t key = syn_stream(seed, TAG_REQ, id);
  for (uint64_t i = 0; i < n; ++i) out[i] = syn_draw(key, i);
  return 0;
}
