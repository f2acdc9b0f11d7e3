/*
 * kc_oracle.c - plain CPU reference of the k-mer counting path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU baseline may load this library.  It shares no code, header,
 * table or constant generator with the GPU library, and neither one includes
 * or links the other.
 *
 * What it computes (paper: Cadenelli, Polo, Carrera, "Accelerating K-mer
 * Frequency Counting with GPU and Non-Volatile Memory"):
 *   - the k-mers of a read are its length-k substrings, M-k+1 of them for a
 *     read of M bases (Sec. II-A), none spanning two reads;
 *   - a k-mer is a 64-bit code of 2 bits per base (Sec. II-A, amplification
 *     paragraph); code A=0 C=1 G=2 T=3, first base most significant;
 *     only the bytes A, C, G, T are valid bases; a window holding any other
 *     byte is skipped;
 *   - the counted key is the canonical form x = min(enc(w), enc(rc(w)));
 *   - the count table keeps k-mers seen at least min_count (>= 2) times
 *     (Sec. II-B, Count unit: unique k-mers are discarded);
 *   - Prune's two-level Bloom filter (Sec. III, Prune unit) read as
 *     saturating per-bit hit counts: B1[b] = [hits(b) >= 1],
 *     B2[b] = [hits(b) >= 2], where every occurrence of x hits each distinct
 *     bit of S(x) once; a key passes the screen iff S(x) is inside B2
 *     (Sec. III, Count unit uses the second filter); keys seen once that pass
 *     are the false-positive singletons F that Unify removes (Sec. III,
 *     Unify unit);
 *   - bit positions (the paper names no hash functions): s_i = mix64(seed +
 *     (i+1)*0x9E3779B97F4A7C15), i = 0, 1; g = mix64(x ^ s_0); block = top
 *     (m_log2 - block_log2) bits of g; with u = mix64(x ^ s_1), a = its top
 *     block_log2 bits and b = the next block_log2 bits, bit_i = block *
 *     2^block_log2 + ((a + i*b) mod 2^block_log2), i = 0..h-1 (double hashing,
 *     Kirsch and Mitzenmacher, "Less hashing, same performance", 2006); mix64
 *     is the SplitMix64 output function.
 *
 *   - stem items (Sec. II-A: the stem of a k-mer is its middle k-2 bases;
 *     Sec. III-D, Unify: counts grouped per stem into items of 16 normal and
 *     16 tumour counts of 2 bytes): for each key x of the final table, S =
 *     its middle k-2 bases; the canonical stem is min(S, rc(S)); if S is the
 *     canonical one the k-mer is read as a S b with a, b its first and last
 *     bases, otherwise as rc(x) = a rc(S) b (a = comp(last), b = comp(first));
 *     its counts go to slot 4a + b of the stem's item, counter 0 in the
 *     first 16 slots and counter 1 in the last 16, each saturated to 65535.
 *
 *   - Filter-unit lookup (Sec. II-B, Filter unit: the input sequences are
 *     read again and their k-mers looked up in the frequency table to select
 *     k-mers with imbalanced frequencies; the imbalance test itself is not
 *     given): with (normal, tumour) = the final table's counters 0 and 1 of
 *     the window's canonical k-mer ((0, 0) for a k-mer not in the table; a
 *     one-counter table reads as normal 0, tumour = its count), a window is
 *     selected iff tumour >= tumour_min and normal <= normal_max; the result
 *     per read is its number of selected windows.
 *
 * Algorithm: enumerate every valid window, push its canonical key, sort
 * (libc qsort), run-length encode into (x, counts), then derive B1/B2 from
 * the run-length list with the saturating update, then the screen, F and the
 * table.  All integer arithmetic, no floating point.  Inputs too large to
 * sort at once go through or_count_ranges: the same steps one value range of
 * the k-mer space at a time (see the comment above it).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_GAMMA 0x9E3779B97F4A7C15ULL

typedef struct {
  uint32_t k;          /* 1..31 */
  uint32_t n_counters; /* 1 or 2 */
  uint32_t min_count;  /* >= 2 */
  uint32_t m_log2;     /* Bloom bits per level = 2^m_log2 */
  uint32_t h;          /* hash functions, 1..8 */
  uint32_t block_log2; /* 1..m_log2 */
  uint64_t seed;
} or_params;

typedef struct {
  uint64_t n_valid, n_distinct, n_pass, entries, sum_counts, fp_singletons, b1_pop, b2_pop;
} or_stats;

typedef struct {
  or_stats st;
  uint64_t n_entries;
  uint64_t* keys;   /* [n_entries], ascending */
  uint32_t* counts; /* [n_entries * n_counters] */
  uint64_t m_words;
  uint64_t* b1;     /* [m_words] little-endian bit order: bit b in word b>>6, bit b&63 */
  uint64_t* b2;
  /* want_bloom = 2: the levels' nonzero words only (level 2 is zero where
   * level 1 is): their indices, ascending, and both levels' words there */
  uint64_t n_touched;
  uint64_t* touched;
  uint64_t* t1;
  uint64_t* t2;
} or_result;

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014). */
uint64_t or_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static int or_code(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

static int or_params_ok(const or_params* p) {
  if (p->k < 1 || p->k > 31) return 0;
  if (p->n_counters < 1 || p->n_counters > 2) return 0;
  if (p->min_count < 2) return 0;
  if (p->h < 1 || p->h > 8) return 0;
  /* a and b are the top two block_log2-bit fields of one 64-bit hash, so a
   * block holds at most 2^32 bits */
  if (p->block_log2 < 1 || p->block_log2 > 32 || p->block_log2 > p->m_log2 || p->m_log2 > 40)
    return 0;
  return 1;
}

/* Window w = s[0..k-1].  enc(w) = sum_j code(w_j) * 4^(k-1-j), evaluated in
 * Horner form.  rc(w)_j = complement of w_{k-1-j}, complement(c) = 3 - c.
 * Returns 0 when the window holds a byte other than A, C, G, T. */
static int or_window(const uint8_t* s, uint32_t k, uint64_t* fwd, uint64_t* rev) {
  uint64_t f = 0, r = 0;
  for (uint32_t j = 0; j < k; ++j) {
    int c = or_code(s[j]);
    if (c < 0) return 0;
    f = f * 4 + (uint64_t)c;
  }
  for (uint32_t j = 0; j < k; ++j) r = r * 4 + (uint64_t)(3 - or_code(s[k - 1 - j]));
  *fwd = f;
  *rev = r;
  return 1;
}

/* Canonical key of the window starting at s (assumed valid). */
static uint64_t or_canonical(const uint8_t* s, uint32_t k, int* ok) {
  uint64_t f = 0, r = 0;
  *ok = or_window(s, k, &f, &r);
  return f < r ? f : r;
}

/* Distinct Bloom bit positions of key x; returns how many (<= h). */
static uint32_t or_bloom_positions(const or_params* p, const uint64_t* salt, uint64_t x,
                                   uint64_t* pos) {
  uint32_t sb = p->m_log2 - p->block_log2;
  uint64_t g = or_mix64(x ^ salt[0]);
  uint64_t block = sb ? (g >> (64 - sb)) : 0;
  uint64_t mask = (1ull << p->block_log2) - 1;
  uint64_t u = or_mix64(x ^ salt[1]);
  uint64_t a = u >> (64 - p->block_log2);
  uint64_t b = (u >> (64 - 2 * p->block_log2)) & mask;
  uint32_t n = 0;
  for (uint32_t i = 0; i < p->h; ++i) {
    uint64_t q = (block << p->block_log2) | ((a + (uint64_t)i * b) & mask);
    int dup = 0;
    for (uint32_t j = 0; j < n; ++j) dup |= (pos[j] == q);
    if (!dup) pos[n++] = q;
  }
  return n;
}

static void or_salts(const or_params* p, uint64_t* salt) {
  for (uint32_t i = 0; i <= p->h; ++i) salt[i] = or_mix64(p->seed + (uint64_t)(i + 1) * OR_GAMMA);
}

static int or_cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

static inline int or_bit(const uint64_t* v, uint64_t b) { return (int)((v[b >> 6] >> (b & 63)) & 1); }
static inline void or_set(uint64_t* v, uint64_t b) { v[b >> 6] |= 1ULL << (b & 63); }

/* Every valid window's canonical key in read order, tagged (key << 1 | tag)
 * where tag is the read's counter (0 when tags is NULL).  Returns the count,
 * or UINT64_MAX when out is too small. */
uint64_t or_enumerate(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                      uint64_t n_reads, const uint8_t* tags, uint64_t* out, uint64_t cap) {
  uint64_t n = 0;
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t lo = offsets[r], hi = offsets[r + 1];
    if (hi - lo < p->k) continue;
    for (uint64_t s = lo; s + p->k <= hi; ++s) {
      int ok;
      uint64_t x = or_canonical(bases + s, p->k, &ok);
      if (!ok) continue;
      if (out) {
        if (n >= cap) return UINT64_MAX;
        out[n] = (x << 1) | (uint64_t)(tags ? tags[r] : 0);
      }
      ++n;
    }
  }
  return n;
}

void or_free(or_result* r) {
  if (!r) return;
  free(r->keys);
  free(r->counts);
  free(r->b1);
  free(r->b2);
  free(r->touched);
  free(r->t1);
  free(r->t2);
  free(r);
}

/* Hands the levels to the result: whole (want_bloom = 1), as their nonzero
 * words (2), or not at all (0).  Returns 0, or -1 when out of memory. */
static int or_give_bloom(or_result* res, uint64_t* b1, uint64_t* b2, uint64_t m_words,
                         int want_bloom) {
  res->m_words = m_words;
  if (want_bloom == 1) {
    res->b1 = b1;
    res->b2 = b2;
    return 0;
  }
  int rc = 0;
  if (want_bloom == 2) {
    uint64_t n = 0;
    for (uint64_t w = 0; w < m_words; ++w) n += b1[w] != 0;
    res->touched = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    res->t1 = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    res->t2 = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    if (res->touched && res->t1 && res->t2) {
      uint64_t j = 0;
      for (uint64_t w = 0; w < m_words; ++w)
        if (b1[w]) {
          res->touched[j] = w;
          res->t1[j] = b1[w];
          res->t2[j] = b2[w];
          ++j;
        }
      res->n_touched = n;
    } else {
      rc = -1;
    }
  }
  free(b1);
  free(b2);
  return rc;
}

/* Full count.  want_bloom = 0 skips returning B1/B2 (they are still used);
 * 2 returns their nonzero words only. */
or_result* or_count(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                    uint64_t n_reads, const uint8_t* tags, int want_bloom) {
  if (!or_params_ok(p)) return NULL;
  if (offsets[0] != 0) return NULL;
  for (uint64_t r = 0; r < n_reads; ++r)
    if (offsets[r + 1] < offsets[r]) return NULL;
  if (tags)
    for (uint64_t r = 0; r < n_reads; ++r)
      if (tags[r] >= p->n_counters) return NULL;

  or_result* res = (or_result*)calloc(1, sizeof(or_result));
  if (!res) return NULL;
  uint32_t nc = p->n_counters;

  /* 1. enumerate W and push tagged canonical keys */
  uint64_t n = or_enumerate(p, bases, offsets, n_reads, tags, NULL, 0);
  uint64_t* occ = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!occ) { or_free(res); return NULL; }
  or_enumerate(p, bases, offsets, n_reads, tags, occ, n);
  res->st.n_valid = n;

  /* 2. sort and run-length encode into (x, c_0 .. c_{nc-1}) */
  qsort(occ, n, sizeof(uint64_t), or_cmp_u64);
  uint64_t nd = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (i == 0 || (occ[i] >> 1) != (occ[i - 1] >> 1)) ++nd;
  uint64_t* rk = (uint64_t*)malloc((nd ? nd : 1) * sizeof(uint64_t));
  uint32_t* rc = (uint32_t*)calloc((nd ? nd : 1) * nc, sizeof(uint32_t));
  if (!rk || !rc) { free(occ); free(rk); free(rc); or_free(res); return NULL; }
  uint64_t d = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (i == 0 || (occ[i] >> 1) != (occ[i - 1] >> 1)) rk[d++] = occ[i] >> 1;
    rc[(d - 1) * nc + (occ[i] & 1)] += 1;
  }
  free(occ);
  res->st.n_distinct = nd;

  /* 3. Bloom levels from the run-length list: hits2[b] = min(2, hits2[b] + c)
   *    kept as two bit arrays, B1 = (hits >= 1), B2 = (hits >= 2). */
  uint64_t m_words = p->m_log2 >= 6 ? (1ULL << (p->m_log2 - 6)) : 1;
  uint64_t* b1 = (uint64_t*)calloc(m_words, sizeof(uint64_t));
  uint64_t* b2 = (uint64_t*)calloc(m_words, sizeof(uint64_t));
  if (!b1 || !b2) { free(rk); free(rc); free(b1); free(b2); or_free(res); return NULL; }
  uint64_t salt[9], pos[8];
  or_salts(p, salt);
  for (uint64_t i = 0; i < nd; ++i) {
    uint64_t c = 0;
    for (uint32_t t = 0; t < nc; ++t) c += rc[i * nc + t];
    uint32_t np = or_bloom_positions(p, salt, rk[i], pos);
    for (uint32_t j = 0; j < np; ++j) {
      if (c >= 2 || or_bit(b1, pos[j])) or_set(b2, pos[j]);
      or_set(b1, pos[j]);
    }
  }
  for (uint64_t w = 0; w < m_words; ++w) {
    res->st.b1_pop += (uint64_t)__builtin_popcountll(b1[w]);
    res->st.b2_pop += (uint64_t)__builtin_popcountll(b2[w]);
  }

  /* 4. screen every distinct key against B2; F, N_pass; the final table */
  uint64_t ne = 0;
  for (uint64_t i = 0; i < nd; ++i) {
    uint64_t c = 0;
    for (uint32_t t = 0; t < nc; ++t) c += rc[i * nc + t];
    uint32_t np = or_bloom_positions(p, salt, rk[i], pos);
    int pass = 1;
    for (uint32_t j = 0; j < np; ++j) pass &= or_bit(b2, pos[j]);
    if (pass) {
      res->st.n_pass += c;
      if (c == 1) res->st.fp_singletons += 1;
    }
    if (c >= p->min_count) ++ne;
  }
  res->keys = (uint64_t*)malloc((ne ? ne : 1) * sizeof(uint64_t));
  res->counts = (uint32_t*)malloc((ne ? ne : 1) * nc * sizeof(uint32_t));
  if (!res->keys || !res->counts) { free(rk); free(rc); free(b1); free(b2); or_free(res); return NULL; }
  uint64_t e = 0;
  for (uint64_t i = 0; i < nd; ++i) {
    uint64_t c = 0;
    for (uint32_t t = 0; t < nc; ++t) c += rc[i * nc + t];
    if (c < p->min_count) continue;
    res->keys[e] = rk[i];
    for (uint32_t t = 0; t < nc; ++t) res->counts[e * nc + t] = rc[i * nc + t];
    res->st.sum_counts += c;
    ++e;
  }
  res->n_entries = ne;
  res->st.entries = ne;
  free(rk);
  free(rc);
  if (or_give_bloom(res, b1, b2, m_words, want_bloom)) {
    or_free(res);
    return NULL;
  }
  return res;
}

/* Bloom bit positions of one key (distinct, in hash order); returns count,
 * or 0 when the parameters are out of range. */
uint32_t or_bloom_bits(const or_params* p, uint64_t x, uint64_t* out) {
  if (!or_params_ok(p)) return 0;
  uint64_t salt[9];
  or_salts(p, salt);
  return or_bloom_positions(p, salt, x, out);
}

/* ------------------------------------------------------------ stem items */
typedef struct {
  uint64_t stem;
  uint32_t slot;
  uint32_t c[2];
} or_stem_rec;

static int or_cmp_stem(const void* a, const void* b) {
  const or_stem_rec* x = (const or_stem_rec*)a;
  const or_stem_rec* y = (const or_stem_rec*)b;
  if (x->stem != y->stem) return x->stem < y->stem ? -1 : 1;
  return x->slot < y->slot ? -1 : (x->slot > y->slot);
}

/* Reverse complement of the n-base code v (first base most significant). */
static uint64_t or_revcomp(uint64_t v, uint32_t n) {
  uint64_t r = 0;
  for (uint32_t i = 0; i < n; ++i) {
    r = (r << 2) | (3u - (v & 3u));
    v >>= 2;
  }
  return r;
}

/* Stem items of a final table (keys[n], counts[n * n_counters]), sorted by
 * stem; *stems_out[*n_out] and *items_out[*n_out * 32] are malloc'd (the
 * caller frees them with or_free_ptr).  Returns 0, or -1 for k < 3 or a
 * failed allocation. */
int or_stem_items(uint32_t k, uint32_t n_counters, const uint64_t* keys, const uint32_t* counts,
                  uint64_t n, uint64_t** stems_out, uint16_t** items_out, uint64_t* n_out) {
  *stems_out = NULL;
  *items_out = NULL;
  *n_out = 0;
  if (k < 3 || k > 31 || n_counters < 1 || n_counters > 2) return -1;
  const uint32_t m = k - 2;
  const uint64_t mmask = (1ULL << (2 * m)) - 1;
  or_stem_rec* rec = (or_stem_rec*)malloc((n ? n : 1) * sizeof(or_stem_rec));
  if (!rec) return -1;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t x = keys[i];
    const uint32_t first = (uint32_t)(x >> (2 * (k - 1))) & 3u, last = (uint32_t)(x & 3u);
    const uint64_t s = (x >> 2) & mmask;
    const uint64_t rs = or_revcomp(s, m);
    uint32_t a = first, b = last;
    uint64_t stem = s;
    if (rs < s) {
      stem = rs;
      a = 3u - last;
      b = 3u - first;
    }
    rec[i].stem = stem;
    rec[i].slot = 4u * a + b;
    for (uint32_t t = 0; t < 2; ++t) {
      const uint32_t c = t < n_counters ? counts[i * n_counters + t] : 0u;
      rec[i].c[t] = c > 65535u ? 65535u : c;
    }
  }
  qsort(rec, n, sizeof(or_stem_rec), or_cmp_stem);
  uint64_t items = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (i == 0 || rec[i].stem != rec[i - 1].stem) ++items;
  uint64_t* stems = (uint64_t*)malloc((items ? items : 1) * 8);
  uint16_t* it = (uint16_t*)calloc((items ? items : 1) * 32, 2);
  if (!stems || !it) {
    free(rec);
    free(stems);
    free(it);
    return -1;
  }
  uint64_t j = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (i == 0 || rec[i].stem != rec[i - 1].stem) stems[j++] = rec[i].stem;
    uint16_t* row = it + (j - 1) * 32;
    row[rec[i].slot] = (uint16_t)rec[i].c[0];
    row[16 + rec[i].slot] = (uint16_t)rec[i].c[1];
  }
  free(rec);
  *stems_out = stems;
  *items_out = it;
  *n_out = items;
  return 0;
}

void or_free_ptr(void* p) { free(p); }

/* -------------------------------------------------------- filter lookup */
static int64_t or_find(const uint64_t* a, uint64_t n, uint64_t v);
/* out[r] = selected windows of read r (see the header); keys[n_keys] is the
 * final table in ascending order with counts[n_keys * n_counters].  Windows
 * are those the count enumerates (valid bases only, inside one read).
 * Returns 0, or -1 for bad arguments. */
int or_filter_reads(uint32_t k, uint32_t n_counters, const uint64_t* keys, const uint32_t* counts,
                    uint64_t n_keys, const uint8_t* bases, const uint64_t* offsets, uint64_t n_reads,
                    uint32_t tumour_min, uint32_t normal_max, uint32_t* out) {
  if (k < 1 || k > 31 || n_counters < 1 || n_counters > 2) return -1;
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint32_t sel = 0;
    const uint64_t lo = offsets[r], hi = offsets[r + 1];
    for (uint64_t j = lo; j + k <= hi; ++j) {
      int ok = 0;
      const uint64_t x = or_canonical(bases + j, k, &ok);
      if (!ok) continue;
      uint32_t normal = 0, tumour = 0;
      const int64_t at = or_find(keys, n_keys, x);
      if (at >= 0) {
        if (n_counters == 2) {
          normal = counts[(uint64_t)at * 2];
          tumour = counts[(uint64_t)at * 2 + 1];
        } else {
          tumour = counts[at];
        }
      }
      if (tumour >= tumour_min && normal <= normal_max) ++sel;
    }
    out[r] = sel;
  }
  return 0;
}

/* ------------------------------------------------------ sampled checking */
/* For workloads too large to sort on the host: exact counts of a sorted list
 * of sample keys, and exact saturating hits of a sorted list of bit
 * positions, each found by scanning every window (threads split the reads). */

typedef struct {
  const or_params* p;
  const uint8_t* bases;
  const uint64_t* offsets;
  const uint8_t* tags;
  const uint64_t* sample;
  uint64_t n_sample;
  uint32_t* counts; /* per thread [n_sample * n_counters] */
  uint64_t n_valid;
  uint64_t lo, hi;
  const uint64_t* salt;
  const uint64_t* blocks; /* mode 1: sorted Bloom blocks of the sampled bits */
  uint64_t n_blocks;
  int mode; /* 0 = key counts, 1 = bit hits */
} or_scan_job;

static int64_t or_find(const uint64_t* a, uint64_t n, uint64_t v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == v) ? (int64_t)lo : -1;
}

static void* or_scan_main(void* arg) {
  or_scan_job* j = (or_scan_job*)arg;
  const or_params* p = j->p;
  uint64_t pos[8];
  for (uint64_t r = j->lo; r < j->hi; ++r) {
    uint64_t lo = j->offsets[r], hi = j->offsets[r + 1];
    if (hi - lo < p->k) continue;
    for (uint64_t s = lo; s + p->k <= hi; ++s) {
      int ok;
      uint64_t x = or_canonical(j->bases + s, p->k, &ok);
      if (!ok) continue;
      j->n_valid++;
      if (j->mode == 0) {
        int64_t at = or_find(j->sample, j->n_sample, x);
        if (at >= 0) j->counts[at * p->n_counters + (j->tags ? j->tags[r] : 0)] += 1;
      } else {
        /* every bit of S(x) lies in x's block: skip keys of other blocks */
        uint32_t sb = p->m_log2 - p->block_log2;
        uint64_t block = sb ? (or_mix64(x ^ j->salt[0]) >> (64 - sb)) : 0;
        if (or_find(j->blocks, j->n_blocks, block) < 0) continue;
        uint32_t np = or_bloom_positions(p, j->salt, x, pos);
        for (uint32_t q = 0; q < np; ++q) {
          int64_t at = or_find(j->sample, j->n_sample, pos[q]);
          if (at >= 0 && j->counts[at] < 2) j->counts[at] += 1;
        }
      }
    }
  }
  return NULL;
}

static int or_scan(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                   uint64_t n_reads, const uint8_t* tags, const uint64_t* sample,
                   uint64_t n_sample, uint32_t* out, uint64_t* n_valid, int threads, int mode) {
  if (!or_params_ok(p)) return -1;
  for (uint64_t i = 1; i < n_sample; ++i)
    if (sample[i] <= sample[i - 1]) return -2;
  if (threads < 1) threads = 1;
  if (threads > 128) threads = 128;
  uint64_t salt[9];
  or_salts(p, salt);
  uint64_t width = mode == 0 ? p->n_counters : 1;
  uint64_t* blocks = (uint64_t*)malloc((n_sample ? n_sample : 1) * sizeof(uint64_t));
  uint64_t n_blocks = 0;
  for (uint64_t i = 0; i < n_sample; ++i) { /* sample is sorted, so are its blocks */
    uint64_t b = sample[i] >> p->block_log2;
    if (!n_blocks || blocks[n_blocks - 1] != b) blocks[n_blocks++] = b;
  }
  or_scan_job jobs[128];
  pthread_t tid[128];
  for (int t = 0; t < threads; ++t) {
    or_scan_job* j = &jobs[t];
    memset(j, 0, sizeof(*j));
    j->p = p; j->bases = bases; j->offsets = offsets; j->tags = tags;
    j->sample = sample; j->n_sample = n_sample; j->salt = salt; j->mode = mode;
    j->blocks = blocks; j->n_blocks = n_blocks;
    j->counts = (uint32_t*)calloc((n_sample ? n_sample : 1) * width, sizeof(uint32_t));
    j->lo = n_reads * (uint64_t)t / (uint64_t)threads;
    j->hi = n_reads * (uint64_t)(t + 1) / (uint64_t)threads;
    pthread_create(&tid[t], NULL, or_scan_main, j);
  }
  uint64_t nv = 0;
  memset(out, 0, n_sample * width * sizeof(uint32_t));
  for (int t = 0; t < threads; ++t) {
    pthread_join(tid[t], NULL);
    nv += jobs[t].n_valid;
    for (uint64_t i = 0; i < n_sample * width; ++i) {
      out[i] += jobs[t].counts[i];
      if (mode == 1 && out[i] > 2) out[i] = 2;
    }
    free(jobs[t].counts);
  }
  free(blocks);
  if (n_valid) *n_valid = nv;
  return 0;
}

/* Exact counts of the sorted, distinct canonical keys in sample. */
int or_sample_counts(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                     uint64_t n_reads, const uint8_t* tags, const uint64_t* sample,
                     uint64_t n_sample, uint32_t* out, uint64_t* n_valid, int threads) {
  return or_scan(p, bases, offsets, n_reads, tags, sample, n_sample, out, n_valid, threads, 0);
}

/* min(2, hits(b)) for the sorted, distinct bit positions in sample. */
int or_sample_hits(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                   uint64_t n_reads, const uint64_t* sample, uint64_t n_sample, uint32_t* out,
                   int threads) {
  return or_scan(p, bases, offsets, n_reads, NULL, sample, n_sample, out, NULL, threads, 1);
}

/* --------------------------------------------------- value-range passes */
/* The same result as or_count, for inputs whose keys do not fit in memory
 * at once.  The k-mer space is cut into Q = 2^qbits value ranges by the top
 * qbits of the 2k-bit code (SMUFIN splits its work into partitions of the
 * k-mer space and re-reads the input once per partition, Sec. II-B).  A pass
 * takes `threads` consecutive ranges, one per thread: the threads split the
 * reads, enumerate every valid window and keep the keys of the pass's ranges
 * in one bucket per (thread, range); then each thread gathers one range's
 * buckets, sorts them (libc qsort) and run-length encodes them.  The ranges
 * are value ranges, so their tables concatenated in range order are the
 * sorted table.  B1/B2 take every range's run-length list with the
 * saturating update of or_count, made with atomic OR so that the order in
 * which ranges finish does not matter: a bit is set in level 2 by a key seen
 * at least twice, or by the second of two keys that hit it (the atomic OR
 * returns the level-1 word as it was).  The screen needs the final level 2,
 * so it runs after the last pass: either over the keys seen once, kept from
 * the passes (a key seen at least twice always passes: each bit of S(x) has
 * at least c(x) >= 2 hits, so N_pass = sum of c over keys with c >= 2, plus
 * F), or, with keep_singles = 0, by a second round of passes that screens
 * every distinct key. */

typedef struct {
  uint64_t* v;
  uint64_t n, cap;
} or_vec64;

typedef struct {
  uint32_t* v;
  uint64_t n, cap;
} or_vec32;

static int or_push64(or_vec64* a, uint64_t x) {
  if (a->n == a->cap) {
    uint64_t c = a->cap ? a->cap + a->cap / 2 : 4096;
    uint64_t* v = (uint64_t*)realloc(a->v, c * sizeof(uint64_t));
    if (!v) return -1;
    a->v = v;
    a->cap = c;
  }
  a->v[a->n++] = x;
  return 0;
}

static int or_push32(or_vec32* a, uint32_t x) {
  if (a->n == a->cap) {
    uint64_t c = a->cap ? a->cap + a->cap / 2 : 4096;
    uint32_t* v = (uint32_t*)realloc(a->v, c * sizeof(uint32_t));
    if (!v) return -1;
    a->v = v;
    a->cap = c;
  }
  a->v[a->n++] = x;
  return 0;
}

static void or_vfree64(or_vec64* a) {
  free(a->v);
  a->v = NULL;
  a->n = a->cap = 0;
}

static void or_vfree32(or_vec32* a) {
  free(a->v);
  a->v = NULL;
  a->n = a->cap = 0;
}

typedef struct {
  uint64_t n_distinct, sum_ge2, entries, sum_counts, n_pass, fp;
} or_range_stats;

/* Receives the final table of value range q (keys ascending, n_counters
 * counts each) once the pass holding q is done; ranges arrive in ascending
 * order.  With a callback the table is handed over range by range instead of
 * being gathered into the result. */
typedef void (*or_range_cb)(void* user, uint64_t q, const uint64_t* keys, const uint32_t* counts,
                            uint64_t n);

typedef struct {
  const or_params* p;
  const uint8_t* bases;
  const uint64_t* offsets;
  uint64_t n_reads;
  const uint8_t* tags;
  const uint64_t* salt;
  uint32_t qbits, threads;
  int keep_singles;
  int sweep;             /* 1: counts, Bloom, table; 2: screen every key */
  uint64_t q0;           /* first range of the pass */
  uint64_t* b1;
  uint64_t* b2;
  or_vec64* bucket;      /* [threads * threads]: thread t, range q0 + j */
  or_vec64* tkeys;       /* [Q] table keys per range */
  or_vec32* tcounts;     /* [Q] their counts, n_counters each */
  or_vec64* singles;     /* [Q] keys seen once (keep_singles) */
  or_range_stats* rst;   /* [Q] */
  uint64_t* nvalid;      /* [threads] */
  int* fail;             /* [threads] */
  or_range_cb cb;        /* NULL: gather the table into the result */
  void* cb_user;
} or_rp;

typedef struct {
  or_rp* rp;
  uint32_t t;
} or_rp_job;

static uint64_t or_range_of(const or_params* p, uint32_t qbits, uint64_t x) {
  return qbits ? x >> (2 * p->k - qbits) : 0;
}

/* Enumeration: thread t takes its share of the reads and keeps the keys of
 * the pass's ranges, tagged (x << 1 | counter) as or_enumerate does. */
static void* or_rp_enum(void* arg) {
  or_rp_job* j = (or_rp_job*)arg;
  or_rp* rp = j->rp;
  const or_params* p = rp->p;
  const uint32_t T = rp->threads;
  const uint64_t lo = rp->n_reads * (uint64_t)j->t / T, hi = rp->n_reads * (uint64_t)(j->t + 1) / T;
  uint64_t nv = 0;
  for (uint64_t r = lo; r < hi; ++r) {
    const uint64_t a = rp->offsets[r], b = rp->offsets[r + 1];
    if (b - a < p->k) continue;
    for (uint64_t s = a; s + p->k <= b; ++s) {
      int ok;
      const uint64_t x = or_canonical(rp->bases + s, p->k, &ok);
      if (!ok) continue;
      ++nv;
      const uint64_t q = or_range_of(p, rp->qbits, x);
      if (q < rp->q0 || q - rp->q0 >= T) continue;
      const uint64_t tagged = (x << 1) | (uint64_t)(rp->tags ? rp->tags[r] : 0);
      if (or_push64(&rp->bucket[(uint64_t)j->t * T + (q - rp->q0)], tagged)) {
        rp->fail[j->t] = 1;
        return NULL;
      }
    }
  }
  rp->nvalid[j->t] = nv;
  return NULL;
}

/* One range: gather its buckets, sort, run-length encode, then (sweep 1) the
 * Bloom update, the table and the kept singletons, or (sweep 2) the screen. */
static void* or_rp_range(void* arg) {
  or_rp_job* j = (or_rp_job*)arg;
  or_rp* rp = j->rp;
  const or_params* p = rp->p;
  const uint32_t T = rp->threads, nc = p->n_counters;
  const uint64_t q = rp->q0 + j->t;
  if (q >= (1ull << rp->qbits)) return NULL;
  uint64_t n = 0;
  for (uint32_t i = 0; i < T; ++i) n += rp->bucket[(uint64_t)i * T + j->t].n;
  uint64_t* occ = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!occ) {
    rp->fail[j->t] = 1;
    return NULL;
  }
  uint64_t at = 0;
  for (uint32_t i = 0; i < T; ++i) {
    or_vec64* b = &rp->bucket[(uint64_t)i * T + j->t];
    if (b->n) memcpy(occ + at, b->v, b->n * sizeof(uint64_t));
    at += b->n;
    or_vfree64(b);
  }
  qsort(occ, n, sizeof(uint64_t), or_cmp_u64);
  or_range_stats* st = &rp->rst[q];
  uint64_t pos[8];
  for (uint64_t i = 0; i < n;) {
    const uint64_t x = occ[i] >> 1;
    uint32_t c[2] = {0, 0};
    uint64_t e = i;
    for (; e < n && (occ[e] >> 1) == x; ++e) c[occ[e] & 1] += 1;
    i = e;
    const uint64_t tot = (uint64_t)c[0] + c[1];
    const uint32_t np = or_bloom_positions(p, rp->salt, x, pos);
    if (rp->sweep == 1) {
      st->n_distinct += 1;
      if (tot >= 2) st->sum_ge2 += tot;
      for (uint32_t k = 0; k < np; ++k) {
        const uint64_t bit = 1ULL << (pos[k] & 63);
        if (tot >= 2) {
          __atomic_fetch_or(&rp->b1[pos[k] >> 6], bit, __ATOMIC_RELAXED);
          __atomic_fetch_or(&rp->b2[pos[k] >> 6], bit, __ATOMIC_RELAXED);
        } else {
          const uint64_t old = __atomic_fetch_or(&rp->b1[pos[k] >> 6], bit, __ATOMIC_RELAXED);
          if (old & bit) __atomic_fetch_or(&rp->b2[pos[k] >> 6], bit, __ATOMIC_RELAXED);
        }
      }
      int bad = 0;
      if (tot >= p->min_count) {
        st->entries += 1;
        st->sum_counts += tot;
        bad |= or_push64(&rp->tkeys[q], x);
        for (uint32_t t = 0; t < nc; ++t) bad |= or_push32(&rp->tcounts[q], c[t]);
      }
      if (tot == 1 && rp->keep_singles) bad |= or_push64(&rp->singles[q], x);
      if (bad) {
        rp->fail[j->t] = 1;
        break;
      }
    } else {
      int pass = 1;
      for (uint32_t k = 0; k < np; ++k) pass &= or_bit(rp->b2, pos[k]);
      if (pass) {
        st->n_pass += tot;
        if (tot == 1) st->fp += 1;
      }
    }
  }
  free(occ);
  return NULL;
}

/* Screen of the kept singletons of ranges j, j + threads, ... */
static void* or_rp_screen_singles(void* arg) {
  or_rp_job* j = (or_rp_job*)arg;
  or_rp* rp = j->rp;
  uint64_t pos[8];
  for (uint64_t q = j->t; q < (1ull << rp->qbits); q += rp->threads) {
    or_range_stats* st = &rp->rst[q];
    for (uint64_t i = 0; i < rp->singles[q].n; ++i) {
      const uint32_t np = or_bloom_positions(rp->p, rp->salt, rp->singles[q].v[i], pos);
      int pass = 1;
      for (uint32_t k = 0; k < np; ++k) pass &= or_bit(rp->b2, pos[k]);
      st->fp += (uint64_t)pass;
    }
    or_vfree64(&rp->singles[q]);
  }
  return NULL;
}

static int or_rp_run(or_rp* rp, void* (*fn)(void*)) {
  const uint32_t T = rp->threads;
  pthread_t* tid = (pthread_t*)malloc(T * sizeof(pthread_t));
  or_rp_job* jobs = (or_rp_job*)malloc(T * sizeof(or_rp_job));
  if (!tid || !jobs) {
    free(tid);
    free(jobs);
    return -1;
  }
  uint32_t started = 0;
  int bad = 0;
  for (uint32_t t = 0; t < T; ++t) {
    jobs[t].rp = rp;
    jobs[t].t = t;
    if (pthread_create(&tid[t], NULL, fn, &jobs[t])) {
      bad = 1;
      break;
    }
    ++started;
  }
  for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
  for (uint32_t t = 0; t < T; ++t) bad |= rp->fail[t];
  free(tid);
  free(jobs);
  return bad ? -1 : 0;
}

/* Passes over all ranges: enumeration, then one range per thread. */
static int or_rp_sweep(or_rp* rp, int sweep, uint64_t* n_valid) {
  const uint64_t Q = 1ull << rp->qbits;
  rp->sweep = sweep;
  for (uint64_t q0 = 0; q0 < Q; q0 += rp->threads) {
    rp->q0 = q0;
    if (or_rp_run(rp, or_rp_enum)) return -1;
    if (n_valid && q0 == 0) {
      *n_valid = 0;
      for (uint32_t t = 0; t < rp->threads; ++t) *n_valid += rp->nvalid[t];
    }
    if (or_rp_run(rp, or_rp_range)) return -1;
    if (sweep == 1 && rp->cb)
      for (uint64_t q = q0; q < q0 + rp->threads && q < Q; ++q) {
        rp->cb(rp->cb_user, q, rp->tkeys[q].v, rp->tcounts[q].v, rp->tkeys[q].n);
        or_vfree64(&rp->tkeys[q]);
        or_vfree32(&rp->tcounts[q]);
      }
  }
  return 0;
}

or_result* or_count_ranges(const or_params* p, const uint8_t* bases, const uint64_t* offsets,
                           uint64_t n_reads, const uint8_t* tags, int want_bloom, uint32_t qbits,
                           int threads, int keep_singles, or_range_cb cb, void* cb_user) {
  if (!or_params_ok(p)) return NULL;
  if (qbits > 2 * p->k || qbits > 20 || threads < 1 || threads > 256) return NULL;
  if (offsets[0] != 0) return NULL;
  for (uint64_t r = 0; r < n_reads; ++r)
    if (offsets[r + 1] < offsets[r]) return NULL;
  if (tags)
    for (uint64_t r = 0; r < n_reads; ++r)
      if (tags[r] >= p->n_counters) return NULL;
  const uint32_t T = (uint32_t)threads, nc = p->n_counters;
  const uint64_t Q = 1ull << qbits;
  uint64_t salt[9];
  or_salts(p, salt);
  or_rp rp;
  memset(&rp, 0, sizeof(rp));
  rp.p = p;
  rp.bases = bases;
  rp.offsets = offsets;
  rp.n_reads = n_reads;
  rp.tags = tags;
  rp.salt = salt;
  rp.qbits = qbits;
  rp.threads = T;
  rp.keep_singles = keep_singles;
  rp.cb = cb;
  rp.cb_user = cb_user;
  const uint64_t m_words = p->m_log2 >= 6 ? (1ULL << (p->m_log2 - 6)) : 1;
  rp.b1 = (uint64_t*)calloc(m_words, sizeof(uint64_t));
  rp.b2 = (uint64_t*)calloc(m_words, sizeof(uint64_t));
  rp.bucket = (or_vec64*)calloc((uint64_t)T * T, sizeof(or_vec64));
  rp.tkeys = (or_vec64*)calloc(Q, sizeof(or_vec64));
  rp.tcounts = (or_vec32*)calloc(Q, sizeof(or_vec32));
  rp.singles = (or_vec64*)calloc(Q, sizeof(or_vec64));
  rp.rst = (or_range_stats*)calloc(Q, sizeof(or_range_stats));
  rp.nvalid = (uint64_t*)calloc(T, sizeof(uint64_t));
  rp.fail = (int*)calloc(T, sizeof(int));
  or_result* res = (or_result*)calloc(1, sizeof(or_result));
  int ok = rp.b1 && rp.b2 && rp.bucket && rp.tkeys && rp.tcounts && rp.singles && rp.rst &&
           rp.nvalid && rp.fail && res;
  uint64_t n_valid = 0;
  if (ok) ok = or_rp_sweep(&rp, 1, &n_valid) == 0;
  if (ok) {
    if (keep_singles) {
      ok = or_rp_run(&rp, or_rp_screen_singles) == 0;
    } else {
      ok = or_rp_sweep(&rp, 2, NULL) == 0;
    }
  }
  if (ok) {
    res->st.n_valid = n_valid;
    uint64_t ne = 0;
    for (uint64_t q = 0; q < Q; ++q) {
      const or_range_stats* s = &rp.rst[q];
      res->st.n_distinct += s->n_distinct;
      res->st.entries += s->entries;
      res->st.sum_counts += s->sum_counts;
      res->st.fp_singletons += s->fp;
      res->st.n_pass += keep_singles ? s->sum_ge2 + s->fp : s->n_pass;
      if (!cb) ne += s->entries;  /* with a callback the table went out range by range */
    }
    for (uint64_t w = 0; w < m_words; ++w) {
      res->st.b1_pop += (uint64_t)__builtin_popcountll(rp.b1[w]);
      res->st.b2_pop += (uint64_t)__builtin_popcountll(rp.b2[w]);
    }
    res->keys = (uint64_t*)malloc((ne ? ne : 1) * sizeof(uint64_t));
    res->counts = (uint32_t*)malloc((ne ? ne : 1) * nc * sizeof(uint32_t));
    ok = res->keys && res->counts;
    if (ok) {
      uint64_t e = 0;
      for (uint64_t q = 0; q < Q; ++q) {
        if (rp.tkeys[q].n) {
          memcpy(res->keys + e, rp.tkeys[q].v, rp.tkeys[q].n * sizeof(uint64_t));
          memcpy(res->counts + e * nc, rp.tcounts[q].v, rp.tkeys[q].n * nc * sizeof(uint32_t));
        }
        e += rp.tkeys[q].n;
      }
      res->n_entries = ne;
    }
  }
  if (rp.bucket)
    for (uint64_t i = 0; i < (uint64_t)T * T; ++i) or_vfree64(&rp.bucket[i]);
  for (uint64_t q = 0; q < Q && rp.tkeys; ++q) or_vfree64(&rp.tkeys[q]);
  for (uint64_t q = 0; q < Q && rp.tcounts; ++q) or_vfree32(&rp.tcounts[q]);
  for (uint64_t q = 0; q < Q && rp.singles; ++q) or_vfree64(&rp.singles[q]);
  free(rp.bucket);
  free(rp.tkeys);
  free(rp.tcounts);
  free(rp.singles);
  free(rp.rst);
  free(rp.nvalid);
  free(rp.fail);
  if (!ok) {
    free(rp.b1);
    free(rp.b2);
    or_free(res);
    return NULL;
  }
  if (or_give_bloom(res, rp.b1, rp.b2, m_words, want_bloom)) {
    or_free(res);
    return NULL;
  }
  return res;
}
