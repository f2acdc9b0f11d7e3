// kc_kernels.hip - gfx950 kernels of the k-mer counter.
//
// Pass 1 (kc_insert_reads): pack ASCII into a 2-bit stream, cut every valid
// window into its canonical 2k-bit key, and shuffle keys by hash partition in
// two counting-sort levels (histogram, exclusive prefix sum, broker scatter;
// the paper's GPU shuffle, Sec. III-B).  Pass 2 (kc_finalize): one workgroup
// per Bloom block builds that block's two Bloom levels in LDS from every
// occurrence in the block (Prune, Sec. III), screens every occurrence against
// level 2 and counts passing keys exactly in an LDS open-addressing table per
// partition (Count, Sec. III), then writes the table to HBM with keys below
// min_count zeroed (Unify, Sec. III).
#include "kc_internal.h"

namespace kc {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Reverse complement of the 32 bases of a packed word (first base in the top
// two bits): complement every 2-bit code (c -> 3-c = ~c) and reverse their order.
__device__ __forceinline__ uint64_t rc_word(uint64_t v) {
  v = ~v;
  v = ((v >> 2) & 0x3333333333333333ull) | ((v & 0x3333333333333333ull) << 2);
  v = ((v >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((v & 0x0F0F0F0F0F0F0F0Full) << 4);
  return __builtin_bswap64(v);
}

__device__ __forceinline__ uint64_t top_bits(uint64_t g, uint32_t n) {
  return n ? (g >> (64 - n)) : 0;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ uint32_t wave_id() { return threadIdx.x >> 6; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive scan over n <= 4 * kThreads LDS counters with all kThreads
// threads: out[i] = sum(in[0..i)), out[n] = total.  scratch: kWaves words.
// Must be reached by every thread of the block; ends with a barrier.
__device__ void block_exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t n,
                                     uint32_t* scratch) {
  const uint32_t t = threadIdx.x;
  const uint32_t per = (n + kThreads - 1) / kThreads;
  uint32_t v[4] = {0, 0, 0, 0};
  uint32_t sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t i = t * per + q;
    if (q < (int)per && i < n) v[q] = in[i];
    sum += v[q];
  }
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(inc, d, 64);
    if ((int)lane_id() >= d) inc += o;
  }
  if (lane_id() == 63) scratch[wave_id()] = inc;
  __syncthreads();
  uint32_t wave_off = 0;
  for (uint32_t w = 0; w < wave_id(); ++w) wave_off += scratch[w];
  uint32_t run = wave_off + inc - sum;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t i = t * per + q;
    if (q < (int)per && i < n) out[i] = run;
    run += v[q];
  }
  if (t == kThreads - 1) out[n] = wave_off + inc;
  __syncthreads();
}

// ------------------------------------------------------------------ pack

__global__ void __launch_bounds__(256) k_pack(const uint8_t* __restrict__ bases, uint64_t total,
                                              uint64_t nwords, uint64_t* __restrict__ packed,
                                              uint64_t* __restrict__ flags, int aligned) {
  uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  uint64_t p0 = w * 32;
  uint8_t b[32];
  if (aligned && p0 + 32 <= total) {
    const uint4* src = reinterpret_cast<const uint4*>(bases + p0);
    uint4 lo = src[0], hi = src[1];
    const uint32_t words[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
    for (int i = 0; i < 32; ++i) b[i] = (uint8_t)(words[i >> 2] >> (8 * (i & 3)));
  } else {
#pragma unroll
    for (int i = 0; i < 32; ++i) b[i] = (p0 + i < total) ? bases[p0 + i] : (uint8_t)'N';
  }
  uint64_t code = 0;
  uint32_t inv = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    uint32_t c = b[i];
    bool ok = (c == 'A') | (c == 'C') | (c == 'G') | (c == 'T');
    uint32_t cd = ((c >> 1) ^ (c >> 2)) & 3u;  // A->0 C->1 G->2 T->3
    code = (code << 2) | (ok ? cd : 0u);
    inv |= (ok ? 0u : 1u) << i;
  }
  packed[w] = code;
  flags[w] = inv;  // read-start bits (high half) are or-ed in by k_rstart
}

// One thread per offset entry: marks the first base of every non-empty read
// and checks the offsets' contract.
__global__ void __launch_bounds__(256) k_rstart(const uint64_t* __restrict__ offsets,
                                                uint64_t n_reads, uint64_t total,
                                                uint64_t* __restrict__ flags,
                                                uint32_t* __restrict__ err) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_reads) return;
  uint64_t o = offsets[i];
  if (i == 0 && o != 0) atomicOr(err, (uint32_t)ERR_OFFSETS);
  if (i == n_reads) {
    if (o != total) atomicOr(err, (uint32_t)ERR_OFFSETS);
    return;
  }
  uint64_t o1 = offsets[i + 1];
  if (o1 < o || o1 > total) {
    atomicOr(err, (uint32_t)ERR_OFFSETS);
    return;
  }
  if (o1 > o && o < total)
    atomicOr(reinterpret_cast<unsigned long long*>(&flags[o >> 5]),
             1ull << (32 + (o & 31)));
}

// ----------------------------------------------------- window extraction

struct WordCtx {
  uint64_t pp, pc, qp, qc;  // packed words w-1, w and their reverse complements
  uint64_t inv, rst;        // invalid / read-start bits of words w-1 (low) and w (high)
};

__device__ __forceinline__ WordCtx load_word(const uint64_t* __restrict__ packed,
                                             const uint64_t* __restrict__ flags, uint64_t w) {
  WordCtx c;
  c.pc = packed[w];
  uint64_t fc = flags[w];
  uint64_t fp = 0xFFFFFFFFull;  // positions before the stream are invalid
  c.pp = 0;
  if (w) {
    c.pp = packed[w - 1];
    fp = flags[w - 1];
  }
  c.qp = rc_word(c.pp);
  c.qc = rc_word(c.pc);
  c.inv = (fp & 0xFFFFFFFFull) | (fc << 32);
  c.rst = (fp >> 32) | (fc & 0xFFFFFFFF00000000ull);
  return c;
}

// Canonical key of the window ending at base j (0..31) of word w, or false if
// the window holds an invalid base or crosses the start of a read.  In the
// 64-base concatenation (w-1, w) the window covers indices [33+j-k, 32+j].
__device__ __forceinline__ bool window_key(const WordCtx& c, uint32_t k, int j, uint64_t* x) {
  const uint64_t ibits = (1ull << k) - 1;
  if ((c.inv >> (33 + j - (int)k)) & ibits) return false;
  if (k > 1 && ((c.rst >> (34 + j - (int)k)) & ((1ull << (k - 1)) - 1))) return false;
  const uint64_t kmask = (1ull << (2 * k)) - 1;
  const int s = 62 - 2 * j;
  uint64_t f = (s ? ((c.pc >> s) | (c.pp << (64 - s))) : c.pc) & kmask;
  const int s2 = 66 + 2 * j - 2 * (int)k;  // in [4, 126]
  uint64_t r = (s2 >= 64 ? (c.qc >> (s2 - 64)) : ((c.qp >> s2) | (c.qc << (64 - s2)))) & kmask;
  *x = f < r ? f : r;
  return true;
}

// --------------------------------------------------- first-level shuffle

__global__ void __launch_bounds__(kThreads) k_hist1(const uint64_t* __restrict__ packed,
                                                    const uint64_t* __restrict__ flags,
                                                    uint64_t nwords, uint32_t k, uint64_t s0,
                                                    uint32_t a1, uint32_t* __restrict__ hist,
                                                    uint64_t ntiles) {
  extern __shared__ uint32_t sh[];
  const uint32_t nb = 1u << a1;
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) sh[i] = 0;
  __syncthreads();
  const uint64_t w = (uint64_t)blockIdx.x * kTileWords + (threadIdx.x >> 1);
  if (w < nwords) {
    const WordCtx c = load_word(packed, flags, w);
    const int j0 = (threadIdx.x & 1) * 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      uint64_t x;
      if (window_key(c, k, j0 + jj, &x)) atomicAdd(&sh[mix64(x ^ s0) >> (64 - a1)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) hist[(uint64_t)i * ntiles + blockIdx.x] = sh[i];
}

// Exclusive scan u32 -> u64 in three phases over chunks of 8192 elements.
constexpr int kScanChunk = kThreads * 8;

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in,
                                                          uint64_t n,
                                                          uint64_t* __restrict__ parts) {
  __shared__ uint64_t red[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 8;
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (base + q < n) s += in[base + q];
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += red[w];
    parts[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kThreads) k_scan_parts(uint64_t* __restrict__ parts,
                                                         uint64_t nparts,
                                                         uint64_t* __restrict__ out_total) {
  __shared__ uint64_t red[kWaves];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint64_t b = 0; b < nparts; b += kThreads) {
    uint64_t i = b + threadIdx.x;
    uint64_t v = i < nparts ? parts[i] : 0;
    uint64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint64_t o = __shfl_up(inc, d, 64);
      if ((int)lane_id() >= d) inc += o;
    }
    if (lane_id() == 63) red[wave_id()] = inc;
    __syncthreads();
    uint64_t off = carry;
    for (uint32_t w = 0; w < wave_id(); ++w) off += red[w];
    if (i < nparts) parts[i] = off + inc - v;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = off + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_total = carry;
}

__global__ void __launch_bounds__(kThreads) k_scan_down(const uint32_t* __restrict__ in,
                                                        uint64_t n,
                                                        const uint64_t* __restrict__ parts,
                                                        uint64_t* __restrict__ out) {
  __shared__ uint64_t red[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 8;
  uint32_t v[8];
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    s += v[q];
  }
  uint64_t inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t o = __shfl_up(inc, d, 64);
    if ((int)lane_id() >= d) inc += o;
  }
  if (lane_id() == 63) red[wave_id()] = inc;
  __syncthreads();
  uint64_t run = parts[blockIdx.x];
  for (uint32_t w = 0; w < wave_id(); ++w) run += red[w];
  run += inc - s;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
}

__global__ void k_bucket_off(const uint64_t* __restrict__ off1, uint64_t ntiles, uint32_t nb1,
                             uint64_t* __restrict__ bucket_off) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= nb1) bucket_off[c] = off1[(uint64_t)c * ntiles];
}

// Re-extracts the tile's keys, sorts them by first-level bucket in LDS and
// writes each bucket's run to its place (bucket-major, tiles in order).
__global__ void __launch_bounds__(kThreads) k_scatter1(const uint64_t* __restrict__ packed,
                                                       const uint64_t* __restrict__ flags,
                                                       uint64_t nwords, uint32_t k, uint64_t s0,
                                                       uint32_t a1,
                                                       const uint64_t* __restrict__ off1,
                                                       uint64_t ntiles, uint64_t tag,
                                                       uint64_t* __restrict__ out) {
  extern __shared__ uint64_t lds64[];
  const uint32_t nb = 1u << a1;
  uint64_t* stage = lds64;                         // kTilePos keys
  uint64_t* dst = stage + kTilePos;                // nb global bases (minus local start)
  uint32_t* cnt = reinterpret_cast<uint32_t*>(dst + nb);
  uint32_t* start = cnt + nb;                      // nb + 1
  uint32_t* scratch = start + nb + 1;              // kWaves
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) cnt[i] = 0;
  __syncthreads();
  const uint64_t w = (uint64_t)blockIdx.x * kTileWords + (threadIdx.x >> 1);
  uint64_t key[16];
  uint32_t meta[16];
  uint32_t valid = 0;
  if (w < nwords) {
    const WordCtx c = load_word(packed, flags, w);
    const int j0 = (threadIdx.x & 1) * 16;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      uint64_t x;
      if (window_key(c, k, j0 + jj, &x)) {
        uint32_t b = (uint32_t)(mix64(x ^ s0) >> (64 - a1));
        uint32_t rank = atomicAdd(&cnt[b], 1u);
        key[jj] = x | tag;
        meta[jj] = (b << 16) | rank;
        valid |= 1u << jj;
      }
    }
  }
  __syncthreads();
  block_exclusive_scan(cnt, start, nb, scratch);
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads)
    dst[i] = off1[(uint64_t)i * ntiles + blockIdx.x] - start[i];
#pragma unroll
  for (int jj = 0; jj < 16; ++jj)
    if (valid & (1u << jj)) stage[start[meta[jj] >> 16] + (meta[jj] & 0xFFFF)] = key[jj];
  __syncthreads();
  const uint32_t total = start[nb];
  for (uint32_t i = threadIdx.x; i < total; i += kThreads) {
    uint32_t lo = 0, hi = nb;  // largest b with start[b] <= i
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (start[mid] <= i) lo = mid; else hi = mid;
    }
    out[dst[lo] + i] = stage[i];
  }
}

// tile_first[c] = sum over c' < c of ceil(n_c' / kT2); tile_first[nb1] = total.
__global__ void __launch_bounds__(kThreads) k_tiles2(const uint64_t* __restrict__ bucket_off,
                                                     uint32_t nb1,
                                                     uint32_t* __restrict__ tile_first) {
  __shared__ uint32_t cnt[kThreads];
  __shared__ uint32_t scratch[kWaves];
  for (uint32_t c = threadIdx.x; c < nb1; c += kThreads) {
    uint64_t n = bucket_off[c + 1] - bucket_off[c];
    cnt[c] = (uint32_t)((n + kT2 - 1) / kT2);
  }
  __syncthreads();
  block_exclusive_scan(cnt, tile_first, nb1, scratch);
}

// In place: each workgroup loads one tile of a first-level bucket, sorts it by
// the next a2 bits of g in LDS and writes it back; meta2 records the offsets.
__global__ void __launch_bounds__(kThreads) k_scatter2(uint64_t* __restrict__ keys,
                                                       const uint64_t* __restrict__ bucket_off,
                                                       const uint32_t* __restrict__ tile_first,
                                                       uint32_t a1, uint32_t a2, uint64_t s0,
                                                       uint32_t* __restrict__ meta2) {
  extern __shared__ uint64_t lds64[];
  const uint32_t nb1 = 1u << a1, nb2 = 1u << a2;
  const uint32_t tt = blockIdx.x;
  if (tt >= tile_first[nb1]) return;
  uint32_t lo = 0, hi = nb1;  // largest c with tile_first[c] <= tt
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (tile_first[mid] <= tt) lo = mid; else hi = mid;
  }
  const uint32_t c = lo;
  const uint64_t r0 = bucket_off[c] + (uint64_t)(tt - tile_first[c]) * kT2;
  const uint64_t r1 = min(r0 + (uint64_t)kT2, bucket_off[c + 1]);
  const uint32_t n = (uint32_t)(r1 - r0);
  uint64_t* stage = lds64;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(stage + kT2);
  uint32_t* start = cnt + nb2;
  uint32_t* scratch = start + nb2 + 1;
  for (uint32_t i = threadIdx.x; i < nb2; i += kThreads) cnt[i] = 0;
  __syncthreads();
  uint64_t kv[kT2 / kThreads];
  uint32_t meta[kT2 / kThreads];
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    uint32_t i = threadIdx.x + r * kThreads;
    if (i < n) {
      kv[r] = keys[r0 + i];
      uint64_t g = mix64((kv[r] & kKeyMask) ^ s0);
      uint32_t sub = (uint32_t)((g >> (64 - a1 - a2)) & (nb2 - 1));
      meta[r] = (sub << 16) | atomicAdd(&cnt[sub], 1u);
    }
  }
  __syncthreads();
  block_exclusive_scan(cnt, start, nb2, scratch);
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    uint32_t i = threadIdx.x + r * kThreads;
    if (i < n) stage[start[meta[r] >> 16] + (meta[r] & 0xFFFF)] = kv[r];
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += kThreads) keys[r0 + i] = stage[i];
  for (uint32_t s = threadIdx.x; s <= nb2; s += kThreads)
    meta2[(uint64_t)tt * (nb2 + 1) + s] = start[s];
}

// ----------------------------------------- per-block Bloom + exact count

// Calls fn(key) for every stored occurrence of partition u, across segments.
// The whole block must call it (ranges are split between waves / threads).
template <typename F>
__device__ __forceinline__ void for_partition(const CountArgs& A, uint32_t u, F&& fn) {
  for (uint32_t s = 0; s < A.nsegs; ++s) {
    const SegDesc sd = A.segs[s];
    const uint32_t c = u >> sd.a2;
    if (sd.a2 == 0) {
      const uint64_t lo = sd.bucket_off[c], hi = sd.bucket_off[c + 1];
      for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) fn(sd.keys[i]);
    } else {
      const uint32_t nb2 = 1u << sd.a2;
      const uint32_t sub = u & (nb2 - 1);
      const uint32_t t0 = sd.tile_first[c], t1 = sd.tile_first[c + 1];
      const uint64_t bo = sd.bucket_off[c];
      for (uint32_t tt = t0 + wave_id(); tt < t1; tt += kWaves) {
        const uint64_t base = bo + (uint64_t)(tt - t0) * kT2;
        const uint32_t* m = sd.meta2 + (uint64_t)tt * (nb2 + 1) + sub;
        const uint32_t m0 = m[0], m1 = m[1];
        for (uint32_t i = m0 + lane_id(); i < m1; i += 64) fn(sd.keys[base + i]);
      }
    }
  }
}

// Distinct in-block bit positions of S(x): pos[i] valid where mask bit i set.
__device__ __forceinline__ uint32_t bloom_positions(const HashCfg& hc, uint64_t x,
                                                    uint32_t pos[8]) {
  uint32_t mask = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (i < (int)hc.h) {
      pos[i] = (uint32_t)(mix64(x ^ hc.salt[i + 1]) >> (64 - hc.bl));
      bool dup = false;
#pragma unroll
      for (int j = 0; j < i; ++j) dup |= ((mask >> j) & 1u) && pos[j] == pos[i];
      if (!dup) mask |= 1u << i;
    }
  }
  return mask;
}

__device__ __forceinline__ bool bloom_screen(const HashCfg& hc, const uint32_t* L2, uint64_t x) {
  bool pass = true;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (i < (int)hc.h) {
      uint32_t p = (uint32_t)(mix64(x ^ hc.salt[i + 1]) >> (64 - hc.bl));
      pass &= ((L2[p >> 5] >> (p & 31)) & 1u) != 0;
    }
  }
  return pass;
}

__device__ void overflow_add(const CountArgs& A, uint64_t x, uint32_t tag, uint64_t th) {
  const uint32_t nc = A.hc.nc;
  const uint64_t mask = (1ull << A.ovf_log2) - 1;
  uint64_t slot = th >> (64 - A.ovf_log2);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    uint64_t cur = __hip_atomic_load(&A.okeys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kEmpty) {
      cur = atomicCAS(reinterpret_cast<unsigned long long*>(&A.okeys[slot]),
                      (unsigned long long)kEmpty, (unsigned long long)x);
      if (cur == kEmpty) {
        uint32_t used = atomicAdd(A.ovf_used, 1u) + 1;
        if (used > A.ovf_limit) atomicOr(A.err, (uint32_t)ERR_OVF_LOAD);
        cur = x;
      }
    }
    if (cur == x) {
      atomicAdd(&A.ocounts[slot * nc + tag], 1u);
      return;
    }
    slot = (slot + 1) & mask;
  }
  atomicOr(A.err, (uint32_t)ERR_OVF_FULL);
}

__global__ void __launch_bounds__(kThreads) k_count(const CountArgs A) {
  extern __shared__ uint32_t lds[];
  const HashCfg& hc = A.hc;
  const uint32_t blk = blockIdx.x;
  const uint32_t nbw = A.nbw;
  uint32_t* L2 = lds;
  uint32_t* L1 = lds + A.l2w;
  uint64_t* tk = reinterpret_cast<uint64_t*>(lds + A.l2w);
  const uint32_t cap = 1u << hc.cap_log2;
  uint32_t* tc = reinterpret_cast<uint32_t*>(tk + cap);
  const uint32_t nc = hc.nc;
  const uint32_t u0 = blk << A.upb_log2, nu = 1u << A.upb_log2;

  uint64_t st[kNst];
#pragma unroll
  for (int i = 0; i < kNst; ++i) st[i] = 0;

  // Bloom levels of this block: every occurrence hits each distinct bit of
  // S(x) once; level 1 records a first hit, level 2 a second one.
  for (uint32_t i = threadIdx.x; i < A.l2w + nbw; i += kThreads) lds[i] = 0;
  __syncthreads();
  for (uint32_t uu = 0; uu < nu; ++uu) {
    for_partition(A, u0 + uu, [&](uint64_t key) {
      uint32_t pos[8];
      const uint32_t m = bloom_positions(hc, key & kKeyMask, pos);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if ((m >> i) & 1u) {
          const uint32_t bit = 1u << (pos[i] & 31);
          if (atomicOr(&L1[pos[i] >> 5], bit) & bit) atomicOr(&L2[pos[i] >> 5], bit);
        }
      }
    });
  }
  __syncthreads();
  if (hc.bl >= 5) {
    for (uint32_t i = threadIdx.x; i < nbw; i += kThreads) {
      const uint32_t a = L1[i], b = L2[i];
      A.b1[(uint64_t)blk * nbw + i] = a;
      A.b2[(uint64_t)blk * nbw + i] = b;
      st[ST_B1POP] += __popc(a);
      st[ST_B2POP] += __popc(b);
    }
  } else if (threadIdx.x == 0) {
    const uint64_t bit0 = (uint64_t)blk << hc.bl;
    const uint32_t msk = (1u << (1u << hc.bl)) - 1u;
    const uint32_t a = L1[0] & msk, b = L2[0] & msk;
    atomicOr(&A.b1[bit0 >> 5], a << (bit0 & 31));
    atomicOr(&A.b2[bit0 >> 5], b << (bit0 & 31));
    st[ST_B1POP] += __popc(a);
    st[ST_B2POP] += __popc(b);
  }
  __syncthreads();  // level 1 is dead from here: its LDS holds the count table

  for (uint32_t uu = 0; uu < nu; ++uu) {
    const uint32_t u = u0 + uu;
    for (uint32_t i = threadIdx.x; i < cap; i += kThreads) tk[i] = kEmpty;
    for (uint32_t i = threadIdx.x; i < cap * nc; i += kThreads) tc[i] = 0;
    __syncthreads();
    for_partition(A, u, [&](uint64_t key) {
      const uint64_t x = key & kKeyMask;
      const uint32_t tag = (uint32_t)(key >> 62);
      const uint64_t th = (x ^ hc.salt[0]) * kTableMul;
      uint32_t slot = (uint32_t)(th >> (64 - hc.cap_log2));
      int screened = 0;  // 0 unknown, 1 passes, -1 fails
      for (uint32_t probe = 0; probe < A.probe_limit; ++probe) {
        uint64_t cur = __hip_atomic_load(&tk[slot], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == kEmpty) {
          if (!screened) screened = bloom_screen(hc, L2, x) ? 1 : -1;
          if (screened < 0) return;  // dropped by the level-2 screen
          cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tk[slot]),
                          (unsigned long long)kEmpty, (unsigned long long)x);
          if (cur == kEmpty) cur = x;
        }
        if (cur == x) {
          atomicAdd(&tc[slot * nc + tag], 1u);
          return;
        }
        slot = (slot + 1) & (cap - 1);
      }
      if (!screened) screened = bloom_screen(hc, L2, x) ? 1 : -1;
      if (screened > 0) {
        st[ST_OVF] += 1;
        overflow_add(A, x, tag, mix64(th));  // re-mixed: the LDS slot used th's top bits
      }
    });
    __syncthreads();
    const uint64_t base = (uint64_t)u << hc.cap_log2;
    for (uint32_t i = threadIdx.x; i < cap; i += kThreads) {
      const uint64_t key = tk[i];
      uint32_t c0 = tc[i * nc], c1 = nc > 1 ? tc[i * nc + 1] : 0;
      if (key != kEmpty) {
        const uint64_t tot = (uint64_t)c0 + c1;
        st[ST_PASSED] += 1;
        st[ST_NPASS] += tot;
        st[ST_FP] += (tot == 1);
        if (tot >= hc.min_count) {
          st[ST_ENTRIES] += 1;
          st[ST_SUM] += tot;
        } else {
          c0 = c1 = 0;
        }
      }
      A.tkeys[base + i] = key;
      A.tcounts[(base + i) * nc] = c0;
      if (nc > 1) A.tcounts[(base + i) * nc + 1] = c1;
    }
    __syncthreads();
  }

  // block statistics: wave sums, then one row per block (LDS table is free)
  uint64_t* red = reinterpret_cast<uint64_t*>(lds + A.l2w);
#pragma unroll
  for (int i = 0; i < kNst; ++i) {
    const uint64_t v = wave_sum(st[i]);
    if (lane_id() == 0) red[wave_id() * kNst + i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNst) {
    uint64_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += red[w * kNst + threadIdx.x];
    A.pstats[(uint64_t)blk * kNst + threadIdx.x] = s;
  }
}

// Unify for the overflow table: statistics and the min_count threshold.
__global__ void __launch_bounds__(256) k_ovf_emit(const CountArgs A, uint64_t* pstats) {
  __shared__ uint64_t red[4 * kNst];
  const uint32_t nc = A.hc.nc;
  const uint64_t n = 1ull << A.ovf_log2;
  uint64_t st[kNst] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (A.okeys[i] == kEmpty) continue;
    uint32_t c0 = A.ocounts[i * nc], c1 = nc > 1 ? A.ocounts[i * nc + 1] : 0;
    const uint64_t tot = (uint64_t)c0 + c1;
    st[ST_PASSED] += 1;
    st[ST_NPASS] += tot;
    st[ST_FP] += (tot == 1);
    if (tot >= A.hc.min_count) {
      st[ST_ENTRIES] += 1;
      st[ST_SUM] += tot;
    } else {
      A.ocounts[i * nc] = 0;
      if (nc > 1) A.ocounts[i * nc + 1] = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < kNst; ++i) {
    const uint64_t v = wave_sum(st[i]);
    if (lane_id() == 0) red[wave_id() * kNst + i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNst) {
    uint64_t s = 0;
    for (int w = 0; w < 4; ++w) s += red[w * kNst + threadIdx.x];
    pstats[(uint64_t)blockIdx.x * kNst + threadIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kThreads) k_reduce(const uint64_t* __restrict__ rows,
                                                     uint64_t nrows, uint64_t* __restrict__ out) {
  __shared__ uint64_t red[kWaves * kNst];
  uint64_t st[kNst] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (uint64_t r = threadIdx.x; r < nrows; r += kThreads)
#pragma unroll
    for (int i = 0; i < kNst; ++i) st[i] += rows[r * kNst + i];
#pragma unroll
  for (int i = 0; i < kNst; ++i) {
    const uint64_t v = wave_sum(st[i]);
    if (lane_id() == 0) red[wave_id() * kNst + i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNst) {
    uint64_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += red[w * kNst + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ----------------------------------------------------------------- query

__device__ __forceinline__ bool probe_table(const uint64_t* keys, uint64_t base, uint32_t log2n,
                                            uint64_t x, uint64_t th, uint64_t* at) {
  const uint64_t mask = (1ull << log2n) - 1;
  uint64_t slot = th >> (64 - log2n);
  for (uint64_t p = 0; p <= mask; ++p) {
    const uint64_t cur = keys[base + slot];
    if (cur == x) {
      *at = base + slot;
      return true;
    }
    if (cur == kEmpty) return false;
    slot = (slot + 1) & mask;
  }
  return false;
}

__global__ void __launch_bounds__(256) k_query(const QueryArgs A, const uint64_t* __restrict__ kmers,
                                               uint64_t n, uint32_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const HashCfg& hc = A.hc;
  const uint32_t nc = hc.nc;
  const uint64_t q = kmers[i];
  uint32_t c0 = 0, c1 = 0;
  if (q >> (2 * hc.k)) {
    atomicOr(A.err, (uint32_t)ERR_QUERY_RANGE);
  } else {
    const uint64_t r = rc_word(q) >> (64 - 2 * hc.k);
    const uint64_t x = q < r ? q : r;
    const uint64_t u = top_bits(mix64(x ^ hc.salt[0]), hc.p_log2);
    const uint64_t th = (x ^ hc.salt[0]) * kTableMul;
    if (!A.resident[u]) {
      const uint32_t at = atomicAdd(A.host_count, 1u);
      A.host_rows[at] = (uint32_t)i;
    } else {
      uint64_t at;
      if (probe_table(A.tkeys, u << hc.cap_log2, hc.cap_log2, x, th, &at)) {
        c0 = A.tcounts[at * nc];
        if (nc > 1) c1 = A.tcounts[at * nc + 1];
      } else if (*A.ovf_used && probe_table(A.okeys, 0, A.ovf_log2, x, mix64(th), &at)) {
        c0 = A.ocounts[at * nc];
        if (nc > 1) c1 = A.ocounts[at * nc + 1];
      }
    }
  }
  out[i * nc] = c0;
  if (nc > 1) out[i * nc + 1] = c1;
}

// Entries with a nonzero count, wave-aggregated append (no particular order).
__global__ void __launch_bounds__(256) k_export(const uint64_t* __restrict__ tkeys,
                                                const uint32_t* __restrict__ tcounts,
                                                uint64_t nslots,
                                                const uint32_t* __restrict__ resident,
                                                uint32_t cap_log2, uint32_t nc,
                                                uint64_t* __restrict__ out_keys,
                                                uint32_t* __restrict__ out_counts,
                                                uint64_t out_cap,
                                                uint64_t* __restrict__ cursor) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  uint64_t key = 0;
  uint32_t c0 = 0, c1 = 0;
  if (i < nslots && (resident == nullptr || resident[i >> cap_log2])) {
    key = tkeys[i];
    c0 = tcounts[i * nc];
    c1 = nc > 1 ? tcounts[i * nc + 1] : 0;
    take = key != kEmpty && (c0 | c1) != 0;
  }
  const uint64_t bal = __ballot(take);
  if (!bal) return;
  uint64_t base = 0;
  if (lane_id() == (uint32_t)(__ffsll((unsigned long long)bal) - 1))
    base = atomicAdd(reinterpret_cast<unsigned long long*>(cursor),
                     (unsigned long long)__popcll(bal));
  base = __shfl(base, __ffsll((unsigned long long)bal) - 1, 64);
  if (take) {
    const uint64_t at = base + __popcll(bal & ((1ull << lane_id()) - 1));
    if (at >= out_cap) return;  // the cursor still counts it: the host sees the mismatch
    out_keys[at] = key;
    out_counts[at * nc] = c0;
    if (nc > 1) out_counts[at * nc + 1] = c1;
  }
}

// Partition of every stored key, derived from its storage position.
__global__ void __launch_bounds__(256) k_debug_part(const SegDesc sd, uint64_t n,
                                                    uint32_t* __restrict__ part) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t nb1 = 1u << sd.a1;
  uint32_t lo = 0, hi = nb1;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (sd.bucket_off[mid] <= i) lo = mid; else hi = mid;
  }
  const uint32_t c = lo;
  uint32_t sub = 0;
  if (sd.a2) {
    const uint32_t nb2 = 1u << sd.a2;
    const uint64_t rel = i - sd.bucket_off[c];
    const uint32_t tt = sd.tile_first[c] + (uint32_t)(rel / kT2);
    const uint32_t o = (uint32_t)(rel % kT2);
    const uint32_t* m = sd.meta2 + (uint64_t)tt * (nb2 + 1);
    uint32_t l2 = 0, h2 = nb2;
    while (h2 - l2 > 1) {
      uint32_t mid = (l2 + h2) >> 1;
      if (m[mid] <= o) l2 = mid; else h2 = mid;
    }
    sub = l2;
  }
  part[i] = (c << sd.a2) | sub;
}

// Compacts one partition table (entries with a nonzero count) in slot order.
__global__ void __launch_bounds__(256) k_gather_part(const uint64_t* __restrict__ tkeys,
                                                     const uint32_t* __restrict__ tcounts,
                                                     uint64_t base, uint64_t cap, uint32_t nc,
                                                     uint64_t* __restrict__ out_keys,
                                                     uint32_t* __restrict__ out_counts,
                                                     uint64_t* __restrict__ cursor) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  uint64_t key = 0;
  uint32_t c0 = 0, c1 = 0;
  if (i < cap) {
    key = tkeys[base + i];
    c0 = tcounts[(base + i) * nc];
    c1 = nc > 1 ? tcounts[(base + i) * nc + 1] : 0;
    take = key != kEmpty && (c0 | c1) != 0;
  }
  const uint64_t bal = __ballot(take);
  if (!bal) return;
  uint64_t b = 0;
  if (lane_id() == (uint32_t)(__ffsll((unsigned long long)bal) - 1))
    b = atomicAdd(reinterpret_cast<unsigned long long*>(cursor), (unsigned long long)__popcll(bal));
  b = __shfl(b, __ffsll((unsigned long long)bal) - 1, 64);
  if (take) {
    const uint64_t at = b + __popcll(bal & ((1ull << lane_id()) - 1));
    out_keys[at] = key;
    out_counts[at * nc] = c0;
    if (nc > 1) out_counts[at * nc + 1] = c1;
  }
}

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_pack(const uint8_t* bases, uint64_t total, uint64_t nwords, uint64_t* packed,
                       uint64_t* flags, hipStream_t s) {
  if (!nwords) return hipSuccess;
  const int aligned = ((uintptr_t)bases & 15) == 0;
  hipLaunchKernelGGL(k_pack, dim3(div_up(nwords, 256)), dim3(256), 0, s, bases, total, nwords,
                     packed, flags, aligned);
  return hipGetLastError();
}

hipError_t launch_rstart(const uint64_t* offsets, uint64_t n_reads, uint64_t total,
                         uint64_t* flags, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_rstart, dim3(div_up(n_reads + 1, 256)), dim3(256), 0, s, offsets, n_reads,
                     total, flags, err);
  return hipGetLastError();
}

hipError_t launch_hist1(const uint64_t* packed, const uint64_t* flags, uint64_t nwords,
                        uint32_t k, uint64_t s0, uint32_t a1, uint32_t* hist, uint64_t ntiles,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_hist1, dim3((uint32_t)ntiles), dim3(kThreads), (1u << a1) * 4, s, packed,
                     flags, nwords, k, s0, a1, hist, ntiles);
  return hipGetLastError();
}

size_t scan_parts(uint64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_scan(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* parts,
                       hipStream_t s) {
  const uint64_t np = (n + kScanChunk - 1) / kScanChunk;
  if (np) {
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)np), dim3(kThreads), 0, s, in, n, parts);
  }
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kThreads), 0, s, parts, np, out + n);
  if (np) {
    hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)np), dim3(kThreads), 0, s, in, n, parts, out);
  }
  return hipGetLastError();
}

hipError_t launch_bucket_off(const uint64_t* off1, uint64_t ntiles, uint32_t nb1,
                             uint64_t* bucket_off, hipStream_t s) {
  hipLaunchKernelGGL(k_bucket_off, dim3(div_up(nb1 + 1, 256)), dim3(256), 0, s, off1, ntiles, nb1,
                     bucket_off);
  return hipGetLastError();
}

static size_t scatter1_lds(uint32_t a1) {
  const uint32_t nb = 1u << a1;
  return (size_t)kTilePos * 8 + (size_t)nb * 8 + (size_t)nb * 4 + (size_t)(nb + 1) * 4 + kWaves * 4;
}

static size_t scatter2_lds(uint32_t a2) {
  const uint32_t nb = 1u << a2;
  return (size_t)kT2 * 8 + (size_t)nb * 4 + (size_t)(nb + 1) * 4 + kWaves * 4;
}

hipError_t launch_scatter1(const uint64_t* packed, const uint64_t* flags, uint64_t nwords,
                           uint32_t k, uint64_t s0, uint32_t a1, const uint64_t* off1,
                           uint64_t ntiles, uint64_t tag, uint64_t* out, hipStream_t s) {
  const size_t lds = scatter1_lds(a1);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_scatter1),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter1, dim3((uint32_t)ntiles), dim3(kThreads), lds, s, packed, flags,
                     nwords, k, s0, a1, off1, ntiles, tag, out);
  return hipGetLastError();
}

hipError_t launch_tiles2(const uint64_t* bucket_off, uint32_t nb1, uint32_t* tile_first,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_tiles2, dim3(1), dim3(kThreads), 0, s, bucket_off, nb1, tile_first);
  return hipGetLastError();
}

hipError_t launch_scatter2(uint64_t* keys, const uint64_t* bucket_off, const uint32_t* tile_first,
                           uint32_t a1, uint32_t a2, uint64_t s0, uint32_t* meta2, uint64_t grid,
                           hipStream_t s) {
  const size_t lds = scatter2_lds(a2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_scatter2),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter2, dim3((uint32_t)grid), dim3(kThreads), lds, s, keys, bucket_off,
                     tile_first, a1, a2, s0, meta2);
  return hipGetLastError();
}

hipError_t launch_count(const CountArgs& a, uint32_t blocks, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_count),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_count, dim3(blocks), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_ovf_emit(const CountArgs& a, uint64_t* pstats_ovf, uint32_t blocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_ovf_emit, dim3(blocks), dim3(256), 0, s, a, pstats_ovf);
  return hipGetLastError();
}

hipError_t launch_reduce(const uint64_t* rows, uint64_t nrows, uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, rows, nrows, out);
  return hipGetLastError();
}

hipError_t launch_query(const QueryArgs& a, const uint64_t* kmers, uint64_t n, uint32_t* out,
                        hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_query, dim3(div_up(n, 256)), dim3(256), 0, s, a, kmers, n, out);
  return hipGetLastError();
}

hipError_t launch_export(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                         const uint32_t* resident, uint32_t cap_log2, uint32_t nc,
                         uint64_t* out_keys, uint32_t* out_counts, uint64_t out_cap,
                         uint64_t* cursor, hipStream_t s) {
  if (!nslots) return hipSuccess;
  hipLaunchKernelGGL(k_export, dim3(div_up(nslots, 256)), dim3(256), 0, s, tkeys, tcounts, nslots,
                     resident, cap_log2, nc, out_keys, out_counts, out_cap, cursor);
  return hipGetLastError();
}

hipError_t launch_debug_part(const SegDesc& sd, uint64_t n, uint32_t* part, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_debug_part, dim3(div_up(n, 256)), dim3(256), 0, s, sd, n, part);
  return hipGetLastError();
}

hipError_t launch_gather_part(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t base,
                              uint64_t cap, uint32_t nc, uint64_t* out_keys, uint32_t* out_counts,
                              uint64_t* cursor, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_part, dim3(div_up(cap, 256)), dim3(256), 0, s, tkeys, tcounts, base,
                     cap, nc, out_keys, out_counts, cursor);
  return hipGetLastError();
}

}  // namespace kc
