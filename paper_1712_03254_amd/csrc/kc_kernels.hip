// kc_kernels.hip - gfx950 kernels of the k-mer counter.
//
// Pass 1 (kc_insert_reads): pack ASCII into a 2-bit stream, cut every valid
// window into its canonical 2k-bit key, and shuffle keys by hash partition in
// two counting-sort levels (histogram, exclusive prefix sum, broker scatter;
// the paper's GPU shuffle, Sec. III-B).  Pass 2 (kc_finalize): one workgroup
// per Bloom block builds that block's two Bloom levels in LDS from every
// occurrence in the block (Prune, Sec. III); then one workgroup per partition
// counts the partition's keys in an LDS open-addressing table, screening each
// new key against level 2 (Count, Sec. III), and writes the table to HBM with
// keys below min_count zeroed (Unify, Sec. III).  After finalize: queries,
// the Filter unit's lookup of every window of a read batch (Sec. II-B), the
// stem layout of the table (Sec. II-A, III-D) and the table export.  The
// batched form's pack and read-start kernels and the fill kernels that
// replace memsets in captured graphs are here too.
#include "kc_internal.h"

namespace kc {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The top 31 bits of mix64(z), in bits 31..1 (bit 0 is not part of them).
// mix64's last step, z ^ (z >> 31), leaves bits 63..33 as they are, and the
// high half of the second product needs three 32-bit multiplies: the
// shuffle levels use only the top log2(partitions) <= 21 bits of g.
__device__ __forceinline__ uint32_t mix64_top31(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  const uint64_t y = z ^ (z >> 27);
  const uint32_t ylo = (uint32_t)y, yhi = (uint32_t)(y >> 32);
  constexpr uint32_t clo = 0x133111EBu, chi = 0x94D049BBu;  // 0x94D049BB133111EB
  return ylo * chi + yhi * clo + __umulhi(ylo, clo);
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
// Wave index in the block, in a scalar register (the compiler cannot tell on
// its own that threadIdx.x >> 6 is the same in every lane of a wave).
__device__ __forceinline__ uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Address-space views of device pointers.  Pointers read out of memory (a
// segment descriptor) are generic to the compiler, which then emits flat
// loads; flat loads also count against the LDS wait counter, so an LDS wait
// would hold until every key load in flight had landed.  gview() restores
// global loads.  cview() marks data no kernel writes while this one runs;
// loads from it at wave-uniform addresses become scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gview(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cview(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// 64-bit value of the lane CTRL names (a DPP row shift or row broadcast),
// 0 where that lane is outside the row or the lane's row is not in ROWS.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, true);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, true);
  return ((uint64_t)hi << 32) | lo;
}

// Sum of a 64-bit value over the 64 lanes of a wave, returned to every lane:
// within each row of 16 lanes, shifted adds by 1, 2, 4 and 8 leave the row's
// sum in its lane 15; two row broadcasts then add row 0 into row 1 and rows
// 0-1 into rows 2-3, so lane 63 holds the total (DPP moves, no LDS).
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
  v += dpp_u64<0x111, 0xF>(v);  // row_shr:1
  v += dpp_u64<0x112, 0xF>(v);  // row_shr:2
  v += dpp_u64<0x114, 0xF>(v);  // row_shr:4
  v += dpp_u64<0x118, 0xF>(v);  // row_shr:8
  v += dpp_u64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_u64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}

// 64-bit inclusive prefix sum across the 64 lanes of a wave (the DPP steps
// of wave_sum, whose partial sums are the prefix sums).
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  v += dpp_u64<0x111, 0xF>(v);
  v += dpp_u64<0x112, 0xF>(v);
  v += dpp_u64<0x114, 0xF>(v);
  v += dpp_u64<0x118, 0xF>(v);
  v += dpp_u64<0x142, 0xA>(v);
  v += dpp_u64<0x143, 0xC>(v);
  return v;
}

// Inclusive prefix sum across the 64 lanes of a wave: the same DPP steps as
// wave_sum, whose partial sums are the prefix sums (each row's by the shifts,
// then the rows before it by the two broadcasts).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += dpp_u32<0x111, 0xF>(v);  // row_shr:1
  v += dpp_u32<0x112, 0xF>(v);  // row_shr:2
  v += dpp_u32<0x114, 0xF>(v);  // row_shr:4
  v += dpp_u32<0x118, 0xF>(v);  // row_shr:8
  v += dpp_u32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_u32<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
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
  // waves whose counters all lie past n hold zeros and skip the wave scan
  if ((t - lane_id()) * per < n) inc = wave_incl_scan(inc);
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

// Codes and validity of the four bases of a 32-bit word (base i in byte i),
// four at a time: each byte's code is bits 1-2 of its ASCII value (A0 C1 G2
// T3), and the byte is a base exactly when it equals "ACGT"[code] (a byte
// permute of the four letters); a nonzero byte of the difference is found
// without carries between bytes.  Returns the 8-bit code of the four bases
// (first base in the top two bits, invalid bases coded 0) in bits 0-7 and
// their invalid bits (base i at bit i) in bits 8-11.
__device__ __forceinline__ uint32_t pack4(uint32_t v) {
  uint32_t c = ((v >> 1) ^ (v >> 2)) & 0x03030303u;
  const uint32_t want = __builtin_amdgcn_perm(0u, 0x54474341u, c);  // 'A' 'C' 'G' 'T'
  const uint32_t z = v ^ want;
  const uint32_t inv = (((((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u) >> 7);
  c &= ~(inv * 3u);
  // bytes 0..3 of c to bits 30, 28, 26, 24; of inv to bits 24..27 (no other
  // product term reaches bit 24)
  return ((c * 0x40100401u) >> 24) | ((((inv * 0x01020408u) >> 24) & 0xFu) << 8);
}

// Two threads per packed word: thread t takes bases [16 t, 16 t + 16) (one
// 16-byte load; a wave reads 1 KB contiguous), thread 2w the first half of
// word w and 2w + 1 the second; the pair exchange halves, then the even
// thread writes the packed word and the odd one the flag word.
__global__ void __launch_bounds__(256) k_pack(const uint8_t* __restrict__ bases, uint64_t total,
                                              uint64_t nwords, uint64_t* __restrict__ packed,
                                              uint64_t* __restrict__ flags, int aligned) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t w = t >> 1;
  const uint64_t p0 = t * 16;
  uint32_t code = 0, inv = 0;  // 16 bases: code (first base on top), invalid bits
  if (w < nwords) {
    uint32_t v[4];
    if (aligned && p0 + 16 <= total) {
      const uint4 q = *reinterpret_cast<const uint4*>(bases + p0);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint32_t x = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint64_t p = p0 + 4 * g + i;
          x |= (uint32_t)(p < total ? bases[p] : (uint8_t)'N') << (8 * i);
        }
        v[g] = x;
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint32_t r = pack4(v[g]);
      code |= (r & 0xFFu) << (24 - 8 * g);
      inv |= (r >> 8) << (4 * g);
    }
  }
  const uint32_t ocode = __shfl_xor(code, 1, 64), oinv = __shfl_xor(inv, 1, 64);
  if (w < nwords) {
    if ((t & 1) == 0)
      packed[w] = ((uint64_t)code << 32) | ocode;
    else
      flags[w] = inv << 16 | oinv;  // read-start bits (high half) are set by k_rstart
  }
}

// Read-start bits (the high half of each flag word; the pack kernels leave it
// zero), one thread per offset entry, without an atomic per read.  Reads tile
// the bases, so every word's first base lies in exactly one non-empty read,
// the word's leader, which writes the word's start bits with one 32-bit store:
// a word wholly inside the read can hold only the read's own start, and the
// last word the read leads also holds the starts of the reads after it that
// begin in that word, found by scanning up to kStartScan offset entries.  A
// start further than that from its word's leader (only runs of empty reads
// make one) is or-ed in atomically, and a leader whose scan was cut short ors
// its bits as well.  Offsets are chunk-relative; word0 is the chunk's first
// word in the flag array (chunks start on a word boundary).  The offsets'
// contract is checked on the way.
constexpr uint32_t kStartScan = 64;

__device__ __forceinline__ void put_starts(uint64_t* flags, uint64_t w, uint32_t bits, bool atomic) {
  uint32_t* hi = reinterpret_cast<uint32_t*>(flags + w) + 1;
  if (atomic)
    atomicOr(hi, bits);
  else
    *hi = bits;
}

__device__ __forceinline__ void read_start(const uint64_t* __restrict__ offsets, uint64_t r,
                                           uint64_t n_reads, uint64_t total, uint64_t word0,
                                           uint64_t* __restrict__ flags, uint32_t* __restrict__ err) {
  const uint64_t o = offsets[r];
  if (r == 0 && o != 0) atomicOr(err, (uint32_t)ERR_OFFSETS);
  if (r == n_reads) {
    if (o != total) atomicOr(err, (uint32_t)ERR_OFFSETS);
    return;
  }
  const uint64_t e = offsets[r + 1];
  if (e < o || e > total) {
    atomicOr(err, (uint32_t)ERR_OFFSETS);
    return;
  }
  if (e == o) return;  // empty read
  // this read's start, when its word's leader is out of scan range: the
  // leader is the last entry at or before the word's first base
  const uint64_t ws = o >> 5;
  if ((o & 31) != 0 && r >= kStartScan && offsets[r - kStartScan] > (ws << 5))
    put_starts(flags, word0 + ws, 1u << (o & 31), true);
  // words whose first base this read holds: wf .. wl
  const uint64_t wf = (o + 31) >> 5, wl = (e - 1) >> 5;
  if (wf > wl) return;
  if (wf < wl && (o & 31) == 0) put_starts(flags, word0 + wf, 1u, false);
  const uint64_t lo = wl << 5;
  uint32_t bits = o == lo ? 1u : 0u;
  bool cut = true;
  for (uint32_t d = 1; d <= kStartScan; ++d) {
    const uint64_t j = r + d;
    if (j >= n_reads) {
      cut = false;
      break;
    }
    const uint64_t v = offsets[j];
    if (v < lo || v >= lo + 32) {
      cut = false;
      break;
    }
    if (offsets[j + 1] > v) bits |= 1u << (v - lo);
  }
  if (bits) put_starts(flags, word0 + wl, bits, cut);
}

__global__ void __launch_bounds__(256) k_rstart(const uint64_t* __restrict__ offsets,
                                                uint64_t n_reads, uint64_t total,
                                                uint64_t* __restrict__ flags,
                                                uint32_t* __restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_reads) read_start(offsets, i, n_reads, total, 0, flags, err);
}

// Largest j < n with key(j) <= v, for a non-decreasing key (chunks with no
// words or reads share their successor's start and are skipped).
template <typename K>
__device__ __forceinline__ uint32_t chunk_of(const ChunkDesc* cd, uint32_t n, uint64_t v, K key) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key(cd[mid]) <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// k_pack over the chunks of a batch group: word w of the group stream is word
// w - word0 of its chunk (positions past the chunk's end are invalid).  As in
// k_pack, two threads per word, 16 bases each (one 16-byte load when aligned
// and inside the chunk), joined by a lane exchange.  A workgroup's 128 words
// lie in one chunk or a few neighbouring ones: one search finds the first
// word's chunk and each thread walks forward from it (a search per thread
// cost 2.3% of the batched graph); the loads go through the global address
// space (chunk pointers are device memory).
__global__ void __launch_bounds__(256) k_pack_batch(const ChunkDesc* __restrict__ cd,
                                                    uint32_t nchunks, uint64_t nwords,
                                                    uint64_t* __restrict__ packed,
                                                    uint64_t* __restrict__ flags) {
  __shared__ uint32_t j0s;
  for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x; b0 < 2 * nwords;
       b0 += (uint64_t)gridDim.x * blockDim.x) {
    // the block's 128 words: one search for the first word's chunk, then a
    // forward walk per thread
    if (threadIdx.x == 0)
      j0s = chunk_of(cd, nchunks, b0 >> 1, [](const ChunkDesc& d) { return d.word0; });
    __syncthreads();
    const uint64_t t = b0 + threadIdx.x;
    const uint64_t w = t >> 1;
    uint32_t j = j0s;
    while (j + 1 < nchunks && cd[j + 1].word0 <= w) ++j;
    if (t < 2 * nwords) {
      typedef uint32_t g32x4 __attribute__((ext_vector_type(4)));
      const __attribute__((address_space(1))) uint8_t* bases =
          (const __attribute__((address_space(1))) uint8_t*)cd[j].bases;
      const uint64_t total = cd[j].total;
      const uint64_t p0 = (w - cd[j].word0) * 32 + (t & 1) * 16;
      uint32_t v[4];
      if (p0 + 16 <= total && ((uintptr_t)(cd[j].bases + p0) & 15) == 0) {
        const g32x4 q = *reinterpret_cast<const __attribute__((address_space(1))) g32x4*>(bases + p0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          uint32_t x = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint64_t p = p0 + 4 * g + i;
            x |= (uint32_t)(p < total ? bases[p] : (uint8_t)'N') << (8 * i);
          }
          v[g] = x;
        }
      }
      uint32_t code = 0, inv = 0;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t r = pack4(v[g]);
        code |= (r & 0xFFu) << (24 - 8 * g);
        inv |= (r >> 8) << (4 * g);
      }
      const uint32_t ocode = __shfl_xor(code, 1, 64), oinv = __shfl_xor(inv, 1, 64);
      if ((t & 1) == 0)
        packed[w] = ((uint64_t)code << 32) | ocode;
      else
        flags[w] = oinv | (inv << 16);
    }
    __syncthreads();
  }
}

// k_rstart over the chunks of a batch group: slot i is read i - read0 of its
// chunk, or the chunk's end check when that equals the chunk's read count.
__global__ void __launch_bounds__(256) k_rstart_batch(const ChunkDesc* __restrict__ cd,
                                                      uint32_t nchunks, uint64_t nslots,
                                                      uint64_t* __restrict__ flags,
                                                      uint32_t* __restrict__ err) {
  __shared__ uint32_t j0s;
  for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x; b0 < nslots;
       b0 += (uint64_t)gridDim.x * blockDim.x) {
    // one search for the workgroup's first slot, then a forward walk (every
    // chunk holds at least its end-check slot, so read0 increases)
    if (threadIdx.x == 0)
      j0s = chunk_of(cd, nchunks, b0, [](const ChunkDesc& d) { return d.read0; });
    __syncthreads();
    const uint64_t i = b0 + threadIdx.x;
    uint32_t j = j0s;
    while (j + 1 < nchunks && cd[j + 1].read0 <= i) ++j;
    if (i < nslots)
      read_start(cd[j].offsets, i - cd[j].read0, cd[j].n_reads, cd[j].total, cd[j].word0, flags,
                 err);
    __syncthreads();
  }
}

// Fills and a one-word copy, for work that may be captured in a graph
// (where memset nodes are avoided).
__global__ void __launch_bounds__(256) k_fill64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void __launch_bounds__(256) k_fill32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_copy64(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// Words idx[i] of two arrays of nwords 64-bit words; an index past the end
// sets ERR_QUERY_RANGE and reads as 0.
__global__ void __launch_bounds__(256) k_gather2(const uint64_t* __restrict__ a,
                                                 const uint64_t* __restrict__ b,
                                                 const uint64_t* __restrict__ idx, uint64_t n,
                                                 uint64_t nwords, uint64_t* __restrict__ out_a,
                                                 uint64_t* __restrict__ out_b,
                                                 uint32_t* __restrict__ err) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t w = idx[i];
    const bool ok = w < nwords;
    if (!ok) atomicOr(err, (uint32_t)ERR_QUERY_RANGE);
    out_a[i] = ok ? a[w] : 0;
    out_b[i] = ok ? b[w] : 0;
  }
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

// OR of z << i over i < w (w < 32): every set bit spread over the w - 1
// indices above it.  w is the same on every lane, so the branches are scalar.
__device__ __forceinline__ uint64_t smear(uint64_t z, uint32_t w) {
  uint64_t acc = 0, cur = z;  // cur: OR of z << i over i < 2^b
  uint32_t sh = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (w & (1u << b)) {
      acc |= cur << sh;
      sh += 1u << b;
    }
    cur |= cur << (1u << b);
  }
  return acc;
}

// Bit j set when the window ending at base j of word w is one window_key
// accepts: the window [33+j-k, 32+j] of the (w-1, w) frame holds no invalid
// base, and no read starts in [34+j-k, 32+j].
__device__ __forceinline__ uint32_t window_mask(const WordCtx& c, uint32_t k) {
  const uint64_t bad = smear(c.inv, k) | smear(c.rst, k - 1);
  return ~(uint32_t)(bad >> 32);
}

// Canonical key of the window ending at base j of word w, whether or not the
// window is valid (window_mask says which are).  Both orientations are taken
// left-aligned, the window in the top 2k bits and the bases after it below:
// where the two codes differ their top bits decide the comparison, and where
// they are equal either choice gives the same key, so the smaller 64-bit
// value shifted down by 64 - 2k is min(enc(w), enc(revcomp(w))).
__device__ __forceinline__ uint64_t window_code(const WordCtx& c, uint32_t k, int j) {
  // forward: bases 33+j-k.. of the (w-1, w) frame at the top
  const int sh = 66 + 2 * j - 2 * (int)k;  // in [4, 126]
  const uint64_t f = sh >= 64 ? c.pc << (sh - 64) : (c.pp << sh) | (c.pc >> (64 - sh));
  // reverse complement: the (w, w-1) frame of reversed, complemented words
  // from the complement of base 32+j on
  const int sr = 62 - 2 * j;  // in [0, 62]
  const uint64_t r = (c.qc << sr) | (sr == 0 ? 0ull : c.qp >> (64 - sr));
  return (f < r ? f : r) >> (64 - 2 * k);
}

// --------------------------------------------------- first-level shuffle

// One pass per tile of kTilePos window positions: extract the canonical keys,
// counting-sort them by the top a1 bits of g in LDS, and write the sorted tile
// to its own region of the tile-major buffer (every store is contiguous).  The
// tile's bucket counts and bucket starts go out bucket-major: the counts for
// the prefix sum that places buckets, the starts for the second level's
// gather, which reads one bucket's starts over consecutive tiles (adjacent
// tiles' entries share cache lines, and their writes merge in L2).
__global__ void __launch_bounds__(kThreads) k_level1(const uint64_t* __restrict__ packed,
                                                     const uint64_t* __restrict__ flags,
                                                     uint64_t nwords, uint32_t k, uint64_t s0,
                                                     uint32_t a1, uint64_t tag,
                                                     uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ lstart,
                                                     uint64_t ntiles,
                                                     uint64_t* __restrict__ out) {
  extern __shared__ uint64_t lds64[];
  // XCD x takes tiles [x * per, (x + 1) * per): the histogram and run-start
  // columns of neighbouring tiles share cache lines, which then fill in one L2
  const uint64_t per = (ntiles + kXcds - 1) / kXcds;
  const uint64_t tile = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (tile >= ntiles) return;
  const uint32_t nb = 1u << a1;
  uint64_t* stage = lds64;                                  // kTilePos keys
  uint32_t* cnt = reinterpret_cast<uint32_t*>(stage + kTilePos);
  uint32_t* start = cnt + nb;                               // nb + 1
  uint32_t* scratch = start + nb + 1;                       // kWaves
  // Context of each of the tile's words, made once per word by the first
  // kTileWords threads (four waves take a word's windows): packed words w-1
  // and w, their reverse complements and the valid-window mask.  It sits in
  // the stage area, which the sorted keys overwrite only after the barrier
  // that ends the extraction.
  uint64_t* cx = stage;                                           // 4 x kTileWords
  uint32_t* cm = reinterpret_cast<uint32_t*>(stage + 4 * kTileWords);  // kTileWords
  static_assert(5 * kTileWords <= kTilePos, "word context fits the stage area");
  if (threadIdx.x < kTileWords) {
    const uint64_t wt = tile * kTileWords + threadIdx.x;
    if (wt < nwords) {
      const WordCtx c = load_word(packed, flags, wt);
      cx[threadIdx.x] = c.pp;
      cx[kTileWords + threadIdx.x] = c.pc;
      cx[2 * kTileWords + threadIdx.x] = c.qp;
      cx[3 * kTileWords + threadIdx.x] = c.qc;
      cm[threadIdx.x] = window_mask(c, k);
    }
  }
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) cnt[i] = 0;
  __syncthreads();
  // Lane l of wave v takes packed word (v mod kWordGroups) * 64 + l and in it
  // the kPP positions from kPP * (v / kWordGroups): the window offsets are the
  // same on every lane, so every shift in the extraction is by a scalar and
  // no branch on them diverges; a wave's word loads are contiguous.
  constexpr int kPP = kTilePos / kThreads;
  constexpr int kWordGroups = kTileWords / 64;
  static_assert(kPP * kThreads == kTilePos && kPP * (kThreads / 64 / kWordGroups) == 32 &&
                    kWordGroups * 64 == kTileWords,
                "level-1 tile shape");
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wl = (wv % kWordGroups) * 64 + (threadIdx.x & 63);
  const uint64_t w = tile * kTileWords + wl;
  uint64_t key[kPP];
  uint32_t meta[kPP];
  uint32_t valid = 0;
  if (w < nwords) {
    WordCtx c;
    c.pp = cx[wl];
    c.pc = cx[kTileWords + wl];
    c.qp = cx[2 * kTileWords + wl];
    c.qc = cx[3 * kTileWords + wl];
    const int j0 = (int)(wv / kWordGroups) * kPP;
    valid = (cm[wl] >> j0) & ((1u << kPP) - 1);
    // keys and hashes of all kPP windows, branch-free; every lane adds to
    // its bucket's count (1 for a valid window, 0 otherwise), so the kPP
    // atomics issue back to back and are waited for once
    uint32_t bk[kPP], rk[kPP];
#pragma unroll
    for (int jj = 0; jj < kPP; ++jj) {
      const uint64_t x = window_code(c, k, j0 + jj);
      bk[jj] = mix64_top31(x ^ s0) >> (32 - a1);
      key[jj] = x | tag;
    }
#pragma unroll
    for (int jj = 0; jj < kPP; ++jj) rk[jj] = atomicAdd(&cnt[bk[jj]], (valid >> jj) & 1u);
#pragma unroll
    for (int jj = 0; jj < kPP; ++jj) meta[jj] = (bk[jj] << 16) | rk[jj];
  }
  __syncthreads();
  block_exclusive_scan(cnt, start, nb, scratch);
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) hist[(uint64_t)i * ntiles + tile] = cnt[i];
  for (uint32_t i = threadIdx.x; i < nb; i += kThreads) lstart[(uint64_t)i * ntiles + tile] = start[i];
#pragma unroll
  for (int jj = 0; jj < kPP; ++jj)
    if (valid & (1u << jj)) stage[start[meta[jj] >> 16] + (meta[jj] & 0xFFFF)] = key[jj];
  __syncthreads();
  const uint32_t total = start[nb];
  uint64_t* dst = out + tile * kTilePos;
  for (uint32_t i = threadIdx.x; i < total; i += kThreads) dst[i] = stage[i];
}

// Exclusive scan u32 -> u64 in three phases over chunks of 8192 elements.
constexpr int kScanChunk = kThreads * 8;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// A thread's 8 consecutive counts (32-byte aligned: the arrays start on
// allocation boundaries): two 16-byte loads, or element loads at a ragged end.
__device__ __forceinline__ void load8(const uint32_t* __restrict__ in, uint64_t base, uint64_t n,
                                      uint32_t v[8]) {
  if (base + 8 <= n) {
    const u32x4 a = *reinterpret_cast<const u32x4*>(in + base);
    const u32x4 b = *reinterpret_cast<const u32x4*>(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = base + q < n ? in[base + q] : 0u;
  }
}

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in,
                                                          uint64_t n,
                                                          uint64_t* __restrict__ parts) {
  __shared__ uint64_t red[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 8;
  uint32_t v[8];
  load8(in, base, n, v);
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += v[q];
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
    const uint64_t inc = wave_incl_scan64(v);
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
  load8(in, base, n, v);
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += v[q];
  const uint64_t inc = wave_incl_scan64(s);
  if (lane_id() == 63) red[wave_id()] = inc;
  __syncthreads();
  uint64_t run = parts[blockIdx.x];
  for (uint32_t w = 0; w < wave_id(); ++w) run += red[w];
  run += inc - s;
  uint64_t o[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    o[q] = run;
    run += v[q];
  }
  if (base + 8 <= n) {  // 64-byte aligned: four 16-byte stores
#pragma unroll
    for (int h = 0; h < 4; ++h)
      *reinterpret_cast<u64x2*>(out + base + 2 * h) = u64x2{o[2 * h], o[2 * h + 1]};
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (base + q < n) out[base + q] = o[q];
  }
}

__global__ void k_bucket_off(const uint64_t* __restrict__ off1, uint64_t ntiles, uint32_t nb1,
                             uint64_t* __restrict__ bucket_off) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= nb1) bucket_off[c] = off1[(uint64_t)c * ntiles];
}

// tile_first[c] = sum over c' < c of ceil(n_c' / 2^t2_log2); tile_first[nb1] = total.
__global__ void __launch_bounds__(kThreads) k_tiles2(const uint64_t* __restrict__ bucket_off,
                                                     uint32_t nb1, uint32_t t2_log2,
                                                     uint32_t* __restrict__ tile_first) {
  __shared__ uint32_t cnt[kThreads];
  __shared__ uint32_t scratch[kWaves];
  for (uint32_t c = threadIdx.x; c < nb1; c += kThreads) {
    uint64_t n = bucket_off[c + 1] - bucket_off[c];
    cnt[c] = (uint32_t)((n + (1ull << t2_log2) - 1) >> t2_log2);
  }
  __syncthreads();
  block_exclusive_scan(cnt, tile_first, nb1, scratch);
}

// For every second-level tile tt, a descriptor for the workgroup of the
// second-level grid (grid8 workgroups) that takes it: tt, its first-level
// bucket c and the first-level tile whose run of c holds the tile's first key
// (largest t with off1[c][t] <= start), packed as tt | c << 20 | t << 30, so
// the workgroup starts from one load instead of searches.  ~0 marks a
// workgroup with no tile.
//
// Order: bucket c's tile j reads the runs of c in a stretch of first-level
// tiles; bucket c + 1's tile j reads the neighbouring runs of nearly the same
// stretch, and the two share a cache line at every run boundary.  The
// buckets are split into min(8, nb1) groups of consecutive buckets, group g
// goes to XCD g, and inside a group tiles are taken j-major (all buckets'
// tile 0, then all tile 1, ...), so the workgroups an XCD runs at once read
// adjacent runs through the same L2.  When a group holds more tiles than its
// XCD has workgroups (skewed buckets) the grid takes tiles in plain order.
__global__ void __launch_bounds__(256) k_tile_desc(const uint64_t* __restrict__ off1,
                                                   uint64_t ntiles1,
                                                   const uint64_t* __restrict__ bucket_off,
                                                   const uint32_t* __restrict__ tile_first,
                                                   uint32_t nb1, uint32_t grid8, uint32_t t2_log2,
                                                   uint64_t* __restrict__ order) {
  __shared__ uint32_t tf[(1u << kMaxA1) + 1];
  for (uint32_t i = threadIdx.x; i <= nb1; i += blockDim.x) tf[i] = tile_first[i];
  __syncthreads();
  const uint32_t tt = blockIdx.x * blockDim.x + threadIdx.x;
  if (tt >= tf[nb1]) return;
  uint32_t lo = 0, hi = nb1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tf[mid] <= tt) lo = mid; else hi = mid;
  }
  const uint32_t c = lo;
  const uint64_t want = bucket_off[c] + ((uint64_t)(tt - tf[c]) << t2_log2);
  const uint64_t* offc = off1 + (uint64_t)c * ntiles1;
  uint64_t a = 0, b = ntiles1;  // largest t in [0, ntiles1) with offc[t] <= want
  while (b - a > 1) {
    const uint64_t mid = (a + b) >> 1;
    if (offc[mid] <= want) a = mid; else b = mid;
  }
  const uint64_t desc = (uint64_t)tt | (uint64_t)c << 20 | a << 30;
  {
    const uint32_t ng = nb1 < kXcds ? nb1 : kXcds, gs = nb1 / ng, per = grid8 / kXcds;
    bool fits = true;
    for (uint32_t g = 0; g < ng; ++g) fits = fits && tf[(g + 1) * gs] - tf[g * gs] <= per;
    if (fits) {
      const uint32_t g = c / gs, j = tt - tf[c];
      uint32_t pos = 0;
      for (uint32_t d = g * gs; d < (g + 1) * gs; ++d) {
        const uint32_t nd = tf[d + 1] - tf[d];
        pos += nd < j ? nd : j;
        if (d < c && nd > j) ++pos;
      }
      order[pos * kXcds + g] = desc;
    } else {
      order[tt] = desc;
    }
  }
}

// Second level: each workgroup takes 2^t2_log2 (at most kT2) consecutive keys of one first-level
// bucket, gathered from that bucket's run in every first-level tile, sorts them
// by the next a2 bits of g in LDS and writes them contiguously into the
// bucket's region; meta2 records where each sub-bucket starts in the tile.
__global__ void __launch_bounds__(kThreads) k_level2(const uint64_t* __restrict__ keys1,
                                                     const uint64_t* __restrict__ off1,
                                                     const uint32_t* __restrict__ lstart,
                                                     uint64_t ntiles1,
                                                     const uint64_t* __restrict__ bucket_off,
                                                     const uint32_t* __restrict__ tile_first,
                                                     const uint64_t* __restrict__ order,
                                                     uint32_t a1, uint32_t a2, uint32_t t2_log2,
                                                     uint64_t s0, uint64_t* __restrict__ keys2,
                                                     uint32_t* __restrict__ meta2) {
  extern __shared__ uint64_t lds64[];
  const uint32_t nb2 = 1u << a2;
  const uint64_t desc = order[blockIdx.x];
  if (desc == kEmpty) return;
  const uint32_t tt = (uint32_t)desc & 0xFFFFF;
  const uint32_t c = (uint32_t)(desc >> 20) & 0x3FF;
  const uint64_t bo = bucket_off[c];
  const uint32_t t2 = 1u << t2_log2;
  const uint32_t p0 = (tt - tile_first[c]) << t2_log2;  // bucket-relative start
  const uint32_t n = (uint32_t)min((uint64_t)t2, bucket_off[c + 1] - bo - p0);
  uint64_t* stage = lds64;                                            // t2
  uint64_t* wsb = stage + t2;                                         // kThreads
  uint32_t* wrel = reinterpret_cast<uint32_t*>(wsb + kThreads);       // kThreads
  // once the gather is done the window arrays are free: the sort's counts,
  // starts and scan scratch take their place (this keeps two workgroups per
  // CU up to 2^10 sub-buckets)
  uint32_t* cnt = reinterpret_cast<uint32_t*>(wsb);                   // nb2
  uint32_t* start = cnt + nb2;                                        // nb2 + 1
  uint32_t* scratch = start + nb2 + 1;                                // kWaves + 1
  uint32_t* wend = reinterpret_cast<uint32_t*>(wsb) +
                   max((uint32_t)kThreads * 3, 2 * nb2 + 2 + kWaves); // 1
  const uint64_t* offc = off1 + (uint64_t)c * ntiles1;

  // gather: windows of kThreads first-level runs, binary search per key.  A
  // tile gathered in one window keeps its keys in registers: thread t holds
  // positions t + q kThreads, the ones the sort below takes.
  constexpr int kPer = kT2 / kThreads;
  uint64_t v[kPer];
  bool in_regs = false;
  uint64_t tw = desc >> 30;
  uint32_t got = 0;
  while (got < n) {
    const uint64_t t = tw + threadIdx.x;
    if (t < ntiles1) {
      const uint32_t rel = (uint32_t)(offc[t] - bo);
      wrel[threadIdx.x] = rel;
      wsb[threadIdx.x] = t * kTilePos + lstart[(uint64_t)c * ntiles1 + t] - rel;
    } else {
      wrel[threadIdx.x] = 0xFFFFFFFFu;
    }
    if (threadIdx.x == 0) {
      const uint64_t tn = tw + kThreads;
      *wend = tn < ntiles1 ? (uint32_t)(offc[tn] - bo) : (uint32_t)(bucket_off[c + 1] - bo);
    }
    __syncthreads();
    const uint32_t upto = min(n, *wend - p0);
    // each thread's kT2/kThreads positions: all run searches, then all loads,
    // then the LDS stores, so the loads are in flight together
    uint64_t src[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t p = got + threadIdx.x + q * kThreads;
      const uint32_t P = p0 + p;
      uint32_t r = 0;
#pragma unroll
      for (uint32_t step = kThreads / 2; step >= 1; step >>= 1)
        if (wrel[r + step] <= P) r += step;
      src[q] = wsb[r] + P;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      v[q] = (got + threadIdx.x + q * kThreads < upto) ? keys1[src[q]] : 0;
    in_regs = got == 0 && upto == n;  // block-uniform
    if (!in_regs) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const uint32_t p = got + threadIdx.x + q * kThreads;
        if (p < upto) stage[p] = v[q];
      }
    }
    got = upto;
    tw += kThreads;
    __syncthreads();
  }

  // sort by sub-bucket
  for (uint32_t i = threadIdx.x; i < nb2; i += kThreads) cnt[i] = 0;
  __syncthreads();
  uint64_t kv[kT2 / kThreads];
  uint32_t meta[kT2 / kThreads];
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    const uint32_t i = threadIdx.x + r * kThreads;
    if (i < n) {
      kv[r] = in_regs ? v[r] : stage[i];
      const uint32_t sub = (mix64_top31((kv[r] & kKeyMask) ^ s0) >> (32 - a1 - a2)) & (nb2 - 1);
      meta[r] = (sub << 16) | atomicAdd(&cnt[sub], 1u);
    }
  }
  __syncthreads();
  block_exclusive_scan(cnt, start, nb2, scratch);
  // sub-bucket starts read together, then the keys scattered; the sorted
  // tile read back from LDS together, then stored
  uint32_t bst[kT2 / kThreads];
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r)
    bst[r] = start[threadIdx.x + r * kThreads < n ? meta[r] >> 16 : 0u];
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    const uint32_t i = threadIdx.x + r * kThreads;
    if (i < n) stage[bst[r] + (meta[r] & 0xFFFF)] = kv[r];
  }
  __syncthreads();
  uint64_t* dst = keys2 + bo + p0;
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    const uint32_t i = threadIdx.x + r * kThreads;
    kv[r] = i < n ? stage[i] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kT2 / kThreads; ++r) {
    const uint32_t i = threadIdx.x + r * kThreads;
    if (i < n) dst[i] = kv[r];
  }
  for (uint32_t s = threadIdx.x; s <= nb2; s += kThreads)
    meta2[(uint64_t)tt * (nb2 + 1) + s] = start[s];
}

// ----------------------------------------- per-block Bloom + exact count

// Calls fn(kv, vmask, nbat, sub) for the stored occurrences of partitions
// [u_lo, u_hi), across segments: kv[b] holds one key per lane for b < nbat,
// valid where bit b of the lane's vmask is set.  Every lane of a wave reaches
// every call.  The whole block must call it.  The range's run inside a
// second-level tile is contiguous.  Wave w takes tiles g0 + w + NW*j (j =
// lane; NW waves per workgroup) and reads their run bounds once into its
// lanes.  Loads of the next B chunks are issued before the current B are
// handed to fn, so one batch is always in flight behind the one in use.
//
// FLAT = false walks run by run in chunks of 64 keys (a run's last chunk is
// partly empty), with wave-uniform bookkeeping: right for long runs.
// FLAT = true walks the concatenation of the wave's runs in full chunks of
// 64: the wave prefix-sums the run lengths; two ballots bound the runs that
// touch a chunk, and each lane steps through the few run starts inside it
// (scalar reads), or binary-searches the sums when a chunk holds many runs:
// right for short runs, where partly empty chunks would dominate.
//
// SUBL > 0 (run-by-run walk only): the range is 2^SUBL sub-ranges of
// sub_span partitions each, all in one first-level bucket, and bits
// 2b..2b+1 of `sub` give the sub-range of kv[b], found from the sub-bucket
// starts of the key's tile.  With SUBL = 0, sub is 0.
// s_waitcnt immediate (gfx9 encoding): vmcnt 0, expcnt and lgkmcnt unbounded.
constexpr int kWaitVm0 = 0x0F70;

template <int B>
struct RunBatch {
  uint64_t kv[B];
  uint32_t vmask;  // bit b: kv[b] holds a key for this lane
  uint32_t sub;    // bits 2b..2b+1: sub-range of kv[b] (SUBL > 0)
  uint32_t n;      // chunks in the batch (wave-uniform)
};


template <int NW, int B, bool FLAT, int SUBL = 0, typename F>
__device__ __forceinline__ void for_runs(const CountArgs& A, uint32_t u_lo, uint32_t u_hi,
                                         uint32_t sub_span, F&& fn) {
  static_assert(!(FLAT && SUBL), "sub-ranges need the run-by-run walk");
  static_assert(SUBL >= 0 && SUBL <= 2 && 2 * B <= 32, "sub-range bits");
  constexpr int NQ = (1 << SUBL) - 1;  // sub-range starts inside the range
  constexpr int NQA = NQ > 0 ? NQ : 1;
  const auto segs = cview(A.segs);
  for (uint32_t s = 0; s < A.nsegs; ++s) {
    const uint32_t a2 = segs[s].a2;
    const uint32_t t2s = segs[s].t2_log2;  // keys per second-level tile (log2)
    const uint32_t nb2 = 1u << a2;
    const uint32_t c_lo = u_lo >> a2, c_hi = (u_hi - 1) >> a2;
    const auto tile_first = cview(segs[s].tile_first);
    const auto bucket_off = cview(segs[s].bucket_off);
    const auto meta2 = gview(segs[s].meta2);
    const auto seg_keys = gview(segs[s].keys);
    for (uint32_t c = c_lo; c <= c_hi; ++c) {
      const uint32_t s_lo = max(u_lo, c << a2) - (c << a2);
      const uint32_t s_hi = min(u_hi, (c + 1) << a2) - (c << a2);
      const uint32_t t0 = tile_first[c], nt = tile_first[c + 1] - t0;
      const auto keys = seg_keys + bucket_off[c];
      for (uint32_t g0 = 0; g0 < nt; g0 += NW * 64) {
        const uint32_t tw = g0 + wave_id();  // this wave's first tile (bucket-relative)
        if (tw >= nt) break;
        const uint32_t nj = min(64u, (nt - tw + NW - 1) / NW);
        const uint32_t ti = tw + NW * lane_id();
        uint32_t mm0 = 0, mm1 = 0;
        uint32_t mq[NQA];  // lane j: tile-relative starts of sub-ranges 1..NQ
#pragma unroll
        for (int q = 0; q < NQA; ++q) mq[q] = 0;
        if (lane_id() < nj) {
          const auto m = meta2 + (uint64_t)(t0 + ti) * (nb2 + 1);
          mm0 = m[s_lo];
          mm1 = m[s_hi];
#pragma unroll
          for (int q = 0; q < NQ; ++q) mq[q] = m[s_lo + (q + 1) * sub_span];
        }
        // Next B chunks of the walk, their loads issued.  The B loads are
        // issued unconditionally, after the bookkeeping, so that the compiler
        // can count them and wait for the older batch only.  Lanes without a
        // key load the bucket's first key (the bucket holds at least one, as
        // it has a tile) and are masked off in vmask.
        uint32_t j = 0;
        uint32_t i = __builtin_amdgcn_readlane(mm0, 0), e = __builtin_amdgcn_readlane(mm1, 0);
        uint32_t bq[NQA];  // sub-range starts of tile j (wave-uniform)
#pragma unroll
        for (int q = 0; q < NQA; ++q) bq[q] = NQ ? __builtin_amdgcn_readlane(mq[q], 0) : 0u;
        // FLAT: lane j's run starts at position excl of the concatenation
        // (lanes past nj hold the total, which no position reaches)
        const uint32_t len = mm1 - mm0;
        const uint32_t incl = FLAT ? wave_incl_scan(len) : 0u;
        const uint32_t total = FLAT ? __builtin_amdgcn_readlane(incl, 63) : 0u;
        const uint32_t excl = lane_id() < nj ? incl - len : total;
        // FLAT: key index of position v in run j is rb(j) + v (mod 2^32),
        // with rb(j) = tile(j) 2^t2s + start(j) - excl(j): one value per run
        // to select per lane, instead of the run, its start and its offset
        const uint32_t rb = FLAT ? ((tw + NW * lane_id()) << t2s) + mm0 - excl : 0u;
        uint32_t v0 = 0;  // FLAT: next position of the concatenation
        auto next_flat = [&](RunBatch<B>& r) {
          uint32_t off[B];
          r.vmask = 0;
          r.sub = 0;
          r.n = v0 < total ? min((uint32_t)B, (total - v0 + 63) >> 6) : 0u;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const uint32_t vb = v0 + 64 * b;  // chunk start (wave-uniform)
            const uint32_t v = vb + lane_id();
            const bool ok = v < total;
            const uint32_t vc = ok ? v : vb;
            // Runs touching the chunk: lanes jlo..jhi (excl is non-decreasing
            // over lanes, so each ballot is a prefix of the lanes).
            const uint64_t le_lo = __ballot(excl <= vb);
            const uint64_t le_hi = __ballot(excl <= vb + 63);
            const uint32_t jlo = le_lo ? 63 - (uint32_t)__builtin_clzll(le_lo) : 0u;
            const uint32_t jhi = le_hi ? 63 - (uint32_t)__builtin_clzll(le_hi) : 0u;
            uint32_t base;
            if (jhi - jlo <= 8) {
              // few run starts inside the chunk: step through them (scalar reads)
              base = __builtin_amdgcn_readlane(rb, jlo);
              for (uint32_t t = jlo + 1; t <= jhi; ++t) {
                const uint32_t et = __builtin_amdgcn_readlane(excl, t);
                const uint32_t bt = __builtin_amdgcn_readlane(rb, t);
                base = vc >= et ? bt : base;
              }
            } else {
              // many short runs: binary search over the lanes' run starts
              uint32_t jj = 0;
#pragma unroll
              for (int sp = 32; sp >= 1; sp >>= 1) {
                const uint32_t e = __shfl(excl, jj + sp, 64);
                jj = e <= vc ? jj + sp : jj;
              }
              base = __shfl(rb, jj, 64);
            }
            off[b] = ok ? base + vc : 0u;
            r.vmask |= (uint32_t)ok << b;
          }
          v0 += 64 * B;
#pragma unroll
          for (int b = 0; b < B; ++b) r.kv[b] = keys[off[b]];
        };
        auto next_runs = [&](RunBatch<B>& r) {
          uint32_t off[B];
          r.n = 0;
          r.vmask = 0;
          r.sub = 0;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            while (j < nj && i >= e) {
              ++j;
              if (j < nj) {
                i = __builtin_amdgcn_readlane(mm0, j);
                e = __builtin_amdgcn_readlane(mm1, j);
#pragma unroll
                for (int q = 0; q < NQ; ++q) bq[q] = __builtin_amdgcn_readlane(mq[q], j);
              }
            }
            off[b] = 0;
            if (j < nj) {
              const uint32_t idx = i + lane_id();
              const bool ok = idx < e;
              off[b] = ok ? ((tw + NW * j) << t2s) + idx : 0u;
              r.vmask |= (uint32_t)ok << b;
              uint32_t sb = 0;
#pragma unroll
              for (int q = 0; q < NQ; ++q) sb += idx >= bq[q] ? 1u : 0u;
              r.sub |= sb << (2 * b);
              i += 64;
              r.n = b + 1;
            }
          }
#pragma unroll
          for (int b = 0; b < B; ++b) r.kv[b] = keys[off[b]];
        };
        auto next = [&](RunBatch<B>& r) {
          if constexpr (FLAT)
            next_flat(r);
          else
            next_runs(r);
        };
        // Two batches alternate roles (no copy of registers whose loads are
        // still in flight, which would have to wait for them).
        RunBatch<B> x, y;
        next(x);
        while (x.n) {
          next(y);
          fn(x.kv, x.vmask, x.n, x.sub);
          if (!y.n) break;
          next(x);
          fn(y.kv, y.vmask, y.n, y.sub);
        }
        // The last batch's (masked) loads land here, once per group of
        // tiles, instead of at the loop head on every pass.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
      }
    }
  }
}

// In-block bit positions of S(x): a + i*b mod 2^bl for i < H, with a and b
// the top two bl-bit fields of mix64(x ^ s_1) (double hashing: one hash for
// all H positions).  dup[i] marks a position equal to an earlier one (S(x) is
// a set: one hit per occurrence per distinct bit).  Position i equals
// position j < i exactly when 2^bl divides (i - j) * b; the largest power of
// two among 1..i is 2^floor(log2 i), so position i repeats an earlier one
// exactly when b has at least bl - floor(log2 i) trailing zero bits (all of
// them when b = 0).
template <int H>
__device__ __forceinline__ void bloom_positions(const HashCfg& hc, uint64_t x, uint32_t pos[H],
                                                bool dup[H]) {
  static_assert(H >= 1 && H <= 8, "bloom_positions: 1..8 hashes");
  const uint64_t u = mix64(x ^ hc.salt[1]);
  const uint32_t mask = (1u << hc.bl) - 1u;
  const uint32_t a = (uint32_t)(u >> (64 - hc.bl));
  const uint32_t b = (uint32_t)(u >> (64 - 2 * hc.bl)) & mask;
  const uint32_t tz = b ? (uint32_t)__builtin_ctz(b) : 32u;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    pos[i] = (a + (uint32_t)i * b) & mask;
    const uint32_t lg = i >= 4 ? 2u : i >= 2 ? 1u : 0u;  // floor(log2 i) for 1 <= i < 8
    dup[i] = i > 0 && tz + lg >= hc.bl;
  }
}

__device__ __forceinline__ uint32_t home_slot(uint64_t th, uint32_t cap) {
  return home_slot_of(th, cap);
}

// Once more keys than ovf_limit have been placed the pass is void (the host
// grows the table and runs it again), so an insert stops as soon as it sees
// the limit passed, on entry and every 32 probes: a table filled far beyond
// its limit would otherwise make each later key probe every slot.
__device__ void overflow_add(const CountArgs& A, uint64_t x, uint32_t tag, uint64_t th) {
  const uint32_t nc = A.hc.nc;
  const uint64_t mask = (1ull << A.ovf_log2) - 1;
  uint64_t slot = th >> (64 - A.ovf_log2);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    if ((probe & 31) == 0 &&
        __hip_atomic_load(A.ovf_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > A.ovf_limit) {
      atomicOr(A.err, (uint32_t)ERR_OVF_LOAD);
      return;
    }
    uint64_t cur = __hip_atomic_load(&A.okeys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kEmpty) {
      cur = atomicCAS(reinterpret_cast<unsigned long long*>(&A.okeys[slot]),
                      (unsigned long long)kEmpty, (unsigned long long)x);
      if (cur == kEmpty) {
        const uint32_t used = atomicAdd(A.ovf_used, 1u) + 1;
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

// Pass 1 (Prune), one workgroup per Bloom block: the block's two levels are
// built in LDS from every occurrence of its partitions (every occurrence hits
// each distinct bit of S(x) once; level 1 records a first hit of a bit, level
// 2 a second one) and written out with their popcounts.  Eight waves per
// SIMD (at most 64 VGPRs): with blocks of up to 2^18 bits two workgroups then
// share a CU.  A workgroup takes 2^SUBL consecutive blocks (blocks smaller
// than 2^18 bits, so that its LDS and its runs are those of one larger
// block); each key's block is its sub-range in the walk.  FLAT picks the walk
// over the runs: the flattened one when the workgroup's blocks hold one or two
// partitions, whose runs in a second-level tile are short; run by run
// otherwise.
template <int H, bool FLAT, int SUBL>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_bloom(const CountArgs A) {
  extern __shared__ uint32_t lds[];
  const HashCfg& hc = A.hc;
  const uint32_t blk = blockIdx.x << SUBL;  // first block of the workgroup
  const uint32_t nbw = A.nbw << SUBL;      // words per level, all its blocks
  const uint32_t span = 1u << A.upb_log2;  // partitions per block
  const uint32_t u0 = blk << A.upb_log2, nu = span << SUBL;
  uint32_t* L2 = lds;
  uint32_t* L1 = lds + A.l2w;
  for (uint32_t i = threadIdx.x; i < A.l2w + nbw; i += kThreads) lds[i] = 0;
  __syncthreads();
  const uint32_t sub_sh = SUBL ? hc.bl - 5 : 0u;  // words per block (log2)
  constexpr int NB = FLAT || SUBL ? 4 : 8;  // chunks per batch (within 64 VGPRs)
  for_runs<kWaves, NB, FLAT, SUBL>(A, u0, u0 + nu, span, [&](const uint64_t (&kv)[NB],
                                                               uint32_t vmask, uint32_t nbat,
                                                               uint32_t sub) {
    constexpr int G = 2;  // keys whose level-1 updates are in flight together
#pragma unroll
    for (int g = 0; g < NB / G; ++g) {
      if (g * G >= (int)nbat) break;
      uint32_t pos[G][H], old[G][H], w0[G];
      bool dup[G][H];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        bloom_positions<H>(hc, kv[g * G + q] & kKeyMask, pos[q], dup[q]);
        w0[q] = SUBL ? ((sub >> (2 * (g * G + q))) & 3u) << sub_sh : 0u;  // the key's block
#pragma unroll
        for (int i = 0; i < H; ++i) dup[q][i] |= !((vmask >> (g * G + q)) & 1u);
      }
#pragma unroll
      for (int q = 0; q < G; ++q)
#pragma unroll
        for (int i = 0; i < H; ++i)
          old[q][i] = dup[q][i] ? 0u
                                : atomicOr(&L1[w0[q] + (pos[q][i] >> 5)], 1u << (pos[q][i] & 31));
#pragma unroll
      for (int q = 0; q < G; ++q)
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const uint32_t bit = 1u << (pos[q][i] & 31);
          if (old[q][i] & bit) atomicOr(&L2[w0[q] + (pos[q][i] >> 5)], bit);
        }
    }
  });
  __syncthreads();
  uint64_t p1 = 0, p2 = 0;
  if (hc.bl >= 5) {
    for (uint32_t i = threadIdx.x; i < nbw; i += kThreads) {
      const uint32_t a = L1[i], b = L2[i];
      A.b1[(uint64_t)blk * A.nbw + i] = a;
      A.b2[(uint64_t)blk * A.nbw + i] = b;
      p1 += __popc(a);
      p2 += __popc(b);
    }
  } else if (threadIdx.x == 0) {
    const uint64_t bit0 = (uint64_t)blk << hc.bl;
    const uint32_t msk = (1u << (1u << hc.bl)) - 1u;
    const uint32_t a = L1[0] & msk, b = L2[0] & msk;
    atomicOr(&A.b1[bit0 >> 5], a << (bit0 & 31));
    atomicOr(&A.b2[bit0 >> 5], b << (bit0 & 31));
    p1 += __popc(a);
    p2 += __popc(b);
  }
  p1 = wave_sum(p1);
  p2 = wave_sum(p2);
  __syncthreads();
  uint64_t* red = reinterpret_cast<uint64_t*>(lds);
  if (lane_id() == 0) {
    red[wave_id() * 2] = p1;
    red[wave_id() * 2 + 1] = p2;
  }
  __syncthreads();
  // one statistics row per workgroup
  if (threadIdx.x < kNst) {
    uint64_t v = 0;
    if (threadIdx.x == ST_B1POP || threadIdx.x == ST_B2POP)
      for (int w = 0; w < kWaves; ++w) v += red[w * 2 + (threadIdx.x == ST_B2POP)];
    A.pstats[(uint64_t)blockIdx.x * kNst + threadIdx.x] = v;
  }
}

// Partition handled by workgroup i.  The hardware hands consecutive
// workgroups to the 8 XCDs in turn; this mapping gives the partitions of one
// Bloom block to workgroups of one XCD, launched close together, so that
// block's level-2 words are read through one L2.
// The launch covers n partitions starting at a Bloom-block boundary; the
// mapping applies when n is a whole number of 8-block groups (otherwise the
// identity).  Returns the partition's index within the launch.
__device__ __forceinline__ uint32_t tally_partition(uint32_t i, uint32_t upb_log2, uint32_t n) {
  const uint32_t upb = 1u << upb_log2;
  if (n & (8 * upb - 1)) return i;
  const uint32_t xcd = i & 7, slot = i >> 3;
  return (slot & (upb - 1)) + upb * (xcd + 8 * (slot >> upb_log2));
}

constexpr int kTallyThreads = kTallyWaves * 64;

// Pass 2 (Count) and Unify, one workgroup per partition.  Every occurrence
// probes the partition's LDS open-addressing table; hits count at once; misses
// (keys not yet in the table) queue per wave and are screened against level 2
// densely, 64 at a time; passing keys are inserted (CAS on the key, add on the
// count), failing ones dropped.  A key whose probe sequence fills up goes,
// with all its occurrences, to the device overflow table.  The table is then
// written to HBM with counts below min_count zeroed.
template <int H>
__global__ void __launch_bounds__(kTallyThreads)
k_tally(const CountArgs A) {
  extern __shared__ uint32_t lds[];
  const HashCfg& hc = A.hc;
  const uint32_t lu = tally_partition(blockIdx.x, A.upb_log2, A.part_n);
  const uint32_t u = A.part_base + lu;
  const uint32_t cap = A.cap;
  const uint32_t nc = hc.nc;
  const uint32_t blk = u >> A.upb_log2;
  const uint64_t bit0 = (uint64_t)blk << hc.bl;
  // the block's level-2 words from the word holding its first bit (a block
  // of fewer than 32 bits lies inside that word, from bit b2_off on)
  const uint32_t* b2 = A.b2 + (bit0 >> 5);
  const uint32_t b2_off = (uint32_t)bit0 & 31u;
  uint64_t* tk = reinterpret_cast<uint64_t*>(lds);
  uint32_t* tc = reinterpret_cast<uint32_t*>(tk + cap);
  uint64_t* qk = reinterpret_cast<uint64_t*>(tc + (size_t)cap * nc) + wave_id() * 64;
  uint32_t* qs = reinterpret_cast<uint32_t*>(reinterpret_cast<uint64_t*>(tc + (size_t)cap * nc) +
                                             kTallyWaves * 64) + wave_id() * 64;
  uint32_t n_ovf = 0;  // occurrences counted in the overflow table
  const uint32_t limit = A.probe_limit;

  // the table cleared with 16-byte stores (cap is a multiple of 64, so both
  // arrays are whole 16-byte units on 16-byte boundaries)
  for (uint32_t i = threadIdx.x; i < cap / 2; i += kTallyThreads)
    reinterpret_cast<u64x2*>(tk)[i] = u64x2{kEmpty, kEmpty};
  for (uint32_t i = threadIdx.x; i < cap * nc / 4; i += kTallyThreads)
    reinterpret_cast<u32x4*>(tc)[i] = u32x4{0u, 0u, 0u, 0u};
  __syncthreads();

  // Resolves the queued occurrences densely, 64 at a time.  Every queued key
  // is screened against level 2 first: the words of its bit positions are
  // loaded for all lanes at once.  Passing is a property of the key (S(x) in
  // B2), so a key that fails is not in the table and is dropped, and a key
  // that passes walks its probe chain with CAS from where the main loop left
  // it (the home slot, or the slot after it when the home slot held another
  // key): it is counted where it is found or inserted at the first empty
  // slot (a CAS lost to another key walks on), or, past the probe limit,
  // counted in the overflow table.
  auto drain = [&](uint32_t n) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const bool have = lane_id() < n;
    uint64_t key = 0;
    uint32_t slot = 0, probes = 0;
    if (have) {
      key = qk[lane_id()];
      // the walk's first slot (bits 0-27) and the slots before it already
      // known to hold other keys (bits 28-30)
      slot = qs[lane_id()] & 0x0FFFFFFFu;
      probes = qs[lane_id()] >> 28;
    }
    const uint64_t x = key & kKeyMask;
    const uint32_t tag = (uint32_t)(key >> 62);
    // positions a + i*b in the partition's Bloom block (in bounds for any x,
    // so lanes without a key load too)
    const uint64_t u = mix64(x ^ hc.salt[1]);
    const uint32_t mask = (1u << hc.bl) - 1u;
    const uint32_t a = (uint32_t)(u >> (64 - hc.bl));
    const uint32_t b = (uint32_t)(u >> (64 - 2 * hc.bl)) & mask;
    uint32_t w[H], q[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      q[i] = b2_off + ((a + (uint32_t)i * b) & mask);
      w[i] = b2[q[i] >> 5];
    }
    bool pass = have;
#pragma unroll
    for (int i = 0; i < H; ++i) pass &= ((w[i] >> (q[i] & 31u)) & 1u) != 0;
    if (pass) {
      const uint64_t th = (x ^ hc.salt[0]) * kTableMul;
      for (;;) {
        if (probes >= limit) {
          ++n_ovf;
          overflow_add(A, x, tag, mix64(th));
          break;
        }
        uint64_t cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tk[slot]),
                                 (unsigned long long)kEmpty, (unsigned long long)x);
        if (cur == kEmpty) cur = x;
        if (cur == x) {
          atomicAdd(&tc[slot * nc + tag], 1u);
          break;
        }
        slot = slot + 1 == cap ? 0 : slot + 1;
        ++probes;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  };

  uint32_t qn = 0;  // wave-uniform queue length
  constexpr int B2 = 2;
  for_runs<kTallyWaves, B2, true>(A, u, u + 1, 1, [&](const uint64_t (&kv)[B2], uint32_t vmask,
                                                     uint32_t nbat, uint32_t /*sub*/) {
    // One read of the home bucket per occurrence (its kBucket keys, two
    // 16-byte LDS loads), scanned in probe order: x found before any open
    // slot counts at once; any other outcome (a new key, a key stored past
    // its bucket, or x behind a slot read while another wave filled it) is
    // queued with the first slot of the bucket not known to hold another
    // key, where the walk resolves it.  The loads are not
    // atomic, so a key being written by another wave's CAS may be read torn,
    // one half still from kEmpty (all ones); no canonical key has a 32-bit
    // half of all ones (x < 2^62, and x ending in 16 T bases would have a
    // smaller reverse complement for k <= 31), so a torn value never equals
    // x and is never taken for a slot that holds another key.
    constexpr int KB = (int)kBucket;
    static_assert(KB == 4, "the bucket read is two 16-byte loads");
    uint32_t stop[B2], slot0[B2];
#pragma unroll
    for (int b = 0; b < B2; ++b) {
      const uint64_t x = kv[b] & kKeyMask;
      slot0[b] = home_slot((x ^ hc.salt[0]) * kTableMul, cap);
      // every lane reads a bucket (a lane without a key holds some stored
      // key, so its slot is in range); the result counts only where valid
      typedef __attribute__((address_space(3))) const volatile u64x2 lds_pair;
      const lds_pair* bp = (const lds_pair*)(tk + slot0[b]);
      const u64x2 lo = bp[0], hi = bp[1];
      const uint64_t v[KB] = {lo.x, lo.y, hi.x, hi.y};
      // The first slot, in probe order, that holds x (bit 3 set) or is empty
      // or torn (a 32-bit half of all ones); KB when all hold other keys.
      // On a miss the slots before it hold other keys.
      stop[b] = KB;
#pragma unroll
      for (int i = KB - 1; i >= 0; --i) {
        const bool is_x = v[i] == x;
        const bool open = max((uint32_t)v[i], (uint32_t)(v[i] >> 32)) == 0xFFFFFFFFu;
        stop[b] = is_x || open ? (uint32_t)i | (is_x ? 8u : 0u) : stop[b];
      }
    }
#pragma unroll
    for (int b = 0; b < B2; ++b) {
      if (b >= (int)nbat) break;
      const uint64_t key = kv[b];
      const uint32_t tag = (uint32_t)(key >> 62);
      const bool valid = (vmask >> b) & 1u;
      const bool hit = valid && (stop[b] & 8u);
      const uint32_t skip = stop[b] & 7u;
      if (hit) atomicAdd(&tc[(slot0[b] + skip) * nc + tag], 1u);
      const bool miss = valid && !hit;
      const uint64_t mb = __ballot(miss);
      const uint32_t nm = (uint32_t)__popcll(mb);
      if (!nm) continue;
      // missing lanes below this one (two mbcnt instructions)
      const uint32_t rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
      const uint32_t room = 64 - qn;
      const uint32_t first = slot0[b] + skip == cap ? 0u : slot0[b] + skip;
      const uint32_t qv = first | (skip << 28);
      if (miss && rank < room) {
        qk[qn + rank] = key;
        qs[qn + rank] = qv;
      }
      if (nm >= room) {
        drain(64);
        if (miss && rank >= room) {
          qk[rank - room] = key;
          qs[rank - room] = qv;
        }
        qn = nm - room;
      } else {
        qn += nm;
      }
    }
  });
  if (qn) drain(qn);
  __syncthreads();

  // Per-wave statistics: slot counts (passed keys, false-positive
  // singletons, entries) by ballot, wave-uniform; count sums per lane, then
  // summed over the wave with the overflow occurrences (three wave sums
  // instead of one per statistic).
  // Two slots per thread and step: 16-byte LDS reads of their keys (and of
  // their counts with two counters) and 16- / 8-byte stores.
  uint64_t npass = 0, sum = 0, passed = 0, fp = 0, entries = 0;
  const uint64_t base = (uint64_t)(A.slot_base + lu) * cap;
  for (uint32_t i2 = threadIdx.x; i2 < cap / 2; i2 += kTallyThreads) {
    const uint32_t i = 2 * i2;
    const u64x2 kp = reinterpret_cast<const u64x2*>(tk)[i2];
    uint32_t c[2][2];
    if (nc > 1) {
      const u32x4 cq = reinterpret_cast<const u32x4*>(tc)[i2];
      c[0][0] = cq.x; c[0][1] = cq.y; c[1][0] = cq.z; c[1][1] = cq.w;
    } else {
      const uint64_t cp = reinterpret_cast<const uint64_t*>(tc)[i2];
      c[0][0] = (uint32_t)cp; c[0][1] = 0; c[1][0] = (uint32_t)(cp >> 32); c[1][1] = 0;
    }
    const uint64_t key[2] = {kp.x, kp.y};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const bool used = key[e] != kEmpty;
      const uint64_t tot = (uint64_t)c[e][0] + c[e][1];
      const bool kept = used && tot >= hc.min_count;
      passed += (uint64_t)__popcll(__ballot(used));
      fp += (uint64_t)__popcll(__ballot(used && tot == 1));
      entries += (uint64_t)__popcll(__ballot(kept));
      npass += used ? tot : 0;
      sum += kept ? tot : 0;
      if (!kept) c[e][0] = c[e][1] = 0;
    }
    *reinterpret_cast<u64x2*>(A.tkeys + base + i) = kp;
    if (nc > 1)
      *reinterpret_cast<u32x4*>(A.tcounts + (base + i) * 2) = u32x4{c[0][0], c[0][1], c[1][0], c[1][1]};
    else
      *reinterpret_cast<uint64_t*>(A.tcounts + base + i) =
          (uint64_t)c[0][0] | ((uint64_t)c[1][0] << 32);
  }
  __syncthreads();
  uint64_t* red = reinterpret_cast<uint64_t*>(lds);
  {
    uint64_t st[kNst];
#pragma unroll
    for (int i = 0; i < kNst; ++i) st[i] = 0;
    st[ST_PASSED] = passed;
    st[ST_FP] = fp;
    st[ST_ENTRIES] = entries;
    st[ST_NPASS] = wave_sum(npass);
    st[ST_SUM] = wave_sum(sum);
    st[ST_OVF] = wave_sum((uint64_t)n_ovf);
    if (lane_id() == 0)
#pragma unroll
      for (int i = 0; i < kNst; ++i) red[wave_id() * kNst + i] = st[i];
  }
  __syncthreads();
  if (threadIdx.x < kNst) {
    uint64_t sum = 0;
    for (int w = 0; w < kTallyWaves; ++w) sum += red[w * kNst + threadIdx.x];
    A.pstats2[(uint64_t)u * kNst + threadIdx.x] = sum;
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

// Column sums of nrows statistics rows into out[kNst] (zeroed before): each
// workgroup sums a grid-stride share of the rows and adds its sums to out
// with integer atomics, so the result does not depend on the order.
__global__ void __launch_bounds__(kThreads) k_reduce(const uint64_t* __restrict__ rows,
                                                     uint64_t nrows, uint64_t* __restrict__ out) {
  __shared__ uint64_t red[kWaves * kNst];
  uint64_t st[kNst] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (uint64_t r = (uint64_t)blockIdx.x * kThreads + threadIdx.x; r < nrows;
       r += (uint64_t)gridDim.x * kThreads)
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
    if (s) atomicAdd(reinterpret_cast<unsigned long long*>(&out[threadIdx.x]), (unsigned long long)s);
  }
}

// ----------------------------------------------------------------- query

// Linear probing in a table of n slots starting at `slot`, at most `limit`
// probes; true with the slot index when x is present.
__device__ __forceinline__ bool probe_table(const uint64_t* keys, uint64_t base, uint64_t n,
                                            uint64_t limit, uint64_t slot, uint64_t x,
                                            uint64_t* at) {
  for (uint64_t p = 0; p < limit; ++p) {
    const uint64_t cur = keys[base + slot];
    if (cur == x) {
      *at = base + slot;
      return true;
    }
    if (cur == kEmpty) return false;
    slot = slot + 1 == n ? 0 : slot + 1;
  }
  return false;
}

// Lookup of canonical key x in a partition table at keys[base ..] (cap slots,
// home slot `slot`, at most `limit` probes; both multiples of kBucket): a
// bucket's kBucket keys are read at once (two 16-byte loads of one aligned
// 32-byte range) and scanned in probe order, which ends at x (true, its slot
// index in *at) or at an empty slot (false: linear probing never stores a key
// past an empty slot of its probe sequence).  With SEL, keys carry the
// filter's selection mark in bit 63, ignored in the comparison; *stored is
// the stored key of a hit.
template <bool SEL>
__device__ __forceinline__ bool probe_buckets(const uint64_t* keys, uint64_t base, uint32_t cap,
                                              uint32_t limit, uint32_t slot, uint64_t x,
                                              uint64_t* at, uint64_t* stored = nullptr) {
  constexpr uint64_t kSel = 1ull << 63;
  for (uint32_t p = 0; p < limit; p += kBucket) {
    const u64x2* b = reinterpret_cast<const u64x2*>(keys + base + slot);
    const u64x2 lo = b[0], hi = b[1];
    const uint64_t v[4] = {lo.x, lo.y, hi.x, hi.y};
    uint32_t found = 0, empty = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      found |= (uint32_t)(((SEL ? v[i] & ~kSel : v[i])) == x) << i;
      empty |= (uint32_t)(v[i] == kEmpty) << i;
    }
    if (found | empty) {
      const uint32_t i = (uint32_t)__builtin_ctz(found | empty);
      *at = base + slot + i;
      if (stored) *stored = i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
      return (found >> i) & 1u;
    }
    slot = slot + kBucket == cap ? 0 : slot + kBucket;
  }
  return false;
}

// Table slot of partition u: computed when the slot map is the layout finalize
// makes (partitions below slot_first spilled, the rest in order), which saves
// a dependent load per lookup; read from the map otherwise.
__device__ __forceinline__ uint32_t table_slot(const QueryArgs& A, uint64_t u) {
  if (A.slot_first >= 0)
    return u >= (uint64_t)A.slot_first ? (uint32_t)(u - (uint64_t)A.slot_first) : kNoSlot;
  return A.slot_of[u];
}

// Counts of the canonical key x in the final tables: its partition's table in
// HBM, else the overflow table (a key lives in one of the two, never both).
// Returns 1 when found, 0 when absent, -1 when its partition's table is not
// in HBM (spilled) and the key is not in the overflow table: then it is
// unknown here.
__device__ __forceinline__ int table_counts(const QueryArgs& A, uint64_t x, uint32_t* c0,
                                            uint32_t* c1) {
  const uint32_t nc = A.hc.nc;
  const uint64_t u = top_bits(mix64(x ^ A.hc.salt[0]), A.hc.p_log2);
  const uint64_t th = (x ^ A.hc.salt[0]) * kTableMul;
  const uint32_t slot = table_slot(A, u);
  uint64_t at;
  if (slot != kNoSlot &&
      probe_buckets<false>(A.tkeys, (uint64_t)slot * A.cap, (uint32_t)A.cap, A.probe_limit,
                           home_slot(th, (uint32_t)A.cap), x, &at)) {
    *c0 = A.tcounts[at * nc];
    if (nc > 1) *c1 = A.tcounts[at * nc + 1];
    return 1;
  }
  if (*A.ovf_used &&
      probe_table(A.okeys, 0, 1ull << A.ovf_log2, 1ull << A.ovf_log2,
                  mix64(th) >> (64 - A.ovf_log2), x, &at)) {
    *c0 = A.ocounts[at * nc];
    if (nc > 1) *c1 = A.ocounts[at * nc + 1];
    return 1;
  }
  return slot == kNoSlot ? -1 : 0;
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
    if (table_counts(A, x, &c0, &c1) < 0) {
      const uint32_t h = atomicAdd(A.host_count, 1u);  // answered from the host copy
      A.host_rows[h] = (uint32_t)i;
      A.host_keys[h] = x;
    }
  }
  out[i * nc] = c0;
  if (nc > 1) out[i * nc + 1] = c1;
}

// The filter's selection rule on a key's counts: tumour count >= tmin and
// normal count <= nmax (counters 1 and 0 of a two-counter table; normal 0
// and tumour = the count for one counter; 0 and 0 when absent).
__device__ __forceinline__ bool filter_pass(uint32_t nc, uint32_t c0, uint32_t c1, uint32_t tmin,
                                            uint32_t nmax) {
  const uint32_t tumour = nc > 1 ? c1 : c0, normal = nc > 1 ? c0 : 0u;
  return tumour >= tmin && normal <= nmax;
}

constexpr uint64_t kSelBit = 1ull << 63;  // selection mark of a filter key (keys are < 2^62)

// One thread per table slot: the slot's key, marked when its counts pass.
__global__ void __launch_bounds__(256) k_filter_keys(const uint64_t* __restrict__ tkeys,
                                                     const uint32_t* __restrict__ tcounts,
                                                     uint64_t nslots, uint32_t nc, uint32_t tmin,
                                                     uint32_t nmax, uint64_t* __restrict__ fkeys) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = tkeys[i];
    const uint32_t c0 = tcounts[i * nc], c1 = nc > 1 ? tcounts[i * nc + 1] : 0u;
    fkeys[i] = key == kEmpty ? kEmpty : key | (filter_pass(nc, c0, c1, tmin, nmax) ? kSelBit : 0);
  }
}

// Whether canonical key x is selected: one probe sequence over the marked
// keys of its partition table (one random line per lookup instead of a key
// line and a count line), else the overflow table's counts, else absent.
__device__ __forceinline__ bool filter_selected(const QueryArgs& A, uint64_t x, uint32_t tmin,
                                                uint32_t nmax) {
  const uint64_t th = (x ^ A.hc.salt[0]) * kTableMul;
  const uint64_t u = top_bits(mix64(x ^ A.hc.salt[0]), A.hc.p_log2);
  const uint64_t base = (uint64_t)table_slot(A, u) * A.cap;
  uint64_t at, stored;
  if (probe_buckets<true>(A.fkeys, base, (uint32_t)A.cap, A.probe_limit,
                          home_slot(th, (uint32_t)A.cap), x, &at, &stored))
    return (stored >> 63) != 0;
  uint32_t c0 = 0, c1 = 0;
  if (*A.ovf_used && probe_table(A.okeys, 0, 1ull << A.ovf_log2, 1ull << A.ovf_log2,
                                 mix64(th) >> (64 - A.ovf_log2), x, &at)) {
    c0 = A.ocounts[at * A.hc.nc];
    if (A.hc.nc > 1) c1 = A.ocounts[at * A.hc.nc + 1];
  }
  return filter_pass(A.hc.nc, c0, c1, tmin, nmax);
}

// Filter-unit lookup, first pass: bit j of hit[w] marks the window ending at
// base j of packed word w when its canonical k-mer is selected (filter_pass).
// Four consecutive threads share a word, eight windows each; every table is
// in HBM (the caller checks).  With A.fkeys the lookups read the marked keys
// (filter_selected), otherwise keys and counts (table_counts).
__global__ void __launch_bounds__(256) k_filter_windows(const QueryArgs A,
                                                        const uint64_t* __restrict__ packed,
                                                        const uint64_t* __restrict__ flags,
                                                        uint64_t nwords, uint32_t tmin,
                                                        uint32_t nmax, uint32_t* __restrict__ hit) {
  constexpr int kPP = 8, kTPW = 4;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t w = t / kTPW;
  uint32_t bits = 0;
  if (w < nwords) {
    const WordCtx c = load_word(packed, flags, w);
    const int j0 = (int)(t % kTPW) * kPP;
    for (int jj = 0; jj < kPP; ++jj) {
      uint64_t x;
      if (!window_key(c, A.hc.k, j0 + jj, &x)) continue;
      bool sel;
      if (A.fkeys) {
        sel = filter_selected(A, x & kKeyMask, tmin, nmax);
      } else {
        uint32_t c0 = 0, c1 = 0;
        table_counts(A, x & kKeyMask, &c0, &c1);
        sel = filter_pass(A.hc.nc, c0, c1, tmin, nmax);
      }
      if (sel) bits |= 1u << (j0 + jj);
    }
  }
  bits |= __shfl_xor(bits, 1, 64);
  bits |= __shfl_xor(bits, 2, 64);
  if (w < nwords && t % kTPW == 0) hit[w] = bits;
}

// Filter-unit lookup, second pass: out[r] = set bits of hit over read r's
// positions [offsets[r], offsets[r+1]) (a window belongs to the read its
// last base is in).  The range is clamped to [0, total): offsets are checked
// on the host only after this pass has run.
__global__ void __launch_bounds__(256) k_filter_reads(const uint64_t* __restrict__ offsets,
                                                      uint64_t n_reads, uint64_t total,
                                                      const uint32_t* __restrict__ hit,
                                                      uint32_t* __restrict__ out) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const uint64_t hi = min(offsets[r + 1], total), lo = min(offsets[r], hi);
  uint32_t n = 0;
  for (uint64_t p = lo; p < hi;) {
    const uint32_t b = (uint32_t)(p & 31);
    const uint64_t take = min((uint64_t)(32 - b), hi - p);
    const uint32_t m = (take == 32 ? 0xFFFFFFFFu : ((1u << take) - 1u)) << b;
    n += __popc(hit[p >> 5] & m);
    p += take;
  }
  out[r] = n;
}

// Entries with a nonzero count, appended in no particular order.  Each
// workgroup walks chunks of kThreads slots (grid-stride) and reserves room for
// a chunk's entries with one atomic on the shared cursor: one atomic per
// kThreads slots, not per wave, keeps the cursor from serialising the pass.
__global__ void __launch_bounds__(kThreads) k_export(const uint64_t* __restrict__ tkeys,
                                                     const uint32_t* __restrict__ tcounts,
                                                     uint64_t nslots,
                                                     const uint32_t* __restrict__ live,
                                                     uint32_t cap, uint32_t nc,
                                                     uint64_t* __restrict__ out_keys,
                                                     uint32_t* __restrict__ out_counts,
                                                     uint64_t out_cap,
                                                     uint64_t* __restrict__ cursor) {
  __shared__ uint32_t wcnt[kWaves];
  __shared__ uint64_t wgbase;
  for (uint64_t c0i = (uint64_t)blockIdx.x * kThreads; c0i < nslots;
       c0i += (uint64_t)gridDim.x * kThreads) {
    const uint64_t i = c0i + threadIdx.x;
    bool take = false;
    uint64_t key = 0;
    uint32_t c0 = 0, c1 = 0;
    if (i < nslots && (live == nullptr || live[i / cap])) {
      key = tkeys[i];
      c0 = tcounts[i * nc];
      c1 = nc > 1 ? tcounts[i * nc + 1] : 0;
      take = key != kEmpty && (c0 | c1) != 0;
    }
    const uint64_t bal = __ballot(take);
    if (lane_id() == 0) wcnt[wave_id()] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = wcnt[w];
        wcnt[w] = tot;  // exclusive prefix over the waves
        tot += c;
      }
      wgbase = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(cursor),
                               (unsigned long long)tot)
                   : 0;
    }
    __syncthreads();
    if (take) {
      const uint64_t at =
          wgbase + wcnt[wave_id()] + __popcll(bal & ((1ull << lane_id()) - 1));
      if (at < out_cap) {  // past it the cursor still counts: the host sees the mismatch
        out_keys[at] = key;
        out_counts[at * nc] = c0;
        if (nc > 1) out_counts[at * nc + 1] = c1;
      }
    }
    __syncthreads();  // wcnt and wgbase are reused by the next chunk
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
    const uint32_t tt = sd.tile_first[c] + (uint32_t)(rel >> sd.t2_log2);
    const uint32_t o = (uint32_t)(rel & ((1ull << sd.t2_log2) - 1));
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

// slot_of[u] = u - first for partitions u >= first (their tables sit in HBM
// slots 0..), kNoSlot below (spilled to host memory).
__global__ void __launch_bounds__(256) k_slot_map(uint32_t* __restrict__ slot_of, uint32_t n,
                                                  uint32_t first) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) slot_of[u] = u >= first ? u - first : kNoSlot;
}

// out[rows[i] * nc + t] = vals[i * nc + t]: results of queries answered on the host.
__global__ void __launch_bounds__(256) k_scatter_rows(const uint32_t* __restrict__ rows,
                                                      const uint32_t* __restrict__ vals, uint32_t n,
                                                      uint32_t nc, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (uint32_t t = 0; t < nc; ++t) out[(uint64_t)rows[i] * nc + t] = vals[(uint64_t)i * nc + t];
}

// ------------------------------------------------------------ stem items

// Canonical stem of the table k-mer x (k >= 3, first base most significant):
// the middle k-2 bases S, or their reverse complement when that is smaller;
// *slot = 4a + b for the k-mer read as a S' b in the stem's orientation (for
// a palindromic stem, as x is written).
__device__ __forceinline__ uint64_t stem_of(uint64_t x, uint32_t k, uint32_t* slot) {
  const uint32_t m = k - 2;
  const uint64_t s = (x >> 2) & ((1ull << (2 * m)) - 1);
  // complement every base, reverse the 32 two-bit groups, keep the top m
  uint64_t u = ~s;
  u = ((u >> 2) & 0x3333333333333333ull) | ((u & 0x3333333333333333ull) << 2);
  u = ((u >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((u & 0x0F0F0F0F0F0F0F0Full) << 4);
  u = __builtin_bswap64(u);
  const uint64_t rs = u >> (64 - 2 * m);
  const uint32_t first = (uint32_t)(x >> (2 * (k - 1))) & 3u, last = (uint32_t)x & 3u;
  if (rs < s) {
    *slot = 4u * (3u - last) + (3u - first);
    return rs;
  }
  *slot = 4u * first + last;
  return s;
}

constexpr uint64_t kStemSalt = 0x2545F4914F6CDD1Dull;  // stem partition hash salt

// Slot i of a table pass (live[i / cap] gates the slots of resident tables;
// nullptr for the overflow table and staged spilled tables): false when it
// holds no k-mer with a count, else its canonical stem, the k-mer's place
// 4a + b in the stem's item (stem_of) and its two counts saturated to 16 bits
// (counter 0 low, counter 1 high).
__device__ __forceinline__ bool stem_entry(const uint64_t* __restrict__ tkeys,
                                           const uint32_t* __restrict__ tcounts,
                                           const uint32_t* __restrict__ live, uint64_t i,
                                           uint32_t cap, uint32_t nc, uint32_t k, uint64_t* stem,
                                           uint32_t* slot, uint32_t* c16) {
  if (live && !live[i / cap]) return false;
  const uint64_t key = tkeys[i];
  const uint32_t c0 = tcounts[i * nc], c1 = nc > 1 ? tcounts[i * nc + 1] : 0u;
  if (key == kEmpty || (c0 | c1) == 0) return false;
  *stem = stem_of(key, k, slot);
  *c16 = min(c0, 65535u) | (min(c1, 65535u) << 16);
  return true;
}

// Partition of a stem: the top p_log2 bits of its hash (0 when p_log2 = 0).
__device__ __forceinline__ uint64_t stem_part(uint64_t stem, uint32_t p_log2) {
  return p_log2 ? mix64(stem ^ kStemSalt) >> (64 - p_log2) : 0;
}

// First pass: entries per stem partition.
__global__ void __launch_bounds__(256) k_stem_count(const uint64_t* __restrict__ tkeys,
                                                    const uint32_t* __restrict__ tcounts,
                                                    uint64_t nslots,
                                                    const uint32_t* __restrict__ live,
                                                    uint32_t cap, uint32_t nc, uint32_t k,
                                                    uint32_t p_log2,
                                                    uint32_t* __restrict__ pcount) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t stem;
    uint32_t slot, c16;
    if (stem_entry(tkeys, tcounts, live, i, cap, nc, k, &stem, &slot, &c16))
      atomicAdd(&pcount[stem_part(stem, p_log2)], 1u);
  }
}

// Second pass: each entry appended to its partition's range as a record, the
// stem with the item place in bits 58-61 (stems have at most 58 bits) and
// the saturated counts beside it.
__global__ void __launch_bounds__(256) k_stem_scatter(const uint64_t* __restrict__ tkeys,
                                                      const uint32_t* __restrict__ tcounts,
                                                      uint64_t nslots,
                                                      const uint32_t* __restrict__ live,
                                                      uint32_t cap, uint32_t nc, uint32_t k,
                                                      uint32_t p_log2,
                                                      unsigned long long* __restrict__ cursor,
                                                      uint64_t* __restrict__ rstem,
                                                      uint32_t* __restrict__ rcnt) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t stem;
    uint32_t slot, c16;
    if (!stem_entry(tkeys, tcounts, live, i, cap, nc, k, &stem, &slot, &c16)) continue;
    const uint64_t at = atomicAdd(&cursor[stem_part(stem, p_log2)], 1ull);
    rstem[at] = stem | ((uint64_t)slot << 58);
    rcnt[at] = c16;
  }
}

constexpr uint32_t kStemTable = 4096;                      // LDS stem slots per partition
constexpr uint32_t kStemPartMax = kStemTable * 3 / 4;      // most entries a partition may hold
constexpr uint64_t kStemMask = (1ull << 58) - 1;

// Third pass, one workgroup per partition: the partition's stems are made
// distinct in an LDS table (linear probing, CAS) and numbered in slot order;
// the workgroup takes the next free range of items with one atomic add, writes
// each stem and zeroes its row, then each record stores its counts at its
// place in its stem's row (the rows of one partition span at most 256 KB, so
// these scattered stores stay in L2).  With count_only only the number of
// distinct stems is added to the cursor.
__global__ void __launch_bounds__(kThreads) k_stem_group(const uint64_t* __restrict__ poff,
                                                         const uint64_t* __restrict__ rstem,
                                                         const uint32_t* __restrict__ rcnt,
                                                         int count_only,
                                                         unsigned long long* __restrict__ cursor,
                                                         uint64_t capacity,
                                                         uint64_t* __restrict__ stems,
                                                         uint16_t* __restrict__ items,
                                                         uint32_t* __restrict__ err) {
  __shared__ uint64_t tab[kStemTable];
  __shared__ uint32_t idx[kStemTable + 1], scratch[kWaves + 1];
  __shared__ unsigned long long base_s;
  const uint64_t r0 = poff[blockIdx.x], r1 = poff[blockIdx.x + 1];
  if (r1 - r0 > kStemPartMax) {  // the host sizes partitions below this
    if (threadIdx.x == 0) atomicOr(err, 2u);
    return;
  }
  for (uint32_t i = threadIdx.x; i < kStemTable; i += kThreads) tab[i] = kEmpty;
  __syncthreads();
  auto find = [&](uint64_t stem, bool insert) -> int {
    uint32_t h = (uint32_t)(mix64(stem ^ kStemSalt) & (kStemTable - 1));
    for (uint32_t probe = 0; probe < kStemTable; ++probe) {
      uint64_t cur = tab[h];
      if (insert && cur == kEmpty) {
        cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[h]),
                        (unsigned long long)kEmpty, (unsigned long long)stem);
        if (cur == kEmpty) cur = stem;
      }
      if (cur == stem) return (int)h;
      if (!insert && cur == kEmpty) return -1;
      h = (h + 1) & (kStemTable - 1);
    }
    return -1;
  };
  for (uint64_t r = r0 + threadIdx.x; r < r1; r += kThreads)
    if (find(rstem[r] & kStemMask, true) < 0) atomicOr(err, 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kStemTable; i += kThreads) idx[i] = tab[i] != kEmpty;
  __syncthreads();
  block_exclusive_scan(idx, idx, kStemTable, scratch);  // in place: every read precedes its first barrier
  const uint32_t n = idx[kStemTable];
  if (threadIdx.x == 0) base_s = atomicAdd(cursor, (unsigned long long)n);
  __syncthreads();
  const uint64_t base = base_s;
  if (count_only || n == 0) return;
  if (base + n > capacity) {
    if (threadIdx.x == 0) atomicOr(err, 4u);
    return;
  }
  for (uint32_t i = threadIdx.x; i < kStemTable; i += kThreads)
    if (tab[i] != kEmpty) stems[base + idx[i]] = tab[i];
  uint32_t* rows = reinterpret_cast<uint32_t*>(items + base * 32);
  for (uint64_t i = threadIdx.x; i < (uint64_t)n * 16; i += kThreads) rows[i] = 0;
  __syncthreads();
  for (uint64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
    const uint64_t v = rstem[r];
    const int h = find(v & kStemMask, false);
    if (h < 0) continue;  // reported by the insert loop
    const uint32_t slot = (uint32_t)(v >> 58) & 15u, c = rcnt[r];
    uint16_t* row = items + (base + idx[h]) * 32;
    row[slot] = (uint16_t)(c & 0xFFFFu);
    row[16 + slot] = (uint16_t)(c >> 16);
  }
}

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- launchers

// Lets a kernel take up to the whole LDS of a CU in dynamic shared memory.
// Always the same value, so contexts launching from several threads cannot
// race each other into a smaller limit than one of their launches needs.
static hipError_t allow_lds(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
}

hipError_t launch_pack(const uint8_t* bases, uint64_t total, uint64_t nwords, uint64_t* packed,
                       uint64_t* flags, hipStream_t s) {
  if (!nwords) return hipSuccess;
  const int aligned = ((uintptr_t)bases & 15) == 0;
  hipLaunchKernelGGL(k_pack, dim3(div_up(2 * nwords, 256)), dim3(256), 0, s, bases, total, nwords,
                     packed, flags, aligned);
  return hipGetLastError();
}

hipError_t launch_rstart(const uint64_t* offsets, uint64_t n_reads, uint64_t total,
                         uint64_t* flags, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_rstart, dim3(div_up(n_reads + 1, 256)), dim3(256), 0, s, offsets, n_reads,
                     total, flags, err);
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

size_t level1_lds(uint32_t a1) {
  const uint32_t nb = 1u << a1;
  return (size_t)kTilePos * 8 + (size_t)nb * 4 + (size_t)(nb + 1) * 4 + kWaves * 4;
}

size_t level2_lds(uint32_t a2, uint32_t t2_log2) {
  const size_t nb = (size_t)1 << a2;
  return ((size_t)8 << t2_log2) + 4 * std::max<size_t>((size_t)kThreads * 3, 2 * nb + 2 + kWaves) + 4;
}

hipError_t launch_level1(const uint64_t* packed, const uint64_t* flags, uint64_t nwords,
                         uint32_t k, uint64_t s0, uint32_t a1, uint64_t tag, uint32_t* hist,
                         uint32_t* lstart, uint64_t ntiles, uint64_t* out, hipStream_t s) {
  if (!ntiles) return hipSuccess;
  const size_t lds = level1_lds(a1);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_level1));
  if (e != hipSuccess) return e;
  const uint64_t grid = (ntiles + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(k_level1, dim3((uint32_t)grid), dim3(kThreads), lds, s, packed, flags,
                     nwords, k, s0, a1, tag, hist, lstart, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_tiles2(const uint64_t* bucket_off, uint32_t nb1, uint32_t t2_log2,
                         uint32_t* tile_first, hipStream_t s) {
  if (t2_log2 < kT2MinLog2 || (1u << t2_log2) > (uint32_t)kT2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tiles2, dim3(1), dim3(kThreads), 0, s, bucket_off, nb1, t2_log2,
                     tile_first);
  return hipGetLastError();
}

hipError_t launch_level2(const uint64_t* keys1, const uint64_t* off1, const uint32_t* lstart,
                         uint64_t ntiles1, const uint64_t* bucket_off, const uint32_t* tile_first,
                         uint64_t* tile_desc, uint32_t a1, uint32_t a2, uint32_t t2_log2,
                         uint64_t s0, uint64_t* keys2, uint32_t* meta2, uint64_t grid,
                         hipStream_t s) {
  if (!grid) return hipSuccess;
  if (t2_log2 < kT2MinLog2 || (1u << t2_log2) > (uint32_t)kT2) return hipErrorInvalidValue;
  // one descriptor per workgroup (tile_desc holds level2_grid(grid)); tiles,
  // buckets and first-level tiles must fit their fields (20, 10 and 34 bits;
  // never all ones)
  const uint64_t grid8 = level2_grid(grid);
  if (grid8 > (1u << 20) || a1 > 10 || ntiles1 >= (1ull << 33)) return hipErrorInvalidValue;
  uint64_t* order = tile_desc;
  hipError_t e = launch_fill64(order, grid8, kEmpty, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_desc, dim3(div_up(grid, 256)), dim3(256), 0, s, off1, ntiles1,
                     bucket_off, tile_first, 1u << a1, (uint32_t)grid8, t2_log2, order);
  const size_t lds = level2_lds(a2, t2_log2);
  e = allow_lds(reinterpret_cast<const void*>(k_level2));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_level2, dim3((uint32_t)grid8), dim3(kThreads), lds, s, keys1, off1, lstart,
                     ntiles1, bucket_off, tile_first, order, a1, a2, t2_log2, s0, keys2, meta2);
  return hipGetLastError();
}

template <int H, bool FLAT, int SUBL>
hipError_t launch_bloom_v(const CountArgs& a, uint32_t blocks, size_t lds, hipStream_t s) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_bloom<H, FLAT, SUBL>));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_bloom<H, FLAT, SUBL>), dim3(blocks >> SUBL), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int H>
hipError_t launch_bloom_h(const CountArgs& a, uint32_t blocks, size_t lds, hipStream_t s) {
  // 2^bsub_log2 blocks per workgroup (their partitions lie in one first-level
  // bucket); the flattened walk when a workgroup's blocks hold at most two
  // partitions
  switch (a.bsub_log2) {
    case 1: return launch_bloom_v<H, false, 1>(a, blocks, lds, s);
    case 2: return launch_bloom_v<H, false, 2>(a, blocks, lds, s);
    default:
      return a.upb_log2 <= 1 ? launch_bloom_v<H, true, 0>(a, blocks, lds, s)
                             : launch_bloom_v<H, false, 0>(a, blocks, lds, s);
  }
}

template <int H>
hipError_t launch_tally_h(const CountArgs& a, uint32_t parts, size_t lds, hipStream_t s) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(k_tally<H>));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tally<H>, dim3(parts), dim3(kTallyThreads), lds, s, a);
  return hipGetLastError();
}

#define KC_DISPATCH_H(fn, ...)                     \
  switch (a.hc.h) {                                \
    case 1: return fn<1>(__VA_ARGS__);             \
    case 2: return fn<2>(__VA_ARGS__);             \
    case 3: return fn<3>(__VA_ARGS__);             \
    case 4: return fn<4>(__VA_ARGS__);             \
    case 5: return fn<5>(__VA_ARGS__);             \
    case 6: return fn<6>(__VA_ARGS__);             \
    case 7: return fn<7>(__VA_ARGS__);             \
    case 8: return fn<8>(__VA_ARGS__);             \
  }                                                \
  return hipErrorInvalidValue;

hipError_t launch_bloom(const CountArgs& a, uint32_t blocks, size_t lds, hipStream_t s) {
  KC_DISPATCH_H(launch_bloom_h, a, blocks, lds, s)
}

hipError_t launch_tally(const CountArgs& a, uint32_t parts, size_t lds, hipStream_t s) {
  KC_DISPATCH_H(launch_tally_h, a, parts, lds, s)
}

int tally_threads() { return kTallyThreads; }

hipError_t launch_ovf_emit(const CountArgs& a, uint64_t* pstats_ovf, uint32_t blocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_ovf_emit, dim3(blocks), dim3(256), 0, s, a, pstats_ovf);
  return hipGetLastError();
}

hipError_t launch_reduce(const uint64_t* rows, uint64_t nrows, uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fill64, dim3(1), dim3(256), 0, s, out, (uint64_t)kNst, (uint64_t)0);
  const uint64_t grid = std::min<uint64_t>(256, std::max<uint64_t>(1, div_up(nrows, (uint64_t)kThreads * 4)));
  hipLaunchKernelGGL(k_reduce, dim3((uint32_t)grid), dim3(kThreads), 0, s, rows, nrows, out);
  return hipGetLastError();
}

hipError_t launch_query(const QueryArgs& a, const uint64_t* kmers, uint64_t n, uint32_t* out,
                        hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_query, dim3(div_up(n, 256)), dim3(256), 0, s, a, kmers, n, out);
  return hipGetLastError();
}

hipError_t launch_export(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                         const uint32_t* live, uint32_t cap, uint32_t nc,
                         uint64_t* out_keys, uint32_t* out_counts, uint64_t out_cap,
                         uint64_t* cursor, hipStream_t s) {
  if (!nslots) return hipSuccess;
  const uint64_t grid = std::min<uint64_t>(4096, div_up(nslots, kThreads));
  hipLaunchKernelGGL(k_export, dim3((uint32_t)grid), dim3(kThreads), 0, s, tkeys, tcounts, nslots,
                     live, cap, nc, out_keys, out_counts, out_cap, cursor);
  return hipGetLastError();
}

hipError_t launch_debug_part(const SegDesc& sd, uint64_t n, uint32_t* part, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_debug_part, dim3(div_up(n, 256)), dim3(256), 0, s, sd, n, part);
  return hipGetLastError();
}

// grid-stride launches: enough workgroups to fill the chip, at most one per 256 items
static uint32_t stride_grid(uint64_t n) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(n, 256), 8192));
}

// A thread per item (up to 2^30 threads; kernels still stride past that):
// for kernels whose items each wait on a global atomic, which a hundred items
// per thread would serialise (the stem passes: 14.2 -> 12.4 ms at 2.5e8 slots).
static uint32_t wide_grid(uint64_t n) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(n, 256), 1u << 22));
}

hipError_t launch_stem_count(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                             const uint32_t* live, uint32_t cap, uint32_t nc, uint32_t k,
                             uint32_t p_log2, uint32_t* pcount, hipStream_t s) {
  if (!nslots) return hipSuccess;
  hipLaunchKernelGGL(k_stem_count, dim3(wide_grid(nslots)), dim3(256), 0, s, tkeys, tcounts,
                     nslots, live, cap, nc, k, p_log2, pcount);
  return hipGetLastError();
}

hipError_t launch_stem_scatter(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                               const uint32_t* live, uint32_t cap, uint32_t nc, uint32_t k,
                               uint32_t p_log2, uint64_t* cursor, uint64_t* rstem, uint32_t* rcnt,
                               hipStream_t s) {
  if (!nslots) return hipSuccess;
  hipLaunchKernelGGL(k_stem_scatter, dim3(wide_grid(nslots)), dim3(256), 0, s, tkeys, tcounts,
                     nslots, live, cap, nc, k, p_log2,
                     reinterpret_cast<unsigned long long*>(cursor), rstem, rcnt);
  return hipGetLastError();
}

uint32_t stem_part_max() { return kStemPartMax; }

hipError_t launch_stem_group(const uint64_t* poff, uint64_t nparts, const uint64_t* rstem,
                             const uint32_t* rcnt, bool count_only, uint64_t* cursor,
                             uint64_t capacity, uint64_t* stems, uint16_t* items, uint32_t* err,
                             hipStream_t s) {
  if (!nparts) return hipSuccess;
  if (nparts > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stem_group, dim3((uint32_t)nparts), dim3(kThreads), 0, s, poff, rstem, rcnt,
                     count_only ? 1 : 0, reinterpret_cast<unsigned long long*>(cursor), capacity,
                     stems, items, err);
  return hipGetLastError();
}

hipError_t launch_filter_keys(const uint64_t* tkeys, const uint32_t* tcounts, uint64_t nslots,
                              uint32_t nc, uint32_t tmin, uint32_t nmax, uint64_t* fkeys,
                              hipStream_t s) {
  if (!nslots) return hipSuccess;
  hipLaunchKernelGGL(k_filter_keys, dim3(stride_grid(nslots)), dim3(256), 0, s, tkeys, tcounts,
                     nslots, nc, tmin, nmax, fkeys);
  return hipGetLastError();
}

hipError_t launch_filter(const QueryArgs& a, const uint64_t* packed, const uint64_t* flags,
                         uint64_t nwords, const uint64_t* offsets, uint64_t n_reads, uint64_t total,
                         uint32_t tmin, uint32_t nmax, uint32_t* hit, uint32_t* out, hipStream_t s) {
  if (nwords)
    hipLaunchKernelGGL(k_filter_windows, dim3(div_up(nwords * 4, 256)), dim3(256), 0, s, a, packed,
                       flags, nwords, tmin, nmax, hit);
  if (n_reads)
    hipLaunchKernelGGL(k_filter_reads, dim3(div_up(n_reads, 256)), dim3(256), 0, s, offsets,
                       n_reads, total, hit, out);
  return hipGetLastError();
}

hipError_t launch_pack_batch(const ChunkDesc* cd, uint32_t nchunks, uint64_t nwords,
                             uint64_t* packed, uint64_t* flags, hipStream_t s) {
  if (!nwords || !nchunks) return hipSuccess;
  hipLaunchKernelGGL(k_pack_batch, dim3(stride_grid(2 * nwords)), dim3(256), 0, s, cd, nchunks,
                     nwords, packed, flags);
  return hipGetLastError();
}

hipError_t launch_rstart_batch(const ChunkDesc* cd, uint32_t nchunks, uint64_t nslots,
                               uint64_t* flags, uint32_t* err, hipStream_t s) {
  if (!nslots || !nchunks) return hipSuccess;
  hipLaunchKernelGGL(k_rstart_batch, dim3(stride_grid(nslots)), dim3(256), 0, s, cd, nchunks,
                     nslots, flags, err);
  return hipGetLastError();
}

hipError_t launch_fill64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill64, dim3(stride_grid(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill32, dim3(stride_grid(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_gather2(const uint64_t* a, const uint64_t* b, const uint64_t* idx, uint64_t n,
                          uint64_t nwords, uint64_t* out_a, uint64_t* out_b, uint32_t* err,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_gather2, dim3((uint32_t)blocks), dim3(256), 0, s, a, b, idx, n, nwords,
                     out_a, out_b, err);
  return hipGetLastError();
}

hipError_t launch_copy64(const uint64_t* src, uint64_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy64, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_slot_map(uint32_t* slot_of, uint32_t n, uint32_t first, hipStream_t s) {
  hipLaunchKernelGGL(k_slot_map, dim3(div_up(n, 256)), dim3(256), 0, s, slot_of, n, first);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const uint32_t* rows, const uint32_t* vals, uint32_t n,
                               uint32_t nc, uint32_t* out, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3(div_up(n, 256)), dim3(256), 0, s, rows, vals, n, nc, out);
  return hipGetLastError();
}

}  // namespace kc
