// kc_probe.hip - LDS atomic throughput microbenchmark (see kc_probe.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_probe.h"

namespace {

constexpr int kProbeThreads = 1024;

// Each thread draws word indices and bit positions from its own xorshift32
// stream (nonzero seed), eight atomics per iteration.  The sum of the array's
// words leaves through one vector store per workgroup.
template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) k_lds_atomics(uint32_t words_log2, uint32_t iters,
                                                                uint64_t* __restrict__ sums) {
  extern __shared__ uint32_t w[];
  __shared__ uint64_t part[kProbeThreads / 64];
  const uint32_t n = 1u << words_log2;
  for (uint32_t i = threadIdx.x; i < n; i += kProbeThreads) w[i] = 0;
  __syncthreads();
  uint32_t x = (blockIdx.x * kProbeThreads + threadIdx.x + 1) * 0x9E3779B9u;
  if (x == 0) x = 1;
  uint32_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      const uint32_t a = x & (n - 1);
      if (KIND == KCP_OR) {
        atomicOr(&w[a], 1u << (x >> 27));
      } else if (KIND == KCP_OR_RTN) {
        acc += atomicOr(&w[a], 1u << (x >> 27)) & 1u;
      } else {
        atomicAdd(&w[a], 1u);
      }
    }
  }
  __syncthreads();
  uint64_t s = 0;
  for (uint32_t i = threadIdx.x; i < n; i += kProbeThreads) s += w[i];
  // keeps the returned words live (never true: acc <= iters * 8 < 2^32 - 1)
  if (KIND == KCP_OR_RTN && acc == 0xFFFFFFFFu) s += 1;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < kProbeThreads / 64; ++i) t += part[i];
    sums[blockIdx.x] = t;
  }
}

template <int KIND>
hipError_t launch(uint32_t words_log2, uint32_t iters, uint32_t blocks, uint64_t* sums,
                  hipStream_t s) {
  const size_t lds = (size_t)4 << words_log2;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_lds_atomics<KIND>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lds_atomics<KIND>, dim3(blocks), dim3(kProbeThreads), lds, s, words_log2,
                     iters, sums);
  return hipGetLastError();
}

}  // namespace

extern "C" int kcp_lds_atomics(int kind, uint32_t words_log2, uint32_t iters, uint32_t blocks,
                               float* ms_out, uint64_t* check_out) {
  if (kind < KCP_OR || kind > KCP_ADD || words_log2 < 6 || words_log2 > 15 || iters < 1 ||
      iters > (1u << 20) || blocks < 1 || blocks > (1u << 20) || !ms_out || !check_out)
    return -1;
  uint64_t* sums = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -2;
  hipError_t e = hipMalloc(&sums, (size_t)blocks * 8);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) {
    if (kind == KCP_OR) e = launch<KCP_OR>(words_log2, iters, blocks, sums, s);
    else if (kind == KCP_OR_RTN) e = launch<KCP_OR_RTN>(words_log2, iters, blocks, sums, s);
    else e = launch<KCP_ADD>(words_log2, iters, blocks, sums, s);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
  if (e == hipSuccess) {
    uint64_t* host = new uint64_t[blocks];
    e = hipMemcpy(host, sums, (size_t)blocks * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      uint64_t t = 0;
      for (uint32_t i = 0; i < blocks; ++i) t += host[i];
      *check_out = t;
      rc = 0;
    }
    delete[] host;
  }
  if (e1) (void)hipEventDestroy(e1);
  if (e0) (void)hipEventDestroy(e0);
  if (s) (void)hipStreamDestroy(s);
  if (sums) (void)hipFree(sums);
  if (rc != 0) (void)hipGetLastError();
  return rc;
}
