/* kc_probe.h - LDS atomic throughput microbenchmark (libkc_probe.so).
 *
 * Measurement support, not part of the counting ABI in kc.h: it gives the
 * peak rate of the LDS atomics the Bloom pass (a bitwise OR that returns the
 * old word) and the count pass (an add) are made of, under the same access
 * pattern (uniformly random words of a block-sized LDS array, 1024-thread
 * workgroups), so that their achieved rates can be quoted as a fraction of it.
 */
#ifndef KC_PROBE_H
#define KC_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kcp_kind {
  KCP_OR = 0,      /* atomicOr, result unused */
  KCP_OR_RTN = 1,  /* atomicOr, old word used */
  KCP_ADD = 2      /* atomicAdd of 1 */
} kcp_kind;

/* Runs `blocks` workgroups of 1024 threads on the current device, each
 * thread doing iters * 8 atomics of `kind` on uniformly random words of a
 * zeroed LDS array of 2^words_log2 32-bit words (6..15), and times the launch
 * with HIP events on a stream of its own.  *ms_out receives the kernel time.
 * *check_out receives the sum over workgroups of the array's words after the
 * run; for KCP_ADD it equals blocks * 1024 * iters * 8.  Device memory for the
 * per-workgroup sums is allocated and freed inside the call.
 * Returns 0 on success, -1 for an argument out of range, -2 for a HIP error. */
int kcp_lds_atomics(int kind, uint32_t words_log2, uint32_t iters, uint32_t blocks,
                    float* ms_out, uint64_t* check_out);

#ifdef __cplusplus
}
#endif

#endif /* KC_PROBE_H */
