/*
 * lbm_probe.h - streaming-ceiling kernels (measurement helpers, not part of
 * the method): what plain streaming of the step's kind of data reaches on
 * this GPU, for the benchmark to report beside the step kernel's rate.
 * Library: liblbmprobe.so.
 */
#ifndef LBM_PROBE_H_
#define LBM_PROBE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueues one pass over `arrays` (9 or 19, the populations of D2Q9 or
 * D3Q19) device arrays of n floats each, array a at
 * element offset a * n of src / dst (so a single allocation of arrays * n
 * floats), on the HIP stream `stream` (NULL: the legacy default stream); a
 * thread issues all its loads before its stores, as the step kernel does:
 *   mode 0  dst = src   (every element read once and written once)
 *   mode 1  read src    (sink, one float, is written only if the data sum to
 *                        1.5e30, i.e. never for finite data)
 *   mode 2  write dst   (every element written once)
 * Every lane moves `vec` consecutive floats per access (1: 4-byte accesses,
 * as the step kernel's gathers and stores; 4: 16-byte accesses); a block of
 * 256 threads covers one run of 256 * vec elements of every array.
 * nontemporal != 0 makes the stores bypass the caches (as the step kernel's
 * whole-line stores do).  Buffers are the caller's and 16-byte aligned; n must
 * be a positive multiple of 256 * vec.  Returns 0, -1 for an invalid argument
 * (nothing enqueued), -2 if the launch failed. */
int lbm_probe_stream(int mode, int vec, int nontemporal, int arrays, uint64_t n,
                     const void *src, void *dst, void *sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_PROBE_H_ */
