// Streaming-ceiling kernels of this GPU (measurement helpers behind
// include/lbm_probe.h).  They move the same kind of data as one step of the
// D3Q19 solver - A arrays of n floats read and/or written, a block covering
// one contiguous run of every array - with nothing else in the way, so the
// benchmark can report how close the step comes to what plain streaming
// reaches on the same GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_probe.h"

namespace {

constexpr int kThreads = 256;

template <int VEC>
struct Vec;
template <>
struct Vec<1> {
  using T = float;
  __device__ static float sum(float v) { return v; }
  __device__ static float make(float x) { return x; }
};
typedef float f4 __attribute__((ext_vector_type(4)));
template <>
struct Vec<4> {
  using T = f4;
  __device__ static float sum(f4 v) { return (v.x + v.y) + (v.z + v.w); }
  __device__ static f4 make(float x) { return f4{x, x, x, x}; }
};

template <class V, bool NT>
__device__ __forceinline__ void put(V* p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// MODE 0: dst = src; 1: read src only; 2: write dst only.  Block b covers
// elements [b * 256 VEC, (b + 1) * 256 VEC) of each of the A arrays; n is a
// multiple of 256 VEC (the host checks).  All A loads of a thread are issued
// before its stores, as in the step kernel.
template <int A, int VEC, bool NT, int MODE>
__global__ __launch_bounds__(kThreads) void k_stream(const float* __restrict__ src,
                                                     float* __restrict__ dst,
                                                     float* __restrict__ sink, uint64_t n) {
  using V = typename Vec<VEC>::T;
  const uint64_t base = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;
  V v[A];
  if constexpr (MODE != 2) {
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = *(const V*)(src + (uint64_t)a * n + base);
  } else {
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = Vec<VEC>::make((float)a);
  }
  if constexpr (MODE == 1) {
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < A; ++a) acc += Vec<VEC>::sum(v[a]);
    if (acc == 1.5e30f) sink[0] = acc;   // keeps the loads; never true for finite data
  } else {
#pragma unroll
    for (int a = 0; a < A; ++a) put<V, NT>((V*)(dst + (uint64_t)a * n + base), v[a]);
  }
}

template <int A, int VEC, bool NT>
hipError_t launch(int mode, const float* src, float* dst, float* sink, uint64_t n, hipStream_t st) {
  const unsigned grid = (unsigned)(n / ((uint64_t)kThreads * VEC));
  if (mode == 0) k_stream<A, VEC, NT, 0><<<grid, kThreads, 0, st>>>(src, dst, sink, n);
  else if (mode == 1) k_stream<A, VEC, NT, 1><<<grid, kThreads, 0, st>>>(src, dst, sink, n);
  else k_stream<A, VEC, NT, 2><<<grid, kThreads, 0, st>>>(src, dst, sink, n);
  return hipGetLastError();
}

template <int A>
hipError_t launch_a(int mode, int vec, int nt, const float* s, float* d, float* k, uint64_t n,
                    hipStream_t st) {
  if (vec == 1) return nt ? launch<A, 1, true>(mode, s, d, k, n, st) : launch<A, 1, false>(mode, s, d, k, n, st);
  return nt ? launch<A, 4, true>(mode, s, d, k, n, st) : launch<A, 4, false>(mode, s, d, k, n, st);
}

}  // namespace

extern "C" int lbm_probe_stream(int mode, int vec, int nontemporal, int arrays, uint64_t n,
                                const void* src, void* dst, void* sink, void* stream) {
  if (mode < 0 || mode > 2 || (vec != 1 && vec != 4) || (arrays != 9 && arrays != 19)) return -1;
  if (n == 0 || n % ((uint64_t)kThreads * vec) != 0 || n / ((uint64_t)kThreads * vec) >= (1ull << 31))
    return -1;
  if ((mode != 2 && !src) || (mode != 1 && !dst) || (mode == 1 && !sink)) return -1;
  if ((((uintptr_t)src | (uintptr_t)dst) & 15) != 0) return -1;
  hipStream_t st = (hipStream_t)stream;
  const float* s = (const float*)src;
  float* d = (float*)dst;
  float* k = (float*)sink;
  const hipError_t e = arrays == 19 ? launch_a<19>(mode, vec, nontemporal, s, d, k, n, st)
                                    : launch_a<9>(mode, vec, nontemporal, s, d, k, n, st);
  return e == hipSuccess ? 0 : -2;
}
