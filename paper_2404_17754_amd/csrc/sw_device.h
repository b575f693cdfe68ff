// Device helpers shared by the kernel sources: 64-wide wavefront and
// workgroup reductions, hardware floating-point atomics, grid sizing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

constexpr int TPB = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over a TPB-thread workgroup, valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) t += sh[i];
  }
  return t;
}

// Sum of v over an NT-thread workgroup (sh holds NT / 64 doubles), valid on
// thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
  }
  return t;
}

// Two sums at once (sh holds 2 * TPB / 64 doubles), valid on thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid] = a;
    sh[TPB / 64 + wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) {
      a += sh[i];
      b += sh[TPB / 64 + i];
    }
  }
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

static inline unsigned nblocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

// Total of N partial sums written by earlier kernels (same address for every
// thread).
template <int N>
__device__ __forceinline__ double slot_sum(const double* s) {
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) t += s[i];
  return t;
}

}  // namespace sw
