// Projection initial guess (gfx950): the step's solution is approximated by
// its Galerkin projection onto the span of the last L increments,
//   x0 = X theta,  (X^T A X) theta = X^T b,
// the combination of past increments closest to the new one in the energy
// norm (projection for successive right-hand sides, P. F. Fischer, Comput.
// Methods Appl. Mech. Engrg. 163 (1998) 193-204).  The images A X are not
// recomputed: each increment x of a converged step comes with A x = b - r,
// its right-hand side minus its final true residual.  The device does the
// long dot products and combinations; the host solves the L x L system.
//
// Vectors are FP64, [slot][n] for the ring X and its images Y.  Dot
// products are reduced per workgroup into a partial array and then summed
// in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// part[blk * L + i] = sum over the workgroup's entries of R_i[k] (v[k] - w[k])
// (w optional), R = ring of L vectors of length n.
template <int L>
__global__ __launch_bounds__(TPB) void k_proj_dots(int64_t n, const double* __restrict__ R,
                                                   const double* __restrict__ v, const double* __restrict__ w,
                                                   double* __restrict__ part) {
  __shared__ double sh[L][TPB / 64];
  double acc[L];
#pragma unroll
  for (int i = 0; i < L; ++i) acc[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) {
    const double t = w ? v[k] - w[k] : v[k];
#pragma unroll
    for (int i = 0; i < L; ++i) acc[i] += R[(int64_t)i * n + k] * t;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const double s = wave_sum(acc[i]);
    if (lane == 0) sh[i][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < L) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < TPB / 64; ++j) s += sh[threadIdx.x][j];
    part[(int64_t)blockIdx.x * L + threadIdx.x] = s;
  }
}

// The same for two right-hand vectors in one pass over the ring:
// part[blk * 2L + i] from v1, part[blk * 2L + L + i] from v2.
template <int L>
__global__ __launch_bounds__(TPB) void k_proj_dots2(int64_t n, const double* __restrict__ R,
                                                    const double* __restrict__ v1, const double* __restrict__ v2,
                                                    double* __restrict__ part) {
  __shared__ double sh[2 * L][TPB / 64];
  double a1[L], a2[L];
#pragma unroll
  for (int i = 0; i < L; ++i) a1[i] = a2[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) {
    const double t1 = v1[k], t2 = v2[k];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const double x = R[(int64_t)i * n + k];
      a1[i] += x * t1;
      a2[i] += x * t2;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const double s1 = wave_sum(a1[i]), s2 = wave_sum(a2[i]);
    if (lane == 0) {
      sh[i][wid] = s1;
      sh[L + i][wid] = s2;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * L) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < TPB / 64; ++j) s += sh[threadIdx.x][j];
    part[(int64_t)blockIdx.x * 2 * L + threadIdx.x] = s;
  }
}

// out[i] = sum_b part[b * L + i], one workgroup, fixed order
__global__ __launch_bounds__(TPB) void k_proj_reduce(int nb, int L, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  __shared__ double sh[TPB / 64];
  for (int i = 0; i < L; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += TPB) s += part[(int64_t)b * L + i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[i] = s;
    __syncthreads();
  }
}

// x = sum_i theta[i] X_i
template <int L>
__global__ __launch_bounds__(TPB) void k_proj_combine(int64_t n, const double* __restrict__ X,
                                                      const double* __restrict__ theta, double* __restrict__ x) {
  double th[L];
#pragma unroll
  for (int i = 0; i < L; ++i) th[i] = theta[i];
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) s += th[i] * X[(int64_t)i * n + k];
    x[k] = s;
  }
}

// x = sum_i theta[i] X_i and its residual r = b - sum_i theta[i] Y_i (the
// images Y_i = A X_i are exact, so no operator pass is needed); workgroup
// partials of r.r into part[blk]
template <int L>
__global__ __launch_bounds__(TPB) void k_proj_combine_res(int64_t n, const double* __restrict__ X,
                                                          const double* __restrict__ Y,
                                                          const double* __restrict__ theta,
                                                          const double* __restrict__ b, double* __restrict__ x,
                                                          double* __restrict__ r, double* __restrict__ part) {
  __shared__ double sh[TPB / 64];
  double th[L];
#pragma unroll
  for (int i = 0; i < L; ++i) th[i] = theta[i];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      sx += th[i] * X[(int64_t)i * n + k];
      sy += th[i] * Y[(int64_t)i * n + k];
    }
    x[k] = sx;
    const double t = b[k] - sy;
    r[k] = t;
    acc += t * t;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// X_slot = x, Y_slot = b - r
__global__ __launch_bounds__(TPB) void k_proj_store(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ b, const double* __restrict__ r,
                                                    double* __restrict__ Xs, double* __restrict__ Ys) {
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) {
    Xs[k] = x[k];
    Ys[k] = b[k] - r[k];
  }
}

static unsigned proj_grid(int64_t n) {
  unsigned g = nblocks(n);
  return g > PROJ_BLOCKS ? PROJ_BLOCKS : (g == 0 ? 1 : g);
}

void launch_proj_dots(int L, int64_t n, const double* R, const double* v, const double* w, double* part,
                      double* out, hipStream_t s) {
  const unsigned g = proj_grid(n);
  switch (L) {
#define SW_PROJ_CASE(K)                                                                          \
  case K:                                                                                        \
    hipLaunchKernelGGL(k_proj_dots<K>, dim3(g), dim3(TPB), 0, s, n, R, v, w, part);              \
    break;
    SW_PROJ_CASE(2) SW_PROJ_CASE(3) SW_PROJ_CASE(4) SW_PROJ_CASE(5) SW_PROJ_CASE(6) SW_PROJ_CASE(7)
    SW_PROJ_CASE(8) SW_PROJ_CASE(9) SW_PROJ_CASE(10) SW_PROJ_CASE(11) SW_PROJ_CASE(12) SW_PROJ_CASE(13)
    SW_PROJ_CASE(14) SW_PROJ_CASE(15) SW_PROJ_CASE(16)
#undef SW_PROJ_CASE
    default:
      return;
  }
  hipLaunchKernelGGL(k_proj_reduce, dim3(1), dim3(TPB), 0, s, (int)g, L, part, out);
}

void launch_proj_dots2(int L, int64_t n, const double* R, const double* v1, const double* v2, double* part,
                       double* out, hipStream_t s) {
  const unsigned g = proj_grid(n);
  switch (L) {
#define SW_PROJ_CASE(K)                                                                          \
  case K:                                                                                        \
    hipLaunchKernelGGL(k_proj_dots2<K>, dim3(g), dim3(TPB), 0, s, n, R, v1, v2, part);           \
    break;
    SW_PROJ_CASE(2) SW_PROJ_CASE(3) SW_PROJ_CASE(4) SW_PROJ_CASE(5) SW_PROJ_CASE(6) SW_PROJ_CASE(7)
    SW_PROJ_CASE(8) SW_PROJ_CASE(9) SW_PROJ_CASE(10) SW_PROJ_CASE(11) SW_PROJ_CASE(12) SW_PROJ_CASE(13)
    SW_PROJ_CASE(14) SW_PROJ_CASE(15) SW_PROJ_CASE(16)
#undef SW_PROJ_CASE
    default:
      return;
  }
  hipLaunchKernelGGL(k_proj_reduce, dim3(1), dim3(TPB), 0, s, (int)g, 2 * L, part, out);
}

void launch_proj_combine(int L, int64_t n, const double* X, const double* theta, double* x, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  switch (L) {
#define SW_PROJ_CASE(K)                                                                 \
  case K:                                                                               \
    hipLaunchKernelGGL(k_proj_combine<K>, dim3(g), dim3(TPB), 0, s, n, X, theta, x);   \
    break;
    SW_PROJ_CASE(2) SW_PROJ_CASE(3) SW_PROJ_CASE(4) SW_PROJ_CASE(5) SW_PROJ_CASE(6) SW_PROJ_CASE(7)
    SW_PROJ_CASE(8) SW_PROJ_CASE(9) SW_PROJ_CASE(10) SW_PROJ_CASE(11) SW_PROJ_CASE(12) SW_PROJ_CASE(13)
    SW_PROJ_CASE(14) SW_PROJ_CASE(15) SW_PROJ_CASE(16)
#undef SW_PROJ_CASE
    default:
      return;
  }
}

void launch_proj_combine_res(int L, int64_t n, const double* X, const double* Y, const double* theta,
                             const double* b, double* x, double* r, double* part, double* rr_out, hipStream_t s) {
  const unsigned g = proj_grid(n);
  switch (L) {
#define SW_PROJ_CASE(K)                                                                                  \
  case K:                                                                                                \
    hipLaunchKernelGGL(k_proj_combine_res<K>, dim3(g), dim3(TPB), 0, s, n, X, Y, theta, b, x, r, part); \
    break;
    SW_PROJ_CASE(2) SW_PROJ_CASE(3) SW_PROJ_CASE(4) SW_PROJ_CASE(5) SW_PROJ_CASE(6) SW_PROJ_CASE(7)
    SW_PROJ_CASE(8) SW_PROJ_CASE(9) SW_PROJ_CASE(10) SW_PROJ_CASE(11) SW_PROJ_CASE(12) SW_PROJ_CASE(13)
    SW_PROJ_CASE(14) SW_PROJ_CASE(15) SW_PROJ_CASE(16)
#undef SW_PROJ_CASE
    default:
      return;
  }
  hipLaunchKernelGGL(k_proj_reduce, dim3(1), dim3(TPB), 0, s, (int)g, 1, part, rr_out);
}

void launch_proj_store(int64_t n, const double* x, const double* b, const double* r, double* Xs, double* Ys,
                       hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_proj_store, dim3(g), dim3(TPB), 0, s, n, x, b, r, Xs, Ys);
}

}  // namespace sw
