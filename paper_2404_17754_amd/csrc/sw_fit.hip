// Input estimation of Section 2 on the GPU (gfx950): the records' side of
// the least-squares problem.
//
// The input along j is sum_l c_jl p(t - l dT), dT = m time steps; the
// response is U_i^k(t) = sum_{j,l} G_ij^k(t - l m) c_jl with G_j the Green's
// records (velocity along i at receiver k for the unit impulse along j).
// With the record cut into nb = n_steps / m blocks of m steps, every entry
// of the normal equations is a sum of block inner products
//     C[(j,b), (j',b')] = sum_{k,i} w_ki sum_{r<m} G_j[b m + r] G_j'[b' m + r]
// (and the same with the observed record in place of G_j'), so one weighted
// Gram matrix of 4 nb block columns (3 nb of Green's blocks, nb of observed
// blocks) holds all of them; the host sums its diagonals into A and b.
#include <hip/hip_runtime.h>

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// o2[pair] = sum_t obs[t][pair]^2, one workgroup per (receiver, component)
__global__ __launch_bounds__(TPB) void k_fit_pair_norms(int n_pairs, int64_t n_steps, const double* __restrict__ obs,
                                                        double* __restrict__ o2) {
  __shared__ double sh[TPB / 64];
  const int pr = blockIdx.x;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n_steps; t += TPB) {
    const double o = obs[t * n_pairs + pr];
    s += o * o;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) o2[pr] = s;
}

// w[pair] = 1 / o2[pair], zero for pairs whose norm is <= 1e-12 of the
// largest (silent records carry no weight)
__global__ __launch_bounds__(TPB) void k_fit_weights(int n_pairs, const double* __restrict__ o2,
                                                     double* __restrict__ w) {
  __shared__ double sh[TPB / 64];
  __shared__ double smax;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n_pairs; i += TPB) mx = fmax(mx, sqrt(o2[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < TPB / 64; ++i) m = fmax(m, sh[i]);
    smax = m;
  }
  __syncthreads();
  const double thr = 1e-12 * smax;
  for (int i = threadIdx.x; i < n_pairs; i += TPB) {
    const double nrm = sqrt(o2[i]);
    w[i] = nrm > thr ? 1.0 / o2[i] : 0.0;
  }
}

// Block column `col` (< 4 nb) at row (pair, r): Green's block (j, b) for
// col = j nb + b (j < 3), observed block b for col = 3 nb + b.
struct FitSrc {
  const double* g[3];
  const double* obs;
  int n_pairs, m, nb;
};

__device__ __forceinline__ double fit_x(const FitSrc& S, int col, int pair, int r) {
  const int j = col / S.nb, b = col - j * S.nb;
  const double* src = j < 3 ? S.g[j] : S.obs;
  return src[(int64_t)(b * S.m + r) * S.n_pairs + pair];
}

// C = X^T diag(w) X for the 4 nb block columns, 16 x 16 output tiles, rows
// (pair, r) streamed through LDS in chunks; tiles below the diagonal skip.
constexpr int FT = 16, FK = 64;
__global__ __launch_bounds__(FT* FT) void k_fit_gram(FitSrc S, const double* __restrict__ w, int ncol,
                                                     double* __restrict__ C) {
  const int ta = blockIdx.y, tb = blockIdx.x;
  if (tb < ta) return;
  __shared__ double xa[FK][FT], xb[FK][FT];
  const int a = threadIdx.x / FT, bcol = threadIdx.x % FT;
  const int ca = ta * FT + a, cb = tb * FT + bcol;
  const int64_t n_rows = (int64_t)S.n_pairs * S.m;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < n_rows; k0 += FK) {
    for (int e = threadIdx.x; e < FK * FT; e += FT * FT) {
      const int kk = e / FT, cc = e % FT;
      const int64_t row = k0 + kk;
      double va = 0.0, vb = 0.0;
      if (row < n_rows) {
        const int pair = (int)(row / S.m), r = (int)(row - (int64_t)pair * S.m);
        const double wr = w[pair];
        if (ta * FT + cc < ncol) va = wr * fit_x(S, ta * FT + cc, pair, r);
        if (tb * FT + cc < ncol) vb = fit_x(S, tb * FT + cc, pair, r);
      }
      xa[kk][cc] = va;
      xb[kk][cc] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < FK; ++kk) acc += xa[kk][a] * xb[kk][bcol];
    __syncthreads();
  }
  // each symmetric pair written by one thread (in a diagonal tile the
  // (a, b) and (b, a) threads round differently), so C is deterministic
  if (ca < ncol && cb < ncol && (tb > ta || bcol >= a)) {
    C[(int64_t)ca * ncol + cb] = acc;
    C[(int64_t)cb * ncol + ca] = acc;
  }
}

// U[t][pair] = sum_j sum_{l <= t/m, l < n_shift} c[j][l] G_j[t - l m][pair]
__global__ __launch_bounds__(TPB) void k_fit_response(FitSrc S, int n_shift, int64_t n_steps,
                                                      const double* __restrict__ c, double* __restrict__ U) {
  const int64_t n = n_steps * S.n_pairs;
  for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
    const int64_t t = e / S.n_pairs;
    const int pair = (int)(e - t * S.n_pairs);
    const int lmax = (int)min((int64_t)n_shift - 1, t / S.m);
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l <= lmax; ++l) s += c[j * n_shift + l] * S.g[j][(t - (int64_t)l * S.m) * S.n_pairs + pair];
    U[e] = s;
  }
}

void launch_fit_weights(int n_pairs, int64_t n_steps, const double* obs, double* o2, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_pair_norms, dim3(n_pairs), dim3(TPB), 0, s, n_pairs, n_steps, obs, o2);
  hipLaunchKernelGGL(k_fit_weights, dim3(1), dim3(TPB), 0, s, n_pairs, o2, w);
}

void launch_fit_gram(const double* const g[3], const double* obs, int n_pairs, int m, int nb, const double* w,
                     double* C, hipStream_t s) {
  FitSrc S{{g[0], g[1], g[2]}, obs, n_pairs, m, nb};
  const int ncol = 4 * nb, nt = (ncol + FT - 1) / FT;
  hipLaunchKernelGGL(k_fit_gram, dim3(nt, nt), dim3(FT * FT), 0, s, S, w, ncol, C);
}

void launch_fit_response(const double* const g[3], int n_pairs, int m, int n_shift, int64_t n_steps,
                         const double* c, double* U, hipStream_t s) {
  FitSrc S{{g[0], g[1], g[2]}, nullptr, n_pairs, m, 0};
  unsigned gsz = nblocks(n_steps * n_pairs);
  if (gsz > 4096) gsz = 4096;
  hipLaunchKernelGGL(k_fit_response, dim3(gsz), dim3(TPB), 0, s, S, n_shift, n_steps, c, U);
}

}  // namespace sw
