// Learned initial guess (gfx950): a per-DOF network 10 -> 64 -> 64 -> 1
// (ReLU) predicting a correction to quadratic extrapolation of the last
// increments.  Inference runs on the matrix cores (v_mfma_f32_16x16x16_f16,
// FP16 weights and activations, FP32 accumulation); training uses FP32
// forward / back-propagation kernels and Adam.  Feature definitions: the
// backward differences of orders 0..3 of the last four increments of the DOF
// and of their element-neighbour means, divided by the largest magnitude s of
// those increments, and the node's Vs/500 and rho/2000; guess = p2 + s * y
// with p2 = 3 d0 - 3 d1 + d2.  The differences are formed in FP64 before the
// rounding to FP16: the higher ones are small (the third is the error the
// quadratic extrapolation made at the last step), and formed after the
// rounding they would be lost in it.
#include <hip/hip_runtime.h>

#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- network

// Network weights held in registers by every lane of a wave, laid out for
// the 16x16x16 MFMA in transposed form (rows = hidden units, columns = the
// 16 DOFs of one pass): lane l (q = l / 16, r = l % 16) holds
//   w1[b]    = W1[16b + r][4q .. 4q+3]          (A operand, layer 1)
//   b1[b]    = b1[16b + 4q .. 16b + 4q + 3]      (accumulator init)
//   w2[c][b] = W2[16c + r][16b + 4q .. +3]       (A operand, layer 2)
//   b2[c], w3[c] likewise for units 16c + 4q .. +3
struct MlpRegs {
  half4 w1[4];
  floatx4 b1[4];
  half4 w2[4][4];
  floatx4 b2[4];
  floatx4 w3[4];
  float b3;
};

__device__ __forceinline__ void mlp_load(const float* __restrict__ th, MlpRegs& R) {
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * q + j;
      R.w1[b][j] = (_Float16)(f < MLP_IN ? th[MLP_OFF_W1 + (16 * b + r) * MLP_IN + f] : 0.0f);
      R.b1[b][j] = th[MLP_OFF_B1 + 16 * b + 4 * q + j];
      R.b2[b][j] = th[MLP_OFF_B2 + 16 * b + 4 * q + j];
      R.w3[b][j] = th[MLP_OFF_W3 + 16 * b + 4 * q + j];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) R.w2[c][b][j] = (_Float16)th[MLP_OFF_W2 + (16 * c + r) * MLP_H + 16 * b + 4 * q + j];
  R.b3 = th[MLP_OFF_B3];
}

// Network output for the 16 inputs of one pass.  xin: lane (q, r) holds
// features 4q .. 4q+3 of input r.  Returns y of input r in every lane.
__device__ __forceinline__ float mlp_eval16(const half4 xin, const MlpRegs& R) {
  half4 h1[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    floatx4 d = __builtin_amdgcn_mfma_f32_16x16x16f16(R.w1[b], xin, R.b1[b], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) h1[b][j] = (_Float16)fmaxf(d[j], 0.0f);
  }
  float part = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    floatx4 acc = R.b2[c];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(R.w2[c][b], h1[b], acc, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) part += R.w3[c][j] * fmaxf(acc[j], 0.0f);
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part + R.b3;
}

// y[i] = net(X[i, 0..9]) for i < n (matrix-core path, as in the guess)
__global__ __launch_bounds__(TPB) void k_mlp_forward(int64_t n, const float* __restrict__ X,
                                                     const float* __restrict__ theta, float* __restrict__ y) {
  MlpRegs R;
  mlp_load(theta, R);
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
  const int64_t wave = ((int64_t)blockIdx.x * TPB + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * TPB) >> 6;
  for (int64_t g = wave; g * 16 < n; g += nwave) {
    const int64_t i = g * 16 + r;
    half4 xin;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * q + j;
      xin[j] = (_Float16)((i < n && f < MLP_IN) ? X[i * MLP_IN + f] : 0.0f);
    }
    const float v = mlp_eval16(xin, R);
    if (q == 0 && i < n) y[i] = v;
  }
}

void launch_mlp_forward(int64_t n, const float* X, const float* theta, float* y, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)((n / 16 + 3) / 4 + 1);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(TPB), 0, s, n, X, theta, y);
}

// ------------------------------------------------------------ features

struct GuessIn {
  double d[4];
  float nb[4];
  float vs, rho;
};

__device__ __forceinline__ void load_features(const MlpFeat& F, int64_t dof, GuessIn& o) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o.d[k] = F.hist[(int64_t)((F.head - k) & 3) * F.n_dof + dof];
    o.nb[k] = F.nbh[(int64_t)((F.nb_head - k) & 3) * F.n_dof + dof];
  }
  const int64_t node = dof / 3;
  o.vs = F.node_mat[2 * node];
  o.rho = F.node_mat[2 * node + 1];
}

// scale s and the normalised feature quartet of lane group q
__device__ __forceinline__ double feat_scale(const GuessIn& g) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s = fmax(s, fmax(fabs(g.d[k]), fabs((double)g.nb[k])));
  return s;
}

// backward differences of orders 0..3 of a[0..3] (newest first)
__device__ __forceinline__ void differences(const double a[4], double o[4]) {
  o[0] = a[0];
  o[1] = a[0] - a[1];
  o[2] = a[0] - 2.0 * a[1] + a[2];
  o[3] = a[0] - 3.0 * a[1] + 3.0 * a[2] - a[3];
}

// the ten features (FP32; the network rounds them to FP16)
__device__ __forceinline__ void features(const GuessIn& g, double s, float f[MLP_IN]) {
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  double nb[4], dd[4], dn[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) nb[k] = (double)g.nb[k];
  differences(g.d, dd);
  differences(nb, dn);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[k] = (float)(dd[k] * inv);
    f[4 + k] = (float)(dn[k] * inv);
  }
  f[8] = g.vs / 500.0f;
  f[9] = g.rho / 2000.0f;
}

__device__ __forceinline__ half4 feat_quartet(const GuessIn& g, double s, int q) {
  float f[MLP_IN];
  features(g, s, f);
  half4 x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * q + j;
    x[j] = (_Float16)(k < MLP_IN ? f[k] : 0.0f);
  }
  return x;
}

// x = p2 + s * net(features) per DOF (corr: the correction s * net alone);
// x = 0 when ||b|| = 0 or s = 0
__global__ __launch_bounds__(TPB) void k_mlp_guess(MlpFeat F, const float* __restrict__ theta,
                                                   double* __restrict__ x, const CgCtl* ctl, int corr) {
  MlpRegs R;
  mlp_load(theta, R);
  const bool zero = !(ctl->bb > 0.0);
  const int l = threadIdx.x & 63, q = l >> 4, r = l & 15;
  const int64_t wave = ((int64_t)blockIdx.x * TPB + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * TPB) >> 6;
  for (int64_t g = wave; g * 16 < F.n_dof; g += nwave) {
    const int64_t dof = g * 16 + r;
    GuessIn in{};
    if (dof < F.n_dof) load_features(F, dof, in);
    const double s = feat_scale(in);
    const float y = mlp_eval16(feat_quartet(in, s, q), R);
    if (q == 0 && dof < F.n_dof) {
      const double p2 = corr ? 0.0 : 3.0 * in.d[0] - 3.0 * in.d[1] + in.d[2];
      x[dof] = (zero || !(s > 0.0)) ? 0.0 : p2 + s * (double)y;
    }
  }
}

void launch_mlp_guess(const MlpFeat& F, const float* theta, double* x, const CgCtl* ctl, bool corr, hipStream_t s) {
  unsigned g = (unsigned)((F.n_dof / 16 + 3) / 4 + 1);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_mlp_guess, dim3(g), dim3(TPB), 0, s, F, theta, x, ctl, corr ? 1 : 0);
}

// Counter-based sampling: SplitMix64 finaliser of (seed, step, j).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Training rows for `count` DOFs drawn by (seed, step, j): the ten features
// (before the step), the target (du - p2) / s and the weight s^2.  Rows go
// to out[(row0 + j) mod capacity][12].
__global__ __launch_bounds__(TPB) void k_mlp_collect(MlpFeat F, const double* __restrict__ du, int count,
                                                     uint64_t seed, int64_t step, int64_t row0, int64_t capacity,
                                                     float* __restrict__ out) {
  const int j = blockIdx.x * TPB + threadIdx.x;
  if (j >= count) return;
  const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)step * 0x100000001B3ull + (uint64_t)j));
  const int64_t dof = (int64_t)(h % (uint64_t)F.n_dof);
  GuessIn in;
  load_features(F, dof, in);
  const double s = feat_scale(in);
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  float* o = out + ((row0 + j) % capacity) * MLP_ROW;
  float f[MLP_IN];
  features(in, s, f);
  for (int k = 0; k < MLP_IN; ++k) o[k] = f[k];
  const double p2 = 3.0 * in.d[0] - 3.0 * in.d[1] + in.d[2];
  o[10] = (float)((du[dof] - p2) * inv);
  o[11] = (float)(s * s);
}

void launch_mlp_collect(const MlpFeat& F, const double* du, int count, uint64_t seed, int64_t step, int64_t row0,
                        int64_t capacity, float* out, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_mlp_collect, dim3((count + TPB - 1) / TPB), dim3(TPB), 0, s, F, du, count, seed, step, row0,
                     capacity, out);
}

// -------------------------------------------------------------- training

constexpr int GCHUNK = 128;  // samples per block pass (one per work-item)

// Gradient of L = sum w (y - t)^2 / sum w, accumulated un-normalised:
// grad += sum_i 2 w_i (y_i - t_i) dy_i/dtheta, loss2 += (sum w e^2, sum w).
// Samples: rows i < n of S (all, in order) when nb == 0; otherwise nb rows
// drawn by (seed, batch) with replacement.
__global__ __launch_bounds__(GCHUNK) void k_mlp_grad(const float* __restrict__ S, int64_t n, int64_t nb,
                                                     uint64_t seed, int64_t batch, const float* __restrict__ theta,
                                                     double* __restrict__ grad, double* __restrict__ loss2) {
  __shared__ float th[MLP_NP];
  __shared__ float Xs[GCHUNK][MLP_IN];
  __shared__ float H1[GCHUNK][MLP_H + 1];
  __shared__ float H2[GCHUNK][MLP_H + 1];
  __shared__ float D2[GCHUNK][MLP_H + 1];
  __shared__ float D1[GCHUNK][MLP_H + 1];
  __shared__ float DY[GCHUNK];
  __shared__ double red[2 * GCHUNK / 64];
  const int tid = threadIdx.x;
  for (int j = tid; j < MLP_NP; j += GCHUNK) th[j] = theta[j];
  constexpr int PER = (MLP_NP + GCHUNK - 1) / GCHUNK;
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;
  double lw = 0.0, ww = 0.0;
  const int64_t total = nb > 0 ? nb : n;
  __syncthreads();
  for (int64_t c0 = (int64_t)blockIdx.x * GCHUNK; c0 < total; c0 += (int64_t)gridDim.x * GCHUNK) {
    // phase 1: forward and back-propagation of one sample per work-item
    const int64_t k = c0 + tid;
    float dy = 0.0f;
    if (k < total) {
      int64_t i = k;
      if (nb > 0) i = (int64_t)(splitmix64(seed ^ splitmix64((uint64_t)batch * 0x100000001B3ull + (uint64_t)k)) %
                                (uint64_t)n);
      const float* row = S + i * MLP_ROW;
      for (int f = 0; f < MLP_IN; ++f) Xs[tid][f] = row[f];
      for (int u = 0; u < MLP_H; ++u) {
        float z = th[MLP_OFF_B1 + u];
        for (int f = 0; f < MLP_IN; ++f) z += th[MLP_OFF_W1 + u * MLP_IN + f] * Xs[tid][f];
        H1[tid][u] = fmaxf(z, 0.0f);
      }
      float y = th[MLP_OFF_B3];
      for (int u = 0; u < MLP_H; ++u) {
        float z = th[MLP_OFF_B2 + u];
        for (int v = 0; v < MLP_H; ++v) z += th[MLP_OFF_W2 + u * MLP_H + v] * H1[tid][v];
        H2[tid][u] = fmaxf(z, 0.0f);
        y += th[MLP_OFF_W3 + u] * H2[tid][u];
      }
      const float w = row[11];
      const float e = y - row[10];
      dy = 2.0f * w * e;
      lw += (double)w * (double)e * (double)e;
      ww += (double)w;
      for (int u = 0; u < MLP_H; ++u) D2[tid][u] = H2[tid][u] > 0.0f ? dy * th[MLP_OFF_W3 + u] : 0.0f;
      for (int v = 0; v < MLP_H; ++v) {
        float sacc = 0.0f;
        for (int u = 0; u < MLP_H; ++u) sacc += D2[tid][u] * th[MLP_OFF_W2 + u * MLP_H + v];
        D1[tid][v] = H1[tid][v] > 0.0f ? sacc : 0.0f;
      }
    } else {
      for (int f = 0; f < MLP_IN; ++f) Xs[tid][f] = 0.0f;
      for (int u = 0; u < MLP_H; ++u) H1[tid][u] = H2[tid][u] = D2[tid][u] = D1[tid][u] = 0.0f;
    }
    DY[tid] = dy;
    __syncthreads();
    // phase 2: parameter j sums its products over the chunk
    const int ns = (int)((total - c0) < GCHUNK ? (total - c0) : GCHUNK);
#pragma unroll
    for (int kk = 0; kk < PER; ++kk) {
      const int j = tid + kk * GCHUNK;
      if (j >= MLP_NP) break;
      float sacc = 0.0f;
      if (j < MLP_OFF_B1) {
        const int u = j / MLP_IN, f = j % MLP_IN;
        for (int s = 0; s < ns; ++s) sacc += D1[s][u] * Xs[s][f];
      } else if (j < MLP_OFF_W2) {
        const int u = j - MLP_OFF_B1;
        for (int s = 0; s < ns; ++s) sacc += D1[s][u];
      } else if (j < MLP_OFF_B2) {
        const int u = (j - MLP_OFF_W2) / MLP_H, v = (j - MLP_OFF_W2) % MLP_H;
        for (int s = 0; s < ns; ++s) sacc += D2[s][u] * H1[s][v];
      } else if (j < MLP_OFF_W3) {
        const int u = j - MLP_OFF_B2;
        for (int s = 0; s < ns; ++s) sacc += D2[s][u];
      } else if (j < MLP_OFF_B3) {
        const int u = j - MLP_OFF_W3;
        for (int s = 0; s < ns; ++s) sacc += DY[s] * H2[s][u];
      } else {
        for (int s = 0; s < ns; ++s) sacc += DY[s];
      }
      acc[kk] += (double)sacc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int kk = 0; kk < PER; ++kk) {
    const int j = tid + kk * GCHUNK;
    if (j < MLP_NP && acc[kk] != 0.0) atomic_add(&grad[j], acc[kk]);
  }
  lw = wave_sum(lw);
  ww = wave_sum(ww);
  if ((tid & 63) == 0) {
    atomic_add(&loss2[0], lw);
    atomic_add(&loss2[1], ww);
  }
}

void launch_mlp_grad(const float* S, int64_t n, int64_t nb, uint64_t seed, int64_t batch, const float* theta,
                     double* grad, double* loss2, hipStream_t s) {
  const int64_t total = nb > 0 ? nb : n;
  if (total <= 0) return;
  unsigned g = (unsigned)((total + GCHUNK - 1) / GCHUNK);
  if (g > 512) g = 512;
  hipLaunchKernelGGL(k_mlp_grad, dim3(g), dim3(GCHUNK), 0, s, S, n, nb, seed, batch, theta, grad, loss2);
}

// Adam on the FP32 master weights with the gradient normalised by sum w;
// clears the gradient for the next batch.
__global__ __launch_bounds__(TPB) void k_mlp_adam(float* __restrict__ theta, float* __restrict__ m,
                                                  float* __restrict__ v, double* __restrict__ grad,
                                                  const double* __restrict__ loss2, int64_t step, float lr) {
  const int j = blockIdx.x * TPB + threadIdx.x;
  if (j >= MLP_NP) return;
  const double sw = loss2[1];
  const float g = sw > 0.0 ? (float)(grad[j] / sw) : 0.0f;
  grad[j] = 0.0;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mj = b1 * m[j] + (1.0f - b1) * g;
  const float vj = b2 * v[j] + (1.0f - b2) * g * g;
  m[j] = mj;
  v[j] = vj;
  const float mh = mj / (1.0f - powf(b1, (float)step));
  const float vh = vj / (1.0f - powf(b2, (float)step));
  theta[j] -= lr * mh / (sqrtf(vh) + eps);
}

void launch_mlp_adam(float* theta, float* m, float* v, double* grad, const double* loss2, int64_t step, float lr,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NP + TPB - 1) / TPB), dim3(TPB), 0, s, theta, m, v, grad, loss2, step,
                     lr);
}

// ----------------------------------------------- element-to-node averages

// out[node][k] (+)= (1/valence(node)) * sum over the node's elements of an
// element value: mode 0, the element mean of the node field in (3
// components, FP64); mode 1, (Vs, rho) of the element's material.  Interior
// nodes are stored, shared nodes added atomically (out cleared beforehand).
template <int K>
__global__ __launch_bounds__(TPB) void k_elem_to_node(MeshDev m, const double* __restrict__ in,
                                                      const uint8_t* __restrict__ emat,
                                                      const MatDev* __restrict__ mats, float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  int32_t* gid = reinterpret_cast<int32_t*>(acc + K * m.max_tile_nodes);
  float* xs = reinterpret_cast<float*>(gid + m.max_tile_nodes);
  const int t = blockIdx.x;
  const int n0 = m.tile_node_off[t];
  const int nt = m.tile_node_off[t + 1] - n0;
  const int nint = m.tile_nint[t];
  const int64_t ib = (int64_t)m.tile_int_base[t];
  for (int j = threadIdx.x; j < nt; j += TPB) gid[j] = m.tile_nodes[n0 + j];
  __syncthreads();
  for (int k = threadIdx.x; k < K * nt; k += TPB) {
    acc[k] = 0.0;
    if constexpr (K == 3) xs[k] = (float)in[3 * (int64_t)gid[k / 3] + (k % 3)];
  }
  __syncthreads();
  for (int e = m.tile_elem_off[t] + threadIdx.x; e < m.tile_elem_off[t + 1]; e += TPB) {
    int ln[10];
    for (int a = 0; a < 10; ++a) ln[a] = m.conn_loc[a * m.tet_stride + e] / 3;
    float val[K];
    if constexpr (K == 3) {
      for (int c = 0; c < 3; ++c) {
        float s = 0.0f;
        for (int a = 0; a < 10; ++a) s += xs[3 * ln[a] + c];
        val[c] = 0.1f * s;
      }
    } else {
      const MatDev mt = mats[emat[e]];
      val[0] = (float)(mt.zs / mt.rho);
      val[K - 1] = (float)mt.rho;
    }
    for (int a = 0; a < 10; ++a)
      for (int c = 0; c < K; ++c) atomicAdd(&acc[K * ln[a] + c], (double)val[c]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K * nt; k += TPB) {
    const int j = k / K;
    const int64_t g = gid[j];
    const float v = (float)(acc[k] * (double)m.inv_valence[g]);
    if (j < nint)
      out[K * (ib + j) + (k - K * j)] = v;
    else
      atomic_add(&out[K * g + (k - K * j)], v);
  }
}

void launch_neighbour_mean(const MeshDev& m, const double* in, float* out, hipStream_t s) {
  const size_t lds = (size_t)m.max_tile_nodes * (3 * sizeof(double) + sizeof(int32_t) + 3 * sizeof(float));
  hipLaunchKernelGGL(k_elem_to_node<3>, dim3(m.n_tiles), dim3(TPB), lds, s, m, in, (const uint8_t*)nullptr,
                     (const MatDev*)nullptr, out);
}

void launch_node_material(const MeshDev& m, const uint8_t* emat, const MatDev* mats, float* out, hipStream_t s) {
  const size_t lds = (size_t)m.max_tile_nodes * (2 * sizeof(double) + sizeof(int32_t));
  hipLaunchKernelGGL(k_elem_to_node<2>, dim3(m.n_tiles), dim3(TPB), lds, s, m, (const double*)nullptr, emat, mats,
                     out);
}

}  // namespace sw
