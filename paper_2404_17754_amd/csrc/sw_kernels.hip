// Node-parallel HIP kernels (gfx950) of the implicit wave-propagation step:
// fused CG vector updates with the 3x3 block-Jacobi preconditioner, dot
// products, mixed-precision refinement glue, initial guesses, the Newmark
// update, receiver recording and the ERR misfit of Eq. (eqerr).
//
// Every vector is node-major [node][3] in the mesh's internal node order.
// Partial dot products are reduced across the 64-wide wavefront with
// shuffles, across the workgroup through LDS, and across the grid with one
// FP64 atomic per workgroup into a device control block.
#include <hip/hip_runtime.h>

#include "sw_bf16.h"
#include "sw_device.h"
#include "sw_internal.h"

namespace sw {

// --------------------------------------------------------- CG vector ops

__device__ __forceinline__ float to_t(__half v, float) { return __half2float(v); }
__device__ __forceinline__ float to_t(float v, float) { return v; }
__device__ __forceinline__ double to_t(double v, double) { return v; }

// the six values (xx yy zz yz xz xy) of node i's block
template <typename T, typename PT>
__device__ __forceinline__ void bj_load(const PT* __restrict__ P, int64_t i, T v[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = to_t(P[6 * i + k], T());
}
// FP16 blocks: three 32-bit loads of two values each (12-byte records are
// 4-byte aligned)
template <>
__device__ __forceinline__ void bj_load<float, __half>(const __half* __restrict__ P, int64_t i, float v[6]) {
  const __half2* P2 = reinterpret_cast<const __half2*>(P) + 3 * i;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float2 f = __half22float2(P2[k]);
    v[2 * k] = f.x;
    v[2 * k + 1] = f.y;
  }
}

// z = P r for the symmetric 3x3 block of node i (xx yy zz yz xz xy), stored
// in PT, applied in T
template <typename T, typename PT>
__device__ __forceinline__ void bj_apply(const PT* __restrict__ P, int64_t i, const T r[3], T z[3]) {
  T v[6];
  bj_load<T, PT>(P, i, v);
  const T a = v[0], b = v[1], c = v[2], yz = v[3], xz = v[4], xy = v[5];
  z[0] = a * r[0] + xy * r[1] + xz * r[2];
  z[1] = xy * r[0] + b * r[1] + yz * r[2];
  z[2] = xz * r[0] + yz * r[1] + c * r[2];
}

// Grid for the node-parallel kernels: grid-stride loops over a capped grid
// (enough workgroups to fill 256 CUs several times over).
static inline unsigned vgrid(int64_t n) {
  unsigned g = nblocks(n);
  return g > 8192 ? 8192 : (g == 0 ? 1 : g);
}

// r = b - q, z = P r, p = z, q = 0; rz[0], rr[0]
template <typename T, typename PT>
__device__ __forceinline__ void cg_init_body(int64_t n, const T* __restrict__ b, const T* __restrict__ q,
                                             const PT* __restrict__ P, T* __restrict__ r, T* __restrict__ z,
                                             T* __restrict__ p, T* __restrict__ qz, CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    T rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = b[3 * i + c] - (q ? q[3 * i + c] : (T)0);
    bj_apply<T, PT>(P, i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[3 * i + c] = rv[c];
      z[3 * i + c] = zv[c];
      p[3 * i + c] = zv[c];
      if (qz) qz[3 * i + c] = (T)0;
      rz += (double)rv[c] * (double)zv[c];
      rr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(rz, rr, sh);
  if (threadIdx.x == 0) {
    atomic_add(&ctl->rz[0][blockIdx.x % NSLOT], rz);
    atomic_add(&ctl->rr[0][blockIdx.x % NSLOT], rr);
  }
}

// alpha = rz[par] / pAp; r -= alpha q; z = P r; q = 0 (shared nodes);
// rz[par^1] += r.z, rr[par^1] += r.r.  The solution update x += alpha p is
// left to the direction kernel, which reads p anyway: alpha and whether this
// iteration ran go to ctl->alpha and ctl->live (the direction kernel cannot
// take that from ctl->done, which its own first workgroup may set while the
// others still run).
template <typename T, typename PT>
__device__ __forceinline__ void cg_update_body(int64_t n, int64_t n_int, int par, const PT* __restrict__ P,
                                               T* __restrict__ r, T* __restrict__ z, T* __restrict__ q,
                                               CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (ctl->done) {
    if (lead) ctl->live = 0;
    return;
  }
  const T alpha = (T)(slot_sum<NSLOT>(ctl->rz[par]) / slot_sum<NSLOT>(ctl->pAp));
  if (lead) {
    ctl->alpha = (double)alpha;
    ctl->live = 1;
    ctl->iter_cur = ctl->iters;
  }
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    // every load of the node first (12-byte accesses), then the stores; r
    // and q are not read again before the next iteration's operator pass
    // and update, so they go through the caches non-temporally (z, read by
    // the direction kernel right after, and the preconditioner blocks, read
    // every iteration, stay cached)
    T rv[3], qv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rv[c] = __builtin_nontemporal_load(&r[3 * i + c]);
      qv[c] = __builtin_nontemporal_load(&q[3 * i + c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] -= alpha * qv[c];
    bj_apply<T, PT>(P, i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(rv[c], &r[3 * i + c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) z[3 * i + c] = zv[c];
    if (i >= n_int) {
#pragma unroll
      for (int c = 0; c < 3; ++c) q[3 * i + c] = (T)0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rz += (double)rv[c] * (double)zv[c];
      rr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(rz, rr, sh);
  if (threadIdx.x == 0) {
    atomic_add(&ctl->rz[par ^ 1][blockIdx.x % NSLOT], rz);
    atomic_add(&ctl->rr[par ^ 1][blockIdx.x % NSLOT], rr);
  }
}

// After a live update: x += alpha p with the update's alpha, the convergence
// test, then (unless the solve stops here) p = z + beta p with
// beta = rz[par^1] / rz[par].  ctl->iters (the step's iterations so far) is
// written by the first workgroup only; the update kernel before it keeps a
// copy in ctl->iter_cur, so that no workgroup reads a value another one is
// writing.
template <typename T>
__device__ __forceinline__ void cg_dir_body(int64_t n, int par, int iter_abs, int max_iter, const T* __restrict__ z,
                                            T* __restrict__ p, T* __restrict__ x, CgCtl* ctl) {
  if (!ctl->live) return;
  // iter_abs < 0: the iteration index from the control block (graph replays
  // launch the same arguments for every pair of iterations)
  if (iter_abs < 0) iter_abs = ctl->iter_cur;
  const double rr = slot_sum<NSLOT>(ctl->rr[par ^ 1]);
  const bool stop = !(rr > ctl->tol2) || (iter_abs + 1 >= max_iter);  // NaN stops too
  const T alpha = (T)ctl->alpha;
  const T beta = (T)(slot_sum<NSLOT>(ctl->rz[par ^ 1]) / slot_sum<NSLOT>(ctl->rz[par]));
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      ctl->iters = iter_abs + 1;
      if (stop) ctl->done = 1;
    }
    if (threadIdx.x < NSLOT) ctl->pAp[threadIdx.x] = 0.0;
  }
  if constexpr (sizeof(T) == 4) {
    // elementwise over the 3n values, four at a time (16-byte accesses; the
    // vectors start 256-byte aligned).  x and z are not read again before
    // the next iteration rewrites them: non-temporal accesses keep them from
    // displacing p, which the next operator pass gathers, in the caches
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const int64_t n3 = 3 * n, n4 = n3 / 4;
    const f32x4* __restrict__ z4 = reinterpret_cast<const f32x4*>(z);
    f32x4* __restrict__ p4 = reinterpret_cast<f32x4*>(p);
    f32x4* __restrict__ x4 = reinterpret_cast<f32x4*>(x);
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * TPB) {
      const f32x4 pv = p4[i];
      f32x4 xv = __builtin_nontemporal_load(x4 + i);
      f32x4 zv = {0.0f, 0.0f, 0.0f, 0.0f};
      if (!stop) zv = __builtin_nontemporal_load(z4 + i);
      xv += alpha * pv;
      __builtin_nontemporal_store(xv, x4 + i);
      if (!stop) p4[i] = zv + beta * pv;
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * TPB + threadIdx.x; i < n3; i += (int64_t)gridDim.x * TPB) {
      const float pv = p[i];
      x[i] += alpha * pv;
      if (!stop) p[i] = z[i] + beta * pv;
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
      T zv[3], pv[3], xv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pv[c] = p[3 * i + c];
        xv[c] = x[3 * i + c];
        zv[c] = stop ? (T)0 : z[3 * i + c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) x[3 * i + c] = xv[c] + alpha * pv[c];
      if (!stop) {
#pragma unroll
        for (int c = 0; c < 3; ++c) p[3 * i + c] = zv[c] + beta * pv[c];
      }
    }
  }
}

// Direction kernel of the SW_MIXED_FP16 inner CG: as cg_dir_body in FP32
// arithmetic, with the direction stored in bfloat16 (p16).  The operator
// pass, x += alpha p and p = z + beta p all use the stored values, so the
// iteration is CG along the rounded directions; the rounding costs
// conjugacy, which the FP64 refinement around the inner solve absorbs.
__global__ __launch_bounds__(TPB) void k_cg_dir_h(int64_t n, int par, int iter_abs, int max_iter,
                                                  const float* __restrict__ z, uint16_t* __restrict__ p16,
                                                  float* __restrict__ x, CgCtl* ctl) {
  if (!ctl->live) return;
  if (iter_abs < 0) iter_abs = ctl->iter_cur;
  const double rr = slot_sum<NSLOT>(ctl->rr[par ^ 1]);
  const bool stop = !(rr > ctl->tol2) || (iter_abs + 1 >= max_iter);  // NaN stops too
  const float alpha = (float)ctl->alpha;
  const float beta = (float)(slot_sum<NSLOT>(ctl->rz[par ^ 1]) / slot_sum<NSLOT>(ctl->rz[par]));
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      ctl->iters = iter_abs + 1;
      if (stop) ctl->done = 1;
    }
    if (threadIdx.x < NSLOT) ctl->pAp[threadIdx.x] = 0.0;
  }
  // four values per work-item (8-byte direction, 16-byte x and z accesses)
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int64_t n3 = 3 * n, n4 = n3 / 4;
  const f32x4* __restrict__ z4 = reinterpret_cast<const f32x4*>(z);
  f32x4* __restrict__ x4 = reinterpret_cast<f32x4*>(x);
  uint2* __restrict__ p4 = reinterpret_cast<uint2*>(p16);
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * TPB) {
    const uint2 ph = p4[i];
    const f32x4 pv = {bf16_value((uint16_t)(ph.x & 0xffffu)), bf16_value((uint16_t)(ph.x >> 16)),
                      bf16_value((uint16_t)(ph.y & 0xffffu)), bf16_value((uint16_t)(ph.y >> 16))};
    f32x4 xv = __builtin_nontemporal_load(x4 + i);
    xv += alpha * pv;
    __builtin_nontemporal_store(xv, x4 + i);
    if (!stop) {
      const f32x4 q = __builtin_nontemporal_load(z4 + i) + beta * pv;
      p4[i] = make_uint2((uint32_t)bf16_round(q.x) | ((uint32_t)bf16_round(q.y) << 16),
                         (uint32_t)bf16_round(q.z) | ((uint32_t)bf16_round(q.w) << 16));
    }
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * TPB + threadIdx.x; i < n3; i += (int64_t)gridDim.x * TPB) {
    const float pv = bf16_value(p16[i]);
    x[i] += alpha * pv;
    if (!stop) p16[i] = bf16_round(z[i] + beta * pv);
  }
}

template <typename T, typename PT>
__global__ __launch_bounds__(TPB) void k_cg_init(int64_t n, const T* b, const T* q, const PT* P, T* r, T* z, T* p,
                                                 T* qz, CgCtl* ctl) {
  cg_init_body<T, PT>(n, b, q, P, r, z, p, qz, ctl);
}
template <typename T, typename PT>
__global__ __launch_bounds__(TPB) void k_cg_update(int64_t n, int64_t n_int, int par, const PT* P, T* r, T* z, T* q,
                                                   CgCtl* ctl) {
  cg_update_body<T, PT>(n, n_int, par, P, r, z, q, ctl);
}
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_dir(int64_t n, int par, int iter_abs, int max_iter, const T* z, T* p,
                                                T* x, CgCtl* ctl) {
  cg_dir_body<T>(n, par, iter_abs, max_iter, z, p, x, ctl);
}

void launch_cg_init_f64(int64_t n, const double* b, const double* q, const double* P, double* r, double* z, double* p,
                        double* qz, CgCtl* ctl, hipStream_t s, bool det) {
  hipLaunchKernelGGL((k_cg_init<double, double>), dim3(det ? NSLOT : vgrid(n)), dim3(TPB), 0, s, n, b, q, P, r, z, p,
                     qz, ctl);
}
void launch_cg_init_f32(int64_t n, const float* b, const float* q, const __half* P, float* r, float* z, float* p,
                        float* qz, CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_init<float, __half>), dim3(vgrid(n)), dim3(TPB), 0, s, n, b, q, P, r, z, p, qz, ctl);
}
void launch_cg_update_f64(int64_t n, int par, const double* P, double* r, double* z, double* q, CgCtl* ctl,
                          hipStream_t s, bool det) {
  hipLaunchKernelGGL((k_cg_update<double, double>), dim3(det ? NSLOT : vgrid(n)), dim3(TPB), 0, s, n, (int64_t)0, par,
                     P, r, z, q, ctl);
}
void launch_cg_update_f32(int64_t n, int64_t n_int, int par, const __half* P, float* r, float* z, float* q,
                          CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_update<float, __half>), dim3(vgrid(n)), dim3(TPB), 0, s, n, n_int, par, P, r, z, q, ctl);
}
void launch_cg_dir_h(int64_t n, int par, int iter_abs, int max_iter, const float* z, uint16_t* p16, float* x,
                     CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir_h, dim3(vgrid(n)), dim3(TPB), 0, s, n, par, iter_abs, max_iter, z, p16, x, ctl);
}
void launch_cg_dir_f64(int64_t n, int par, int iter_abs, int max_iter, const double* z, double* p, double* x,
                       CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir<double>, dim3(vgrid(n)), dim3(TPB), 0, s, n, par, iter_abs, max_iter, z, p, x, ctl);
}
void launch_cg_dir_f32(int64_t n, int par, int iter_abs, int max_iter, const float* z, float* p, float* x,
                       CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir<float>, dim3(vgrid(n)), dim3(TPB), 0, s, n, par, iter_abs, max_iter, z, p, x, ctl);
}

// ------------------------------------------------------------ scalars

__device__ __forceinline__ void ctl_prepare_body(CgCtl* ctl, double rtol) {
  const int i = threadIdx.x;
  if (i < NSLOT) {
    ctl->pAp[i] = 0.0;
    ctl->rz[0][i] = ctl->rz[1][i] = 0.0;
    ctl->rr[0][i] = ctl->rr[1][i] = 0.0;
  }
  if (i == 0) {
    ctl->tol2 = rtol * rtol * ctl->bb;
    ctl->rr_true = 0.0;
    ctl->done = 0;
    ctl->iters = 0;
  }
}
__global__ void k_ctl_prepare(CgCtl* ctl, double rtol) { ctl_prepare_body(ctl, rtol); }
void launch_ctl_prepare(CgCtl* ctl, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_prepare, dim3(1), dim3(64), 0, s, ctl, rtol);
}

__global__ __launch_bounds__(TPB) void k_norm2(int64_t n, const double* __restrict__ x, double* out) {
  __shared__ double sh[2 * TPB / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) acc += x[i] * x[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) atomic_add(out, acc);
}
void launch_norm2(int64_t n, const double* x, double* out, hipStream_t s, bool det) {
  unsigned g = nblocks(n);
  if (g > 4096) g = 4096;
  if (det || g == 0) g = 1;
  hipLaunchKernelGGL(k_norm2, dim3(g), dim3(TPB), 0, s, n, x, out);
}

// r = b - q (n doubles), rr_true += r.r (ctl->rr_true cleared by the caller)
__global__ __launch_bounds__(TPB) void k_true_res(int64_t n, const double* __restrict__ b,
                                                  const double* __restrict__ q, double* __restrict__ r, CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double t = b[i] - q[i];
    r[i] = t;
    acc += t * t;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) atomic_add(&ctl->rr_true, acc);
}
void launch_true_residual(int64_t n, const double* b, const double* q, double* r, CgCtl* ctl, hipStream_t s,
                          bool det) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  if (det || g == 0) g = 1;
  hipLaunchKernelGGL(k_true_res, dim3(g), dim3(TPB), 0, s, n, b, q, r, ctl);
}

// Start of a refinement round in one pass: the FP32 inner system's
// right-hand side r32 = r / ||r|| (||r||^2 = rr_true of ctl64, kept as its
// scale), the inner solution d32 = 0, and the CG start z = P r32, p = z
// with r32.z and r32.r32 into slot ring 0 of ctl32 (cleared beforehand).
__global__ __launch_bounds__(TPB) void k_ir_begin(int64_t n_nodes, const double* __restrict__ r64,
                                                  const __half* __restrict__ P, float* __restrict__ r32,
                                                  float* __restrict__ z32, float* __restrict__ p32,
                                                  uint16_t* __restrict__ p16, float* __restrict__ d32, CgCtl* ctl64,
                                                  CgCtl* ctl32) {
  __shared__ double sh[2 * TPB / 64];
  const double nr = sqrt(ctl64->rr_true);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl64->scale = nr;
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n_nodes; i += (int64_t)gridDim.x * TPB) {
    float rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = (float)(r64[3 * i + c] * inv);
    bj_apply<float, __half>(P, i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r32[3 * i + c] = rv[c];
      z32[3 * i + c] = zv[c];
      if (p16)
        p16[3 * i + c] = bf16_round(zv[c]);
      else
        p32[3 * i + c] = zv[c];
      d32[3 * i + c] = 0.0f;
      rz += (double)rv[c] * (double)zv[c];
      rr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(rz, rr, sh);
  if (threadIdx.x == 0) {
    atomic_add(&ctl32->rz[0][blockIdx.x % NSLOT], rz);
    atomic_add(&ctl32->rr[0][blockIdx.x % NSLOT], rr);
  }
}
void launch_ir_begin(int64_t n_nodes, const double* r64, const __half* P, float* r32, float* z32, float* p32,
                     uint16_t* p16, float* d32, CgCtl* ctl64, CgCtl* ctl32, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_begin, dim3(vgrid(n_nodes)), dim3(TPB), 0, s, n_nodes, r64, P, r32, z32, p32, p16, d32,
                     ctl64, ctl32);
}

__global__ __launch_bounds__(TPB) void k_ir_update(int64_t n, double* __restrict__ x, const float* __restrict__ d,
                                                   const CgCtl* ctl) {
  const double sc = ctl->scale;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
    x[i] += sc * (double)d[i];
}
void launch_ir_update(int64_t n, double* x64, const float* d32, const CgCtl* ctl, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_ir_update, dim3(g), dim3(TPB), 0, s, n, x64, d32, ctl);
}

// ------------------------------------------------ flexible outer CG (FP64)
//
// One outer iteration of the flexible (variable-preconditioned) CG whose
// preconditioner is the FP32 inner CG: z = scale d32 (the inner solution of
// the scaled residual system), w = A z (FP64 operator pass), then
//   p = z - beta p_prev,  q = w - beta q_prev,  beta = (z.q_prev)/(p_prev.q_prev)
//   x += alpha p,  r -= alpha q,                alpha = (p.r)/(p.q)
// (truncation to one previous direction).  Dot products go through dots[]
// (cleared by the host before each kernel that adds into them): dots[0]
// z.q_prev, dots[1] p.r, dots[2 + parity] p.q of the iteration of that
// parity, and r.r into ctl->rr_true.

__global__ __launch_bounds__(TPB) void k_fcg_begin(int64_t n, const float* __restrict__ d32, const CgCtl* ctl,
                                                   const double* __restrict__ q_prev, double* __restrict__ z,
                                                   double* dots) {
  __shared__ double sh[2 * TPB / 64];
  const double sc = ctl->scale;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double v = sc * (double)d32[i];
    z[i] = v;
    if (q_prev) acc += v * q_prev[i];
  }
  if (q_prev) {
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) atomic_add(&dots[0], acc);
  }
}
void launch_fcg_begin(int64_t n, const float* d32, const CgCtl* ctl64, const double* q_prev, double* z,
                      double* dots, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fcg_begin, dim3(g), dim3(TPB), 0, s, n, d32, ctl64, q_prev, z, dots);
}

__global__ __launch_bounds__(TPB) void k_fcg_dir(int64_t n, const double* __restrict__ z,
                                                 const double* __restrict__ w, const double* __restrict__ r,
                                                 const double* __restrict__ p_prev, const double* __restrict__ q_prev,
                                                 double* __restrict__ p, double* __restrict__ q, double* dots,
                                                 int par) {
  __shared__ double sh[2 * TPB / 64];
  const double beta = p_prev ? dots[0] / dots[2 + (par ^ 1)] : 0.0;
  double pr = 0.0, pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    double pv = z[i], qv = w[i];
    if (p_prev) {
      pv -= beta * p_prev[i];
      qv -= beta * q_prev[i];
    }
    p[i] = pv;
    q[i] = qv;
    pr += pv * r[i];
    pq += pv * qv;
  }
  block_sum2(pr, pq, sh);
  if (threadIdx.x == 0) {
    atomic_add(&dots[1], pr);
    atomic_add(&dots[2 + par], pq);
  }
}
void launch_fcg_dir(int64_t n, const double* z, const double* w, const double* r, const double* p_prev,
                    const double* q_prev, double* p, double* q, double* dots, int par, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fcg_dir, dim3(g), dim3(TPB), 0, s, n, z, w, r, p_prev, q_prev, p, q, dots, par);
}

__global__ __launch_bounds__(TPB) void k_fcg_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* dots, int par, CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  const double alpha = dots[1] / dots[2 + par];
  double rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    x[i] += alpha * p[i];
    const double rv = r[i] - alpha * q[i];
    r[i] = rv;
    rr += rv * rv;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) atomic_add(&ctl->rr_true, rr);
}
void launch_fcg_update(int64_t n, double* x, double* r, const double* p, const double* q, const double* dots,
                       int par, CgCtl* ctl64, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fcg_update, dim3(g), dim3(TPB), 0, s, n, x, r, p, q, dots, par, ctl64);
}

// ------------------------------------------------------------- guesses

// Lagrange extrapolation of order p from the last p+1 increments:
// x = sum_j (-1)^j C(p+1, j+1) hist[head - j]
__device__ __forceinline__ void guess_poly_body(int64_t n, const double* __restrict__ hist, int head, int order,
                                                double* __restrict__ x, const CgCtl* ctl) {
  const bool zero = !(ctl->bb > 0.0) || order < 0;
  double coef[4] = {0, 0, 0, 0};
  if (!zero) {
    const double tab[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
    for (int j = 0; j <= order; ++j) coef[j] = tab[order][j];
  }
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    double acc = 0.0;
    if (!zero) {
      for (int j = 0; j <= order; ++j) acc += coef[j] * hist[(int64_t)((head - j + 4) & 3) * n + i];
    }
    x[i] = acc;
  }
}
__global__ __launch_bounds__(TPB) void k_guess_poly(int64_t n, const double* hist, int head, int order, double* x,
                                                    const CgCtl* ctl) {
  guess_poly_body(n, hist, head, order, x, ctl);
}
void launch_guess_poly(int64_t n, const double* hist, int head, int order, double* x, const CgCtl* ctl,
                       hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_guess_poly, dim3(g), dim3(TPB), 0, s, n, hist, head, order, x, ctl);
}

// ------------------------------------------------------------ Newmark

__device__ __forceinline__ void newmark_body(int64_t n, double dt, const double* __restrict__ du,
                                             double* __restrict__ u, double* __restrict__ v, double* __restrict__ a,
                                             double* __restrict__ hist) {
  const double c2 = 2.0 / dt, c4 = 4.0 / (dt * dt), c4v = 4.0 / dt;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double d = du[i], vo = v[i];
    u[i] += d;
    v[i] = c2 * d - vo;
    a[i] = c4 * d - c4v * vo - a[i];
    if (hist) hist[i] = d;
  }
}
__global__ __launch_bounds__(TPB) void k_newmark(int64_t n, double dt, const double* du, double* u, double* v,
                                                 double* a, double* hist) {
  newmark_body(n, dt, du, u, v, a, hist);
}
void launch_newmark(int64_t n, double dt, const double* du, double* u, double* v, double* a, double* hist_slot,
                    hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_newmark, dim3(g), dim3(TPB), 0, s, n, dt, du, u, v, a, hist_slot);
}

__global__ void k_log_step(int32_t* it_dst, int32_t iters, double* rel_dst, double rel) {
  if (threadIdx.x == 0) {
    *it_dst = iters;
    *rel_dst = rel;
  }
}
void launch_log_step(int32_t* it_dst, int32_t iters, double* rel_dst, double rel, hipStream_t s) {
  hipLaunchKernelGGL(k_log_step, dim3(1), dim3(64), 0, s, it_dst, iters, rel_dst, rel);
}

__global__ void k_record(int n_rec, const int32_t* __restrict__ rec, const double* __restrict__ v,
                         double* __restrict__ row) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n_rec) row[i] = v[3 * (int64_t)rec[i / 3] + i % 3];
}
void launch_record(int n_rec, const int32_t* rec, const double* v, double* row, hipStream_t s) {
  if (n_rec <= 0) return;
  hipLaunchKernelGGL(k_record, dim3((3 * n_rec + 255) / 256), dim3(256), 0, s, n_rec, rec, v, row);
}

// --------------------------------------------------------------- misfit

// pair_buf[2 * pair] = sum_t (U - obs)^2, pair_buf[2 * pair + 1] = sum_t obs^2
__global__ __launch_bounds__(TPB) void k_misfit_pairs(int n_pairs, int64_t n_steps, const double* __restrict__ U,
                                                      const double* __restrict__ obs, double* __restrict__ buf) {
  __shared__ double sh[2 * TPB / 64];
  const int pr = blockIdx.x;
  double d2 = 0.0, o2 = 0.0;
  for (int64_t t = threadIdx.x; t < n_steps; t += TPB) {
    const double o = obs[t * n_pairs + pr];
    const double d = U[t * n_pairs + pr] - o;
    d2 += d * d;
    o2 += o * o;
  }
  block_sum2(d2, o2, sh);
  if (threadIdx.x == 0) {
    buf[2 * pr] = d2;
    buf[2 * pr + 1] = o2;
  }
}

// out2[0] = mean over used pairs of sqrt(d2)/sqrt(o2); out2[1] = pairs used
__global__ __launch_bounds__(TPB) void k_misfit_final(int n_pairs, const double* __restrict__ buf,
                                                      double* __restrict__ out2) {
  __shared__ double sh[2 * TPB / 64];
  __shared__ double smax;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n_pairs; i += TPB) mx = fmax(mx, sqrt(buf[2 * i + 1]));
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
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n_pairs; i += TPB) {
    const double on = sqrt(buf[2 * i + 1]);
    if (on > thr) {
      s += sqrt(buf[2 * i]) / on;
      c += 1.0;
    }
  }
  __syncthreads();
  block_sum2(s, c, sh);
  if (threadIdx.x == 0) {
    out2[0] = c > 0.0 ? s / c : __builtin_nan("");
    out2[1] = c;
  }
}

void launch_misfit(int n_rec, int64_t n_steps, const double* U, const double* obs, double* pair_buf, double* out2,
                   hipStream_t s) {
  const int np = 3 * n_rec;
  hipLaunchKernelGGL(k_misfit_pairs, dim3(np), dim3(TPB), 0, s, np, n_steps, U, obs, pair_buf);
  hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(TPB), 0, s, np, pair_buf, out2);
}

// ---------------------------------------------------------------- fills

template <typename T>
__global__ __launch_bounds__(TPB) void k_fill(int64_t n, T* __restrict__ x, T v) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) x[i] = v;
}
void launch_fill_f64(int64_t n, double* x, double val, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = nblocks(n);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(TPB), 0, s, n, x, val);
}
void launch_fill_f32(int64_t n, float* x, float val, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = nblocks(n);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(TPB), 0, s, n, x, val);
}

// ---------------------------------------------------------- permutation

template <typename T>
__global__ __launch_bounds__(TPB) void k_permute(int64_t n, int w, const T* __restrict__ src,
                                                 const int32_t* __restrict__ map, T* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n * w; k += (int64_t)gridDim.x * TPB) {
    const int64_t i = k / w;
    dst[k] = src[(int64_t)map[i] * w + (k - i * w)];
  }
}
void launch_permute_f64(int64_t n, int w, const double* src, const int32_t* map, double* dst, hipStream_t s) {
  unsigned g = nblocks(n * w);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_permute<double>, dim3(g), dim3(TPB), 0, s, n, w, src, map, dst);
}
void launch_permute_f32(int64_t n, int w, const float* src, const int32_t* map, float* dst, hipStream_t s) {
  unsigned g = nblocks(n * w);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_permute<float>, dim3(g), dim3(TPB), 0, s, n, w, src, map, dst);
}

// ---------------------------------------------------------------- lanes
//
// Several cases (lanes) in one launch: grid (blocks per lane, lanes), each
// lane's blocks run the same body as the single-case kernel on that lane's
// vectors; lanes marked inactive return at once.

template <int OP>
__global__ __launch_bounds__(TPB) void k_lane_op(const LaneDev* __restrict__ lanes, const LaneState* __restrict__ st,
                                                 LaneInfo* __restrict__ info) {
  const int l = blockIdx.y;
  if (st != nullptr && !st[l].active) return;
  const LaneDev& L = lanes[l];
  const int64_t nn = L.n_nodes, nd = 3 * nn;
  const int64_t i0 = (int64_t)blockIdx.x * TPB + threadIdx.x, stride = (int64_t)gridDim.x * TPB;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if constexpr (OP == LANE_BEGIN_STEP) {
    if (lead) L.ctl64->bb = 0.0;
    for (int64_t i = i0; i < nd; i += stride) L.b[i] = 0.0;
  } else if constexpr (OP == LANE_NORM2_B) {
    __shared__ double sh[TPB / 64];
    double acc = 0.0;
    for (int64_t i = i0; i < nd; i += stride) acc += L.b[i] * L.b[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) atomic_add(&L.ctl64->bb, acc);
  } else if constexpr (OP == LANE_PREPARE64) {
    if (blockIdx.x == 0) ctl_prepare_body(L.ctl64, L.rtol);
  } else if constexpr (OP == LANE_GUESS) {
    if (L.guess_order >= -1) guess_poly_body(nd, L.hist, L.hist_head, L.guess_order, L.x, L.ctl64);
  } else if constexpr (OP == LANE_RRTRUE_RESET) {
    if (lead) L.ctl64->rr_true = 0.0;
  } else if constexpr (OP == LANE_TRUE_RES) {
    __shared__ double sh[TPB / 64];
    const bool zq = st != nullptr && st[l].zero_q;
    double acc = 0.0;
    for (int64_t i = i0; i < nd; i += stride) {
      const double t = L.b[i] - L.q[i];
      L.r[i] = t;
      if (zq) L.q[i] = 0.0;
      acc += t * t;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) atomic_add(&L.ctl64->rr_true, acc);
  } else if constexpr (OP == LANE_TO_F32) {
    const double nr = sqrt(L.ctl64->rr_true);
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    if (blockIdx.x == 0) {
      CgCtl* c = L.ctl32;
      if (threadIdx.x < NSLOT) {
        c->pAp[threadIdx.x] = 0.0;
        c->rz[0][threadIdx.x] = c->rz[1][threadIdx.x] = 0.0;
        c->rr[0][threadIdx.x] = c->rr[1][threadIdx.x] = 0.0;
      }
      if (threadIdx.x == 0) {
        const double tol = st != nullptr ? st[l].tol : 0.5;
        L.ctl64->scale = nr;
        c->bb = 1.0;
        c->tol2 = tol * tol;
        c->rr_true = 0.0;
        c->scale = 0.0;
        c->done = 0;
        c->iters = 0;
      }
    }
    for (int64_t i = i0; i < nd; i += stride) {
      L.r32[i] = (float)(L.r[i] * inv);
      L.d32[i] = 0.0f;
    }
  } else if constexpr (OP == LANE_CG_INIT32) {
    cg_init_body<float, __half>(nn, L.r32, nullptr, L.pinv16, L.r32, L.z32, L.p32, nullptr, L.ctl32);
  } else if constexpr (OP == LANE_CG_INIT64) {
    cg_init_body<double, double>(nn, L.b, L.q, L.pinv64, L.r, L.z, L.p, L.q, L.ctl64);
  } else if constexpr (OP == LANE_IR_UPDATE) {
    const double sc = L.ctl64->scale;
    for (int64_t i = i0; i < nd; i += stride) L.x[i] += sc * (double)L.d32[i];
  } else if constexpr (OP == LANE_ZERO_Q) {
    for (int64_t i = i0; i < nd; i += stride) L.q[i] = 0.0;
  } else if constexpr (OP == LANE_NEWMARK) {
    newmark_body(nd, L.dt, L.x, L.u, L.v, L.a, L.hist + (int64_t)((L.hist_head + 1) & 3) * nd);
  } else if constexpr (OP == LANE_RECORD) {
    double* row = L.wave + L.step * 3 * (int64_t)L.n_rec;
    for (int64_t i = i0; i < 3 * (int64_t)L.n_rec; i += stride) row[i] = L.v[3 * (int64_t)L.rec[i / 3] + i % 3];
    if (lead && st != nullptr) {
      L.log_it[L.step] = st[l].iters;
      L.log_rel[L.step] = st[l].rel;
    }
  } else if constexpr (OP == LANE_GATHER) {
    if (lead) {
      LaneInfo o;
      o.bb = L.ctl64->bb;
      o.rr_true = L.ctl64->rr_true;
      o.rr0 = slot_sum<NSLOT>(L.ctl64->rr[0]);
      o.done64 = L.ctl64->done;
      o.iters64 = L.ctl64->iters;
      o.done32 = L.ctl32 ? L.ctl32->done : 0;
      o.iters32 = L.ctl32 ? L.ctl32->iters : 0;
      info[l] = o;
    }
  }
}

// CG update (DIR false) or direction (DIR true) kernel of iteration `iter`
// of every active lane's current solve (FP32 inner or FP64).
// dev_index: the iteration's index in the step comes from each lane's
// control block (graph replays), not from iter_base + iter.
template <typename T, bool DIR>
__global__ __launch_bounds__(TPB) void k_lane_cg(const LaneDev* __restrict__ lanes, const LaneState* __restrict__ st,
                                                 int iter, int dev_index) {
  const int l = blockIdx.y;
  if (!st[l].active) return;
  const LaneDev& L = lanes[l];
  const int par = iter & 1;
  const int iabs = dev_index ? -1 : st[l].iter_base + iter;
  if constexpr (sizeof(T) == 4) {
    if constexpr (DIR)
      cg_dir_body<float>(L.n_nodes, par, iabs, L.max_iter, L.z32, L.p32, L.d32, L.ctl32);
    else
      cg_update_body<float, __half>(L.n_nodes, L.n_interior, par, L.pinv16, L.r32, L.z32, L.q32, L.ctl32);
  } else {
    if constexpr (DIR)
      cg_dir_body<double>(L.n_nodes, par, iabs, L.max_iter, L.z, L.p, L.x, L.ctl64);
    else
      cg_update_body<double, double>(L.n_nodes, 0, par, L.pinv64, L.r, L.z, L.q, L.ctl64);
  }
}

// Blocks per lane: enough in total to fill the chip several times over,
// never more than the largest lane needs.
static unsigned lane_blocks(int n_lanes, int64_t max_items, unsigned total_cap) {
  unsigned per = total_cap / (unsigned)(n_lanes > 0 ? n_lanes : 1);
  if (per < 32) per = 32;
  const unsigned need = nblocks(max_items);
  if (per > need) per = need;
  return per == 0 ? 1 : per;
}

void launch_lanes(LaneOp op, int n_lanes, int64_t max_nodes, const LaneDev* lanes, const LaneState* st,
                  LaneInfo* info, hipStream_t s) {
  if (n_lanes <= 0) return;
  const unsigned bn = lane_blocks(n_lanes, max_nodes, 2048);       // node loops (dot products into slots)
  const unsigned bd = lane_blocks(n_lanes, 3 * max_nodes, 8192);   // DOF loops
  switch (op) {
#define SW_LANE_CASE(OP, BX)                                                                          \
  case OP:                                                                                            \
    hipLaunchKernelGGL(k_lane_op<OP>, dim3(BX, n_lanes), dim3(TPB), 0, s, lanes, st, info);           \
    break;
    SW_LANE_CASE(LANE_BEGIN_STEP, bd)
    SW_LANE_CASE(LANE_NORM2_B, bd)
    SW_LANE_CASE(LANE_PREPARE64, 1)
    SW_LANE_CASE(LANE_GUESS, bd)
    SW_LANE_CASE(LANE_RRTRUE_RESET, 1)
    SW_LANE_CASE(LANE_TRUE_RES, bd)
    SW_LANE_CASE(LANE_TO_F32, bd)
    SW_LANE_CASE(LANE_CG_INIT32, bn)
    SW_LANE_CASE(LANE_CG_INIT64, bn)
    SW_LANE_CASE(LANE_IR_UPDATE, bd)
    SW_LANE_CASE(LANE_ZERO_Q, bd)
    SW_LANE_CASE(LANE_NEWMARK, bd)
    SW_LANE_CASE(LANE_RECORD, 8)
    SW_LANE_CASE(LANE_GATHER, 1)
#undef SW_LANE_CASE
  }
}

void launch_lanes_cg(bool f32, bool dir, int n_lanes, int64_t max_nodes, const LaneDev* lanes, const LaneState* st,
                     int iter, hipStream_t s, bool dev_index) {
  const unsigned bn = lane_blocks(n_lanes, max_nodes, 2048);
  const dim3 g(bn, n_lanes);
  const int dv = dev_index ? 1 : 0;
  if (f32) {
    if (dir)
      hipLaunchKernelGGL((k_lane_cg<float, true>), g, dim3(TPB), 0, s, lanes, st, iter, dv);
    else
      hipLaunchKernelGGL((k_lane_cg<float, false>), g, dim3(TPB), 0, s, lanes, st, iter, dv);
  } else {
    if (dir)
      hipLaunchKernelGGL((k_lane_cg<double, true>), g, dim3(TPB), 0, s, lanes, st, iter, dv);
    else
      hipLaunchKernelGGL((k_lane_cg<double, false>), g, dim3(TPB), 0, s, lanes, st, iter, dv);
  }
}

}  // namespace sw
