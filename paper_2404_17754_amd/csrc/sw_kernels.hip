// HIP kernels (gfx950) of the implicit wave-propagation step: matrix-free
// element-by-element operator, boundary faces, 3x3 block-Jacobi
// preconditioner, fused CG vector updates with wavefront reductions, Newmark
// update, receiver recording and the ERR misfit of Eq. (eqerr).
//
// Every vector is node-major [node][3].  One work-item handles one tet, one
// face or one node; partial dot products are reduced across the 64-wide
// wavefront with shuffles, across the workgroup through LDS, and across the
// grid with one FP64 atomic per workgroup into a device control block.
#include <hip/hip_runtime.h>

#include "sw_elem.h"
#include "sw_internal.h"

namespace sw {

constexpr int TPB = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the workgroup, returned on thread 0 (TPB threads).
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

// ------------------------------------------------------------ EBE operator

// Iteration-mode protocol (par >= 0): the kernel returns at once when the
// solve is done; on the first iteration it also ends a solve whose initial
// residual already meets the tolerance; workgroup 0 clears the scalar slots
// that the next update kernel accumulates into.  par < 0: plain application.
template <typename T, int MODE>
__global__ __launch_bounds__(TPB) void k_ebe(MeshDev m, const uint8_t* __restrict__ tet_mat,
                                             const MatDev* __restrict__ mats, T sM, T sK,
                                             const T* __restrict__ x, T* __restrict__ y,
                                             const double* __restrict__ u, const double* __restrict__ v,
                                             const double* __restrict__ a, double c1, double bR, CgCtl* ctl,
                                             int iter) {
  __shared__ double sh[2 * TPB / 64];
  const int par = iter & 1, first_iter = iter == 0;
  if (iter >= 0) {
    if (ctl->done) return;
    if (first_iter && ctl->rr[0] <= ctl->tol2) {
      if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done = 1;
      return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->rz[par ^ 1] = 0.0;
      ctl->rr[par ^ 1] = 0.0;
    }
  }
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double energy = 0.0;
  if (e < m.n_tets) {
    int nd[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) nd[k] = m.conn[k * m.tet_stride + e];
    double X[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int d = 0; d < 3; ++d) X[k][d] = m.xyz[3 * (int64_t)nd[k] + d];
    }
    Geo<T> G;
    tet_geometry<T>(X, G);
    const MatDev mt = mats[tet_mat[e]];
    T out[10][3];
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k][0] = out[k][1] = out[k][2] = (T)0;
    if (MODE == EBE_APPLY) {
      T w[10][3];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) w[k][c] = x[3 * (int64_t)nd[k] + c];
      }
      stiffness_apply<T>(G, (T)mt.lam, (T)mt.mu, sK, w, out);
      mass_apply<T>((T)mt.rho * G.vol, sM, w, out);
      if (ctl != nullptr) {
#pragma unroll
        for (int k = 0; k < 10; ++k) {
#pragma unroll
          for (int c = 0; c < 3; ++c) energy += (double)w[k][c] * (double)out[k][c];
        }
      }
    } else {
      T w1[10][3], w2[10][3];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int64_t i = 3 * (int64_t)nd[k] + c;
          const double vv = v[i];
          w1[k][c] = (T)(a[i] + c1 * vv);
          w2[k][c] = (T)(u[i] - bR * vv);
        }
      }
      stiffness_apply<T>(G, (T)mt.lam, (T)mt.mu, (T)-1, w2, out);
      mass_apply<T>((T)mt.rho * G.vol, (T)1, w1, out);
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) atomic_add(&y[3 * (int64_t)nd[k] + c], out[k][c]);
    }
  }
  if (ctl != nullptr && MODE == EBE_APPLY) {
    double t = block_sum(energy, sh);
    if (threadIdx.x == 0) atomic_add(&ctl->pAp, t);
  }
}

void launch_ebe_apply_f64(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sM, double sK,
                          const double* x, double* y, CgCtl* ctl, int iter, hipStream_t s) {
  hipLaunchKernelGGL((k_ebe<double, EBE_APPLY>), dim3(nblocks(m.n_tets)), dim3(TPB), 0, s, m, tet_mat, mats, sM, sK,
                     x, y, nullptr, nullptr, nullptr, 0.0, 0.0, ctl, iter);
}
void launch_ebe_apply_f32(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sM, double sK,
                          const float* x, float* y, CgCtl* ctl, int iter, hipStream_t s) {
  hipLaunchKernelGGL((k_ebe<float, EBE_APPLY>), dim3(nblocks(m.n_tets)), dim3(TPB), 0, s, m, tet_mat, mats,
                     (float)sM, (float)sK, x, y, nullptr, nullptr, nullptr, 0.0, 0.0, ctl, iter);
}
void launch_ebe_rhs(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double c1, double bR,
                    const double* u, const double* v, const double* a, double* y, hipStream_t s) {
  hipLaunchKernelGGL((k_ebe<double, EBE_RHS>), dim3(nblocks(m.n_tets)), dim3(TPB), 0, s, m, tet_mat, mats, 1.0, -1.0,
                     (const double*)nullptr, y, u, v, a, c1, bR, (CgCtl*)nullptr, -1);
}

// ------------------------------------------------------------------ faces

template <typename T, int MODE>
__global__ __launch_bounds__(TPB) void k_face(MeshDev m, const uint8_t* __restrict__ tet_mat,
                                              const MatDev* __restrict__ mats, T sc, const T* __restrict__ x,
                                              T* __restrict__ y, CgCtl* ctl, const double* __restrict__ vin3) {
  __shared__ double sh[2 * TPB / 64];
  if (ctl != nullptr && ctl->done) return;
  const int64_t f = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double energy = 0.0;
  if (f < m.n_faces) {
    int nd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) nd[k] = m.fconn[k * m.face_stride + f];
    double P[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int d = 0; d < 3; ++d) P[k][d] = m.xyz[3 * (int64_t)nd[k] + d];
    }
    const FaceGeo g = face_geometry(P);
    const MatDev mt = mats[tet_mat[m.face_tet[f]]];
    T w[6][3], out[6][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[k][c] = x[3 * (int64_t)nd[k] + c];
        out[k][c] = (T)0;
      }
    }
    const T n[3] = {(T)g.n[0], (T)g.n[1], (T)g.n[2]};
    face_dashpot_apply<T>(n, (T)g.area, (T)mt.zp, (T)mt.zs, sc, w, out);
    if (MODE == EBE_RHS && m.face_role[f] == 2) {
      // incident wave: traction 2 Z v_in, consistent load A/3 on edge nodes
      const double vi[3] = {vin3[0], vin3[1], vin3[2]};
      const double nv = g.n[0] * vi[0] + g.n[1] * vi[1] + g.n[2] * vi[2];
      const double w3 = g.area / 3.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double t = 2.0 * (mt.zs * vi[c] + (mt.zp - mt.zs) * nv * g.n[c]);
        out[3][c] += (T)(w3 * t);
        out[4][c] += (T)(w3 * t);
        out[5][c] += (T)(w3 * t);
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        atomic_add(&y[3 * (int64_t)nd[k] + c], out[k][c]);
        energy += (double)w[k][c] * (double)out[k][c];
      }
    }
  }
  if (ctl != nullptr) {
    double t = block_sum(energy, sh);
    if (threadIdx.x == 0) atomic_add(&ctl->pAp, t);
  }
}

void launch_face_apply_f64(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sc,
                           const double* x, double* y, CgCtl* ctl, hipStream_t s) {
  if (m.n_faces == 0) return;
  hipLaunchKernelGGL((k_face<double, EBE_APPLY>), dim3(nblocks(m.n_faces)), dim3(TPB), 0, s, m, tet_mat, mats, sc, x,
                     y, ctl, (const double*)nullptr);
}
void launch_face_apply_f32(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sc,
                           const float* x, float* y, CgCtl* ctl, hipStream_t s) {
  if (m.n_faces == 0) return;
  hipLaunchKernelGGL((k_face<float, EBE_APPLY>), dim3(nblocks(m.n_faces)), dim3(TPB), 0, s, m, tet_mat, mats,
                     (float)sc, x, y, ctl, (const double*)nullptr);
}
void launch_face_rhs(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, const double* v,
                     const double* vin3, double* y, hipStream_t s) {
  if (m.n_faces == 0) return;
  hipLaunchKernelGGL((k_face<double, EBE_RHS>), dim3(nblocks(m.n_faces)), dim3(TPB), 0, s, m, tet_mat, mats, 1.0, v,
                     y, (CgCtl*)nullptr, vin3);
}

// --------------------------------------------------------- block Jacobi

__global__ __launch_bounds__(TPB) void k_diag_elem(MeshDev m, const uint8_t* __restrict__ tet_mat,
                                                   const MatDev* __restrict__ mats, double cM, double cK,
                                                   double* __restrict__ diag6) {
  const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= m.n_tets) return;
  int nd[10];
  for (int k = 0; k < 10; ++k) nd[k] = m.conn[k * m.tet_stride + e];
  double X[4][3];
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < 3; ++d) X[k][d] = m.xyz[3 * (int64_t)nd[k] + d];
  Geo<double> G;
  tet_geometry<double>(X, G);
  const MatDev mt = mats[tet_mat[e]];
  double out[10][6];
  diag_blocks<double>(G, mt.lam, mt.mu, mt.rho, cM, cK, out);
  for (int k = 0; k < 10; ++k)
    for (int j = 0; j < 6; ++j) atomic_add(&diag6[6 * (int64_t)nd[k] + j], out[k][j]);
}

__global__ __launch_bounds__(TPB) void k_diag_face(MeshDev m, const uint8_t* __restrict__ tet_mat,
                                                   const MatDev* __restrict__ mats, double cC,
                                                   double* __restrict__ diag6) {
  const int64_t f = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (f >= m.n_faces) return;
  int nd[6];
  for (int k = 0; k < 6; ++k) nd[k] = m.fconn[k * m.face_stride + f];
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) P[k][d] = m.xyz[3 * (int64_t)nd[k] + d];
  const FaceGeo g = face_geometry(P);
  const MatDev mt = mats[tet_mat[m.face_tet[f]]];
  const double dz = mt.zp - mt.zs;
  const double Z[6] = {mt.zs + dz * g.n[0] * g.n[0], mt.zs + dz * g.n[1] * g.n[1], mt.zs + dz * g.n[2] * g.n[2],
                       dz * g.n[1] * g.n[2],         dz * g.n[0] * g.n[2],         dz * g.n[0] * g.n[1]};
  for (int k = 0; k < 6; ++k) {
    const double s = cC * g.area / 180.0 * (k < 3 ? 6.0 : 32.0);
    for (int j = 0; j < 6; ++j) atomic_add(&diag6[6 * (int64_t)nd[k] + j], s * Z[j]);
  }
}

__global__ __launch_bounds__(TPB) void k_invert(int64_t n, const double* __restrict__ d6, double* __restrict__ p64,
                                                float* __restrict__ p32, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const double a = d6[6 * i + 0], b = d6[6 * i + 1], c = d6[6 * i + 2];
  const double yz = d6[6 * i + 3], xz = d6[6 * i + 4], xy = d6[6 * i + 5];
  // inverse of [[a xy xz][xy b yz][xz yz c]] by cofactors
  const double c00 = b * c - yz * yz, c11 = a * c - xz * xz, c22 = a * b - xy * xy;
  const double c12 = -(a * yz - xy * xz), c02 = xy * yz - b * xz, c01 = -(xy * c - yz * xz);
  const double det = a * c00 + xy * c01 + xz * c02;
  if (!(det > 0.0) || !(a > 0.0)) {
    *bad = 1;
  }
  const double id = 1.0 / det;
  const double r[6] = {c00 * id, c11 * id, c22 * id, c12 * id, c02 * id, c01 * id};
  for (int k = 0; k < 6; ++k) {
    p64[6 * i + k] = r[k];
    p32[6 * i + k] = (float)r[k];
  }
}

void launch_diag_blocks(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double cM, double cK,
                        double cC, double* diag6, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_elem, dim3(nblocks(m.n_tets)), dim3(TPB), 0, s, m, tet_mat, mats, cM, cK, diag6);
  if (m.n_faces)
    hipLaunchKernelGGL(k_diag_face, dim3(nblocks(m.n_faces)), dim3(TPB), 0, s, m, tet_mat, mats, cC, diag6);
}
void launch_invert_blocks(int64_t n_nodes, const double* diag6, double* pinv64, float* pinv32, int* bad,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(nblocks(n_nodes)), dim3(TPB), 0, s, n_nodes, diag6, pinv64, pinv32, bad);
}

// --------------------------------------------------------- CG vector ops

template <typename T>
__device__ __forceinline__ void bj_apply(const T* __restrict__ P, int64_t i, const T r[3], T z[3]) {
  const T a = P[6 * i + 0], b = P[6 * i + 1], c = P[6 * i + 2];
  const T yz = P[6 * i + 3], xz = P[6 * i + 4], xy = P[6 * i + 5];
  z[0] = a * r[0] + xy * r[1] + xz * r[2];
  z[1] = xy * r[0] + b * r[1] + yz * r[2];
  z[2] = xz * r[0] + yz * r[1] + c * r[2];
}

// r = b - q, z = P r, p = z, q = 0; rz[0], rr[0]
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_init(int64_t n, const T* __restrict__ b, const T* __restrict__ q,
                                                 const T* __restrict__ P, T* __restrict__ r, T* __restrict__ z,
                                                 T* __restrict__ p, T* __restrict__ qz, CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    T rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = b[3 * i + c] - (q ? q[3 * i + c] : (T)0);
    bj_apply<T>(P, i, rv, zv);
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
    atomic_add(&ctl->rz[0], rz);
    atomic_add(&ctl->rr[0], rr);
  }
}

// alpha = rz[par] / pAp; x += alpha p; r -= alpha q; z = P r; q = 0;
// rz[par^1] += r.z, rr[par^1] += r.r
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_update(int64_t n, int par, const T* __restrict__ P, T* __restrict__ x,
                                                   T* __restrict__ r, T* __restrict__ z, const T* __restrict__ p,
                                                   T* __restrict__ q, CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  if (ctl->done) return;
  const T alpha = (T)(ctl->rz[par] / ctl->pAp);
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    T rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * i + c;
      x[k] += alpha * p[k];
      rv[c] = r[k] - alpha * q[k];
      q[k] = (T)0;
    }
    bj_apply<T>(P, i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[3 * i + c] = rv[c];
      z[3 * i + c] = zv[c];
      rz += (double)rv[c] * (double)zv[c];
      rr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(rz, rr, sh);
  if (threadIdx.x == 0) {
    atomic_add(&ctl->rz[par ^ 1], rz);
    atomic_add(&ctl->rr[par ^ 1], rr);
  }
}

// convergence test, then p = z + beta p with beta = rz[par^1] / rz[par]
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_dir(int64_t n, int par, int iter_abs, int max_iter,
                                                const T* __restrict__ z, T* __restrict__ p, CgCtl* ctl) {
  if (ctl->done) return;
  const double rr = ctl->rr[par ^ 1];
  const bool stop = !(rr > ctl->tol2) || (iter_abs + 1 >= max_iter);  // NaN stops too
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->iters = iter_abs + 1;
    if (stop) ctl->done = 1;
    ctl->pAp = 0.0;
  }
  if (stop) return;
  const T beta = (T)(ctl->rz[par ^ 1] / ctl->rz[par]);
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) {
#pragma unroll
    for (int c = 0; c < 3; ++c) p[3 * i + c] = z[3 * i + c] + beta * p[3 * i + c];
  }
}

void launch_cg_init_f64(int64_t n, const double* b, const double* q, const double* P, double* r, double* z, double* p,
                        double* qz, CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init<double>, dim3(nblocks(n)), dim3(TPB), 0, s, n, b, q, P, r, z, p, qz, ctl);
}
void launch_cg_init_f32(int64_t n, const float* b, const float* q, const float* P, float* r, float* z, float* p,
                        float* qz, CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init<float>, dim3(nblocks(n)), dim3(TPB), 0, s, n, b, q, P, r, z, p, qz, ctl);
}
void launch_cg_update_f64(int64_t n, int par, const double* P, double* x, double* r, double* z, const double* p,
                          double* q, CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update<double>, dim3(nblocks(n)), dim3(TPB), 0, s, n, par, P, x, r, z, p, q, ctl);
}
void launch_cg_update_f32(int64_t n, int par, const float* P, float* x, float* r, float* z, const float* p, float* q,
                          CgCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update<float>, dim3(nblocks(n)), dim3(TPB), 0, s, n, par, P, x, r, z, p, q, ctl);
}
void launch_cg_dir_f64(int64_t n, int par, int iter_abs, int max_iter, const double* z, double* p, CgCtl* ctl,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir<double>, dim3(nblocks(n)), dim3(TPB), 0, s, n, par, iter_abs, max_iter, z, p, ctl);
}
void launch_cg_dir_f32(int64_t n, int par, int iter_abs, int max_iter, const float* z, float* p, CgCtl* ctl,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir<float>, dim3(nblocks(n)), dim3(TPB), 0, s, n, par, iter_abs, max_iter, z, p, ctl);
}

// ------------------------------------------------------------ scalars

__global__ void k_ctl_prepare(CgCtl* ctl, double rtol, int clear_bb) {
  if (threadIdx.x != 0) return;
  if (clear_bb) ctl->bb = 0.0;
  ctl->tol2 = rtol * rtol * ctl->bb;
  ctl->pAp = 0.0;
  ctl->rz[0] = ctl->rz[1] = 0.0;
  ctl->rr[0] = ctl->rr[1] = 0.0;
  ctl->rr_true = 0.0;
  ctl->done = 0;
  ctl->iters = 0;
}
void launch_ctl_prepare(CgCtl* ctl, double rtol, int clear_bb, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_prepare, dim3(1), dim3(64), 0, s, ctl, rtol, clear_bb);
}

__global__ __launch_bounds__(TPB) void k_norm2(int64_t n, const double* __restrict__ x, double* out) {
  __shared__ double sh[2 * TPB / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) acc += x[i] * x[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) atomic_add(out, acc);
}
void launch_norm2(int64_t n, const double* x, double* out, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 4096) g = 4096;
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
void launch_true_residual(int64_t n, const double* b, const double* q, double* r, CgCtl* ctl, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_true_res, dim3(g), dim3(TPB), 0, s, n, b, q, r, ctl);
}

__global__ __launch_bounds__(TPB) void k_to_f32(int64_t n, const double* __restrict__ r, float* __restrict__ r32,
                                                CgCtl* ctl) {
  const double nr = sqrt(ctl->rr_true);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->scale = nr;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
    r32[i] = (float)(r[i] * inv);
}
void launch_to_f32_scaled(int64_t n, const double* r64, float* r32, CgCtl* ctl, hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(TPB), 0, s, n, r64, r32, ctl);
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

// ------------------------------------------------------------- guesses

// Lagrange extrapolation of order p from the last p+1 increments:
// x = sum_j (-1)^j C(p+1, j+1) hist[head - j]
__global__ __launch_bounds__(TPB) void k_guess_poly(int64_t n, const double* __restrict__ hist, int head, int order,
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
void launch_guess_poly(int64_t n, const double* hist, int head, int order, double* x, const CgCtl* ctl,
                       hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_guess_poly, dim3(g), dim3(TPB), 0, s, n, hist, head, order, x, ctl);
}

// ------------------------------------------------------------ Newmark

__global__ __launch_bounds__(TPB) void k_newmark(int64_t n, double dt, const double* __restrict__ du,
                                                 double* __restrict__ u, double* __restrict__ v,
                                                 double* __restrict__ a, double* __restrict__ hist) {
  const double c2 = 2.0 / dt, c4 = 4.0 / (dt * dt), c4v = 4.0 / dt;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double d = du[i], vo = v[i];
    u[i] += d;
    v[i] = c2 * d - vo;
    a[i] = c4 * d - c4v * vo - a[i];
    if (hist) hist[i] = d;
  }
}
void launch_newmark(int64_t n, double dt, const double* du, double* u, double* v, double* a, double* hist_slot,
                    hipStream_t s) {
  unsigned g = nblocks(n);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_newmark, dim3(g), dim3(TPB), 0, s, n, dt, du, u, v, a, hist_slot);
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

__global__ void k_step_log(const CgCtl* ctl, int32_t* it, double* rel, int32_t* total) {
  if (threadIdx.x != 0) return;
  *it = ctl->iters;
  *rel = ctl->bb > 0.0 ? sqrt(ctl->rr_true / ctl->bb) : 0.0;
  if (total) *total += ctl->iters;
}
void launch_step_log(const CgCtl* ctl, int32_t* it, double* rel, int32_t* total, hipStream_t s) {
  hipLaunchKernelGGL(k_step_log, dim3(1), dim3(64), 0, s, ctl, it, rel, total);
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

}  // namespace sw
