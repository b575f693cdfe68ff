// Internal structures shared by the runtime (sw_api.cpp) and the kernels
// (sw_kernels.hip).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

// Per-material constants on the device.
struct MatDev {
  double lam, mu, rho, zp, zs;  // Lame constants, density, rho*Vp, rho*Vs
};

// Device-resident control block of one CG solve (one per case, FP64 scalars
// whatever the vector precision).  Kernels accumulate the dot products into
// it and decide convergence from it, so a chunk of iterations runs without
// the host.
struct CgCtl {
  double pAp;      // p . A p (element energies)
  double rz[2];    // r . z, ring indexed by iteration parity
  double rr[2];    // r . r, same ring
  double bb;       // ||b||^2 of the FP64 right-hand side
  double tol2;     // stop when rr <= tol2
  double rr_true;  // ||b - A x||^2 recomputed in FP64
  double scale;    // mixed precision: residual scaling of the inner system
  int32_t done;    // 1 once converged or capped
  int32_t iters;   // iterations of the current solve
  int32_t pad[2];
};

// Mesh in device memory.
struct MeshDev {
  int64_t n_nodes, n_tets, n_faces;
  int64_t tet_stride;        // padded n_tets: conn[a * tet_stride + e]
  const int32_t* conn;       // [10][tet_stride]
  const double* xyz;         // [n_nodes][3]
  const int32_t* fconn;      // [6][face_stride]
  int64_t face_stride;
  const int32_t* face_tet;   // [n_faces]
  const uint8_t* face_role;  // [n_faces]
};

// ---- launch wrappers implemented in sw_kernels.hip -----------------------

enum EbeMode { EBE_APPLY = 0, EBE_RHS = 1 };

// y += sM M x + sK K x.  iter >= 0: CG iteration `iter` of the solve in ctl
// (early exit when done, p.Ap accumulated into ctl); iter < 0: plain apply.
void launch_ebe_apply_f64(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sM, double sK,
                          const double* x, double* y, CgCtl* ctl, int iter, hipStream_t s);
void launch_ebe_apply_f32(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sM, double sK,
                          const float* x, float* y, CgCtl* ctl, int iter, hipStream_t s);
// y += M (a + c1 v) - K (u - bR v)
void launch_ebe_rhs(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double c1, double bR,
                    const double* u, const double* v, const double* a, double* y, hipStream_t s);
// y += s C_abs x (+ energy)
void launch_face_apply_f64(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sc,
                           const double* x, double* y, CgCtl* ctl, hipStream_t s);
void launch_face_apply_f32(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double sc,
                           const float* x, float* y, CgCtl* ctl, hipStream_t s);
// y += C_abs v + F(v_in) on base faces
void launch_face_rhs(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, const double* v,
                     const double* vin3, double* y, hipStream_t s);

void launch_diag_blocks(const MeshDev& m, const uint8_t* tet_mat, const MatDev* mats, double cM, double cK,
                        double cC, double* diag6, hipStream_t s);
void launch_invert_blocks(int64_t n_nodes, const double* diag6, double* pinv64, float* pinv32, int* bad,
                          hipStream_t s);

// CG vector kernels, T = double or float vectors; pinv in matching precision
void launch_cg_init_f64(int64_t n_nodes, const double* b, const double* q, const double* pinv, double* r, double* z,
                        double* p, double* qz, CgCtl* ctl, hipStream_t s);
void launch_cg_init_f32(int64_t n_nodes, const float* b, const float* q, const float* pinv, float* r, float* z,
                        float* p, float* qz, CgCtl* ctl, hipStream_t s);
void launch_cg_update_f64(int64_t n_nodes, int par, const double* pinv, double* x, double* r, double* z,
                          const double* p, double* q, CgCtl* ctl, hipStream_t s);
void launch_cg_update_f32(int64_t n_nodes, int par, const float* pinv, float* x, float* r, float* z,
                          const float* p, float* q, CgCtl* ctl, hipStream_t s);
void launch_cg_dir_f64(int64_t n_nodes, int par, int iter_abs, int max_iter, const double* z, double* p,
                       CgCtl* ctl, hipStream_t s);
void launch_cg_dir_f32(int64_t n_nodes, int par, int iter_abs, int max_iter, const float* z, float* p,
                       CgCtl* ctl, hipStream_t s);

// ctl setup: bb = ||b||^2 must already be in ctl; sets tol2 = rtol^2 bb and clears the rest
void launch_ctl_prepare(CgCtl* ctl, double rtol, int clear_bb, hipStream_t s);
void launch_norm2(int64_t n, const double* x, double* out, hipStream_t s);

// mixed precision glue
// r64 = b - q64, rr_true -> ctl; also r32 = r64 / ||r64|| once the norm is known (second kernel)
void launch_true_residual(int64_t n, const double* b, const double* q, double* r, CgCtl* ctl, hipStream_t s);
void launch_to_f32_scaled(int64_t n, const double* r64, float* r32, CgCtl* ctl, hipStream_t s);
void launch_ir_update(int64_t n, double* x64, const float* d32, const CgCtl* ctl, hipStream_t s);

// initial guess: x = sum_j coef[j] hist[(head - j) mod 4]; zero if ctl->bb == 0
void launch_guess_poly(int64_t n, const double* hist, int head, int order, double* x, const CgCtl* ctl,
                       hipStream_t s);

// Newmark update, history push, receiver record, step log
void launch_newmark(int64_t n, double dt, const double* du, double* u, double* v, double* a, double* hist_slot,
                    hipStream_t s);
void launch_record(int n_rec, const int32_t* rec, const double* v, double* wave_row, hipStream_t s);
void launch_step_log(const CgCtl* ctl, int32_t* iters_out, double* relres_out, int32_t* iter_total, hipStream_t s);

// misfit: per-pair sums then the mean
void launch_misfit(int n_rec, int64_t n_steps, const double* U, const double* obs, double* pair_buf,
                   double* out2, hipStream_t s);

void launch_fill_f64(int64_t n, double* x, double val, hipStream_t s);
void launch_fill_f32(int64_t n, float* x, float val, hipStream_t s);

}  // namespace sw
