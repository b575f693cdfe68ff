// Internal structures shared by the runtime (sw_api.cpp) and the kernels
// (sw_kernels.hip).  Not part of the C-ABI.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

// Per-material constants on the device.
struct MatDev {
  double lam, mu, rho, zp, zs;  // Lame constants, density, rho*Vp, rho*Vs
};

// Device-resident control block of one CG solve (FP64 scalars whatever the
// vector precision).  Kernels accumulate the dot products into it and decide
// convergence from it, so a chunk of iterations runs without the host.  Each
// dot product is spread over NSLOT partial sums (workgroup w adds into slot
// w mod NSLOT) so that thousands of workgroups do not serialise on one
// address; readers add the slots up.
constexpr int NSLOT = 32;
struct CgCtl {
  double pAp[NSLOT];     // p . A p (element energies)
  double rz[2][NSLOT];   // r . z, ring indexed by iteration parity
  double rr[2][NSLOT];   // r . r, same ring
  double bb;       // ||b||^2 of the right-hand side
  double tol2;     // stop when rr <= tol2
  double rr_true;  // ||b - A x||^2 recomputed in FP64
  double scale;    // mixed precision: residual scaling of the inner system
  double alpha;    // step length of the last update kernel's iteration
  int32_t done;    // 1 once converged or capped
  int32_t iters;   // iterations of the current solve
  int32_t live;    // 1 when the last update kernel ran its iteration (the
                   // direction kernel after it applies x += alpha p)
  int32_t iter_cur;  // the running iteration's index in the step (written by the
                     // update kernel, read by the direction kernel launched with
                     // iter_abs < 0, as in a captured graph of iterations)
};

// Tiled mesh in device memory (internal element and node numbering; see
// sw_layout.h).
struct MeshDev {
  int64_t n_nodes, n_tets, n_faces;
  int64_t n_interior;            // nodes [0, n_interior) belong to one tile each
  int32_t n_tiles, max_tile_nodes;
  int64_t tet_stride, face_stride;
  const uint16_t* conn_loc;      // [10][tet_stride], 3 x tile-local node index
  const int32_t* tile_elem_off;  // [n_tiles + 1]
  const int32_t* tile_node_off;  // [n_tiles + 1]
  const int32_t* tile_nodes;
  const int32_t* tile_int_base;
  const int32_t* tile_nint;
  const int32_t* tile_face_off;  // [n_tiles + 1]
  const double* xyz;             // [n_nodes][3]
  const float* geo32;            // [10][tet_stride]: FP32 grad L1..L3 (9) and volume
  const double* geo64;           // [10][tet_stride]: the same in FP64
  const int32_t* fconn;          // [6][face_stride]
  const uint16_t* fconn_loc;     // [6][face_stride]
  const int32_t* face_elem;      // [n_faces]
  const uint8_t* face_role;      // [n_faces]
  const int32_t* node_u2i;       // [n_nodes]
  const int32_t* node_i2u;       // [n_nodes]
  const float* inv_valence;      // [n_nodes] 1 / number of elements containing the node
  // deterministic passes (null unless the mesh was created for them): per
  // node, the element slots e * 10 + k and face slots f * 6 + k touching it,
  // in increasing order
  const int32_t* inc_off;        // [n_nodes + 1]
  const int32_t* inc;
  const int32_t* finc_off;       // [n_nodes + 1]
  const int32_t* finc;
};

// One tiled operator pass:
//   y (=|+=) sM M xe + sK K xe + sC C_abs xf + F(vin)
// with xe = a1 x1 + a2 x2 (x2 optional) gathered into LDS per tile, xf read
// by the face work-items, F the base input force when vin != nullptr.
template <typename T>
struct TileArgs {
  T sM, sK, sC;
  const T* x1;
  // FP32 passes of the SW_MIXED_FP16 inner CG: the input in bfloat16 in
  // place of x1 (a1 = 1, no x2); null otherwise
  const uint16_t* x1h;
  const T* x2;
  T a1, a2;
  const T* xf;
  const double* vin;   // 3 values or nullptr
  T* y;
  int accumulate;      // interior nodes: 0 overwrite, 1 add
  int n_mat;           // materials in the table (0: not given)
  // deterministic FP64 passes: each element's 10 x 3 results and each
  // face's 6 x 3 go here (slot-major), then every node sums its slots in
  // increasing order (null: LDS and global atomics, arrival order)
  double* eout;
  double* fout;
};

// ---- several cases marched together (lanes) ------------------------------

// One lane's operator pass: the lane's mesh, materials, pass arguments and,
// in CG iterations, its control block.
template <typename T>
struct TileLane {
  MeshDev m;
  const uint8_t* emat;
  const MatDev* mats;
  TileArgs<T> A;
  CgCtl* ctl;
};

// One lane's vectors and per-step values (internal node order of its mesh).
struct LaneDev {
  int64_t n_nodes;
  int64_t n_interior;       // q is cleared only past the interior nodes
  double dt;
  double *u, *v, *a, *b, *x, *r, *z, *p, *q;
  double* hist;             // [4][3 n_nodes] increments, ring
  const double* pinv64;
  const __half* pinv16;
  float *r32, *d32, *z32, *p32, *q32;
  CgCtl *ctl64, *ctl32;
  const int32_t* rec;
  double* wave;             // [n_steps][n_rec][3]
  int32_t* log_it;
  double* log_rel;
  double rtol;
  int64_t step;             // the step being solved goes from `step` to `step + 1`
  int32_t n_rec;
  int32_t hist_head;        // ring slot of the newest increment
  int32_t guess_order;      // >= 0: extrapolation order; -1: zero; -2: written by the network
  int32_t max_iter;
};

// Host decisions of the current phase, per lane.
struct LaneState {
  int32_t active;     // takes part in the current phase
  int32_t iter_base;  // CG iterations of this step before the current solve
  double tol;         // relative tolerance of the current inner solve
  double rel;         // the step's final true relative residual (log)
  int32_t iters;      // the step's CG iterations (log)
  int32_t zero_q;     // true residual: clear q after use
};

// What the host reads back after a phase, per lane.
struct LaneInfo {
  double bb, rr_true, rr0;
  int32_t done64, iters64, done32, iters32;
};

void launch_tile_lanes_f64(const TileLane<double>* lanes, const int2* work, int n_work, int max_tile_nodes,
                           const LaneState* st, int iter, hipStream_t s);
// FP32 CG-iteration pass of every lane, persistent and pipelined over items
// (lane, tile) listed tile-major with a tile's lanes adjacent; tiles of at
// most 1280 nodes.
void launch_tile_lanes_pipe_f32(const TileLane<float>* lanes, const int2* items, int n_items, int max_tile_nodes,
                                const LaneState* st, int iter, int grid_cap, hipStream_t s);

// Lane kernels (sw_kernels.hip): one launch covers every lane, grid
// (blocks per lane, lanes); st == nullptr means every lane.
enum LaneOp {
  LANE_BEGIN_STEP,   // b = 0, ctl64->bb = 0
  LANE_NORM2_B,      // ctl64->bb += b.b
  LANE_PREPARE64,    // ctl_prepare(ctl64, rtol)
  LANE_GUESS,        // x = extrapolation / zero (guess_order >= -1)
  LANE_RRTRUE_RESET, // ctl64->rr_true = 0
  LANE_TRUE_RES,     // r = b - q, rr_true; q = 0 when zero_q
  LANE_TO_F32,       // r32 = r / |r|, scale; ctl32 reset with tol; d32 = 0
  LANE_CG_INIT32,    // FP32 CG start on r32
  LANE_CG_INIT64,    // FP64 CG start on r = b - q (q cleared)
  LANE_IR_UPDATE,    // x += scale d32
  LANE_ZERO_Q,       // q = 0
  LANE_NEWMARK,      // Newmark update, increment ring
  LANE_RECORD,       // receivers, step log
  LANE_GATHER,       // LaneInfo of every lane
};
void launch_lanes(LaneOp op, int n_lanes, int64_t max_nodes, const LaneDev* lanes, const LaneState* st,
                  LaneInfo* info, hipStream_t s);
void launch_lanes_cg(bool f32, bool dir, int n_lanes, int64_t max_nodes, const LaneDev* lanes, const LaneState* st,
                     int iter, hipStream_t s, bool dev_index = false);

// Launches (sw_kernels.hip).  iter >= 0: CG iteration `iter` of the solve in
// ctl (early exit when done, p.Ap accumulated into ctl); iter < 0: plain.
// With a.eout set: the deterministic form (element and face results to
// a.eout / a.fout, a node pass summing them in slot order, p.Ap from a
// fixed-order dot product; the mesh needs its incidence lists).
void launch_tile_f64(const MeshDev& m, const uint8_t* emat, const MatDev* mats, const TileArgs<double>& a,
                     CgCtl* ctl, int iter, hipStream_t s);
// grid_cap > 0 limits the workgroups of the persistent FP32 pass (a multiple
// of 8); 0 keeps three per compute unit.
void launch_tile_f32(const MeshDev& m, const uint8_t* emat, const MatDev* mats, const TileArgs<float>& a,
                     CgCtl* ctl, int iter, int grid_cap, hipStream_t s);
// FP32 element geometry for the FP32 operator (once per mesh).
void launch_geom(const MeshDev& m, float* geo32, double* geo64, hipStream_t s);
// Diagonal 3x3 blocks (6 values per node) of cM M + cK K + cC C_abs.
// eout / fout set: the deterministic form (two passes of three values per
// node through the slot buffers, as launch_tile_f64).
void launch_tile_diag(const MeshDev& m, const uint8_t* emat, const MatDev* mats, double cM, double cK, double cC,
                      double* diag6, hipStream_t s, double* eout = nullptr, double* fout = nullptr);
// pinv64 = inverse blocks; pinv16 = the same divided by their largest
// diagonal entry (pmax, one double of scratch), in FP16 for the FP32 CG (a
// constant factor on the preconditioner leaves the CG iterates unchanged)
void launch_invert_blocks(int64_t n_nodes, const double* diag6, double* pinv64, __half* pinv16, double* pmax,
                          int* bad, hipStream_t s);

// CG vector kernels (node-parallel), T = double or float vectors.  det: one
// workgroup per scalar slot, so that each slot receives one workgroup's sum
// (a fixed-order reduction; fewer workgroups than the default grid).
void launch_cg_init_f64(int64_t n_nodes, const double* b, const double* q, const double* pinv, double* r, double* z,
                        double* p, double* qz, CgCtl* ctl, hipStream_t s, bool det = false);
void launch_cg_init_f32(int64_t n_nodes, const float* b, const float* q, const __half* pinv, float* r, float* z,
                        float* p, float* qz, CgCtl* ctl, hipStream_t s);
// update: r -= alpha q, z = P r, dot products; direction: x += alpha p,
// then p = z + beta p unless the solve stops (each iteration launches the
// update, then the direction kernel)
void launch_cg_update_f64(int64_t n_nodes, int par, const double* pinv, double* r, double* z, double* q, CgCtl* ctl,
                          hipStream_t s, bool det = false);
// q is cleared only for nodes >= n_interior (the next operator pass
// overwrites interior nodes)
void launch_cg_update_f32(int64_t n_nodes, int64_t n_interior, int par, const __half* pinv, float* r, float* z,
                          float* q, CgCtl* ctl, hipStream_t s);
void launch_cg_dir_f64(int64_t n_nodes, int par, int iter_abs, int max_iter, const double* z, double* p, double* x,
                       CgCtl* ctl, hipStream_t s);
void launch_cg_dir_f32(int64_t n_nodes, int par, int iter_abs, int max_iter, const float* z, float* p, float* x,
                       CgCtl* ctl, hipStream_t s);
// SW_MIXED_FP16 inner CG: the direction p16 in bfloat16 (FP32 arithmetic)
void launch_cg_dir_h(int64_t n_nodes, int par, int iter_abs, int max_iter, const float* z, uint16_t* p16, float* x,
                     CgCtl* ctl, hipStream_t s);

// ctl setup: bb must already be in ctl; sets tol2 = rtol^2 bb, clears the rest
void launch_ctl_prepare(CgCtl* ctl, double rtol, hipStream_t s);
// *out += x.x (det: one workgroup, a fixed-order sum)
void launch_norm2(int64_t n, const double* x, double* out, hipStream_t s, bool det = false);

// r = b - q, rr_true -> ctl (det: one workgroup)
void launch_true_residual(int64_t n, const double* b, const double* q, double* r, CgCtl* ctl, hipStream_t s,
                          bool det = false);
// r32 = r64 / ||r64|| (||r64|| from ctl->rr_true, kept in ctl->scale), z32 and
// the first direction (into p16 in bfloat16 when given, else p32), d32 = 0
void launch_ir_begin(int64_t n_nodes, const double* r64, const __half* P, float* r32, float* z32, float* p32,
                     uint16_t* p16, float* d32, CgCtl* ctl64, CgCtl* ctl32, hipStream_t s);
// x64 += ctl->scale * d32
void launch_ir_update(int64_t n, double* x64, const float* d32, const CgCtl* ctl, hipStream_t s);
// flexible outer CG (see sw_kernels.hip)
void launch_fcg_begin(int64_t n, const float* d32, const CgCtl* ctl64, const double* q_prev, double* z,
                      double* dots, hipStream_t s);
void launch_fcg_dir(int64_t n, const double* z, const double* w, const double* r, const double* p_prev,
                    const double* q_prev, double* p, double* q, double* dots, int par, hipStream_t s);
void launch_fcg_update(int64_t n, double* x, double* r, const double* p, const double* q, const double* dots,
                       int par, CgCtl* ctl64, hipStream_t s);

// x = sum_j coef[j] hist[(head - j) mod 4]; zero if ctl->bb == 0
void launch_guess_poly(int64_t n, const double* hist, int head, int order, double* x, const CgCtl* ctl,
                       hipStream_t s);

void launch_newmark(int64_t n, double dt, const double* du, double* u, double* v, double* a, double* hist_slot,
                    hipStream_t s);
void launch_record(int n_rec, const int32_t* rec, const double* v, double* wave_row, hipStream_t s);
// one step's log entry (iterations, true relative residual), written by a
// kernel so that the step needs no host synchronisation
void launch_log_step(int32_t* it_dst, int32_t iters, double* rel_dst, double rel, hipStream_t s);

void launch_misfit(int n_rec, int64_t n_steps, const double* U, const double* obs, double* pair_buf,
                   double* out2, hipStream_t s);

// dst[i*w + k] = src[map[i]*w + k], i < n, k < w (w <= 6)
void launch_permute_f64(int64_t n, int w, const double* src, const int32_t* map, double* dst, hipStream_t s);
void launch_permute_f32(int64_t n, int w, const float* src, const int32_t* map, float* dst, hipStream_t s);

// ---- learned initial guess (sw_mlp.hip) ---------------------------------

// Network 10 -> 64 -> 64 -> 1, parameters packed W1[64][10], b1, W2[64][64],
// b2, w3, b3; training rows hold 10 features, the target and the weight.
constexpr int MLP_IN = 10, MLP_H = 64, MLP_NP = 4929, MLP_ROW = 12;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 640, MLP_OFF_W2 = 704, MLP_OFF_B2 = 4800, MLP_OFF_W3 = 4864,
              MLP_OFF_B3 = 4928;

// Where the features of the guess live (all in internal node order).
struct MlpFeat {
  int64_t n_dof;
  const double* hist;     // [4][n_dof] increments, ring
  int head;               // slot of the newest increment
  const float* nbh;       // [4][n_dof] element-neighbour means, ring
  int nb_head;
  const float* node_mat;  // [n_nodes][2]: Vs, rho (element means)
};

void launch_mlp_forward(int64_t n, const float* X, const float* theta, float* y, hipStream_t s);
void launch_mlp_guess(const MlpFeat& F, const float* theta, double* x, const CgCtl* ctl, bool corr, hipStream_t s);
void launch_mlp_collect(const MlpFeat& F, const double* du, int count, uint64_t seed, int64_t step, int64_t row0,
                        int64_t capacity, float* out, hipStream_t s);
void launch_mlp_grad(const float* S, int64_t n, int64_t nb, uint64_t seed, int64_t batch, const float* theta,
                     double* grad, double* loss2, hipStream_t s);
void launch_mlp_adam(float* theta, float* m, float* v, double* grad, const double* loss2, int64_t step, float lr,
                     hipStream_t s);
// out[node][3] = element-neighbour mean of the FP64 node field in (out cleared first)
void launch_neighbour_mean(const MeshDev& m, const double* in, float* out, hipStream_t s);
// out[node][2] = (Vs, rho) averaged over the node's elements (out cleared first)
void launch_node_material(const MeshDev& m, const uint8_t* emat, const MatDev* mats, float* out, hipStream_t s);

// ---- projection initial guess (sw_proj.hip) -------------------------------

constexpr int PROJ_MAX = 16;      // largest ring of past increments
constexpr int PROJ_BLOCKS = 1024; // workgroups of a dot-product pass
// out[i] = R_i . (v - w) for the L ring vectors R_i (w may be null); part
// holds PROJ_BLOCKS * L doubles of workgroup partials
void launch_proj_dots(int L, int64_t n, const double* R, const double* v, const double* w, double* part,
                      double* out, hipStream_t s);
// out[i] = R_i . v1 and out[L + i] = R_i . v2 in one pass over the ring;
// part holds PROJ_BLOCKS * 2L doubles
void launch_proj_dots2(int L, int64_t n, const double* R, const double* v1, const double* v2, double* part,
                       double* out, hipStream_t s);
// x = sum_i theta[i] X_i (theta on the device)
void launch_proj_combine(int L, int64_t n, const double* X, const double* theta, double* x, hipStream_t s);
// x = sum_i theta[i] X_i, r = b - sum_i theta[i] Y_i, *rr_out = r.r
void launch_proj_combine_res(int L, int64_t n, const double* X, const double* Y, const double* theta,
                             const double* b, double* x, double* r, double* part, double* rr_out, hipStream_t s);
// Xs = x, Ys = b - r
void launch_proj_store(int64_t n, const double* x, const double* b, const double* r, double* Xs, double* Ys,
                       hipStream_t s);

// ---- input estimation (sw_fit.hip) ----------------------------------------

// w[pair] = 1 / |obs_pair|^2 (zero for silent pairs); o2: n_pairs scratch
void launch_fit_weights(int n_pairs, int64_t n_steps, const double* obs, double* o2, double* w, hipStream_t s);
// C (4 nb x 4 nb) = weighted Gram matrix of the stride-m blocks of the three
// Green's records and the observed record, records [t][pair]
void launch_fit_gram(const double* const g[3], const double* obs, int n_pairs, int m, int nb, const double* w,
                     double* C, hipStream_t s);
// U[t][pair] = sum_{j,l} c[j][l] g_j[t - l m][pair]
void launch_fit_response(const double* const g[3], int n_pairs, int m, int n_shift, int64_t n_steps,
                         const double* c, double* U, hipStream_t s);

void launch_fill_f64(int64_t n, double* x, double val, hipStream_t s);
void launch_fill_f32(int64_t n, float* x, float val, hipStream_t s);

}  // namespace sw
