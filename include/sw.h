/*
 * sw.h -- C-ABI of the MI355X implicit seismic-wave analysis library.
 *
 * One analysis ("case") is the implicit 3D wave-propagation analysis that the
 * paper runs once per candidate ground model and input direction
 * (Section 3: 236 models x 3 directions): linear elastodynamics
 * (Section 2, Eq. GE:ORG) on second-order (10-node) tetrahedra, traction-free
 * top, absorbing sides and base, the input velocity wave applied at the base
 * as a force (Sections 2-3), marched in time by the Newmark-beta method
 * (Section 3) with beta = 1/4, gamma = 1/2, every step's system
 *     (c_M M + c_K K + 2/dt C_abs) du = b,
 *     c_M = 4/dt^2 + 2 alpha/dt,  c_K = 1 + 2 beta_R/dt,
 * solved by preconditioned conjugate gradients (Section 3 names a CG solver)
 * around a matrix-free element-by-element operator, to a relative residual
 * ||b - A du||_2 <= rtol ||b||_2 recomputed in FP64.  The outputs are
 * velocities at surface observation points and the misfit ERR of
 * Eq. (eqerr).
 *
 * Conventions
 *   - Vectors on the device are FP64, node-major: value[3 * node + comp].
 *   - tet10: vertices 0..3 then edge nodes 01, 12, 02, 03, 13, 23; positive
 *     volume; edge nodes at edge midpoints (straight-sided elements).
 *   - tri6: vertices 0..2 then edge nodes 01, 12, 20.
 *   - face_role: 1 = absorbing side face, 2 = absorbing base face that also
 *     carries the input force 2 Z v_in, Z = rho Vp n n^T + rho Vs (I - n n^T)
 *     with the material of the owning tet.
 *   - material rows are (Vp, Vs, rho).
 *
 * Ownership
 *   - Host arrays passed to *_create are copied before the call returns.
 *   - Device memory is owned by the caller: each object works inside the
 *     workspace the caller passes (size from the matching *_workspace_bytes
 *     call, 256-byte aligned base) and borrows it until destroyed.  The
 *     library itself never allocates device memory.
 *   - All device work is enqueued on the context's stream.
 *
 * Errors
 *   - Every call returns SW_OK (0) or a negative status; sw_last_error()
 *     returns a message for the last failure on the calling thread.  Host
 *     validation (sizes, index ranges, element orientation, parameters) runs
 *     before any device work, so a rejected call leaves no device state
 *     changed.  Non-convergence is not an error of the step call: the step
 *     completes and the case's flags record it.
 *   - One context per host thread; calls on one context are not thread safe.
 */
#ifndef SW_H
#define SW_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SW_API __attribute__((visibility("default")))
#else
#define SW_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sw_ctx sw_ctx;
typedef struct sw_mesh sw_mesh;
typedef struct sw_case sw_case;
typedef struct sw_batch sw_batch;
typedef struct sw_mlp sw_mlp;

enum {
  SW_OK = 0,
  SW_EINVAL = -1,   /* bad argument or parameter */
  SW_ENOWS = -2,    /* workspace missing, misaligned or too small */
  SW_EMESH = -3,    /* invalid mesh (index out of range, inverted or curved element) */
  SW_ENOCONV = -4,  /* reserved: convergence failure is reported through flags */
  SW_EHIP = -5,     /* HIP runtime error */
  SW_ESTATE = -6    /* object used in the wrong state */
};

/* sw_case_stats.flags bits */
enum { SW_FLAG_NOCONV = 1, SW_FLAG_NONFINITE = 2, SW_FLAG_GUESS_FALLBACK = 4 };

/* precision of the per-step solve */
enum {
  SW_FP64 = 0,        /* FP64 preconditioned CG on the FP64 operator */
  SW_MIXED_FP32 = 1,  /* FP32 inner CG (FP32 operator, FP32 vectors) inside FP64
                         iterative refinement; FP64 true residual and update */
  SW_MIXED_FP32_FLEX = 2, /* the same FP32 inner CG as the variable preconditioner of
                             an FP64 flexible CG (one previous direction kept; the
                             CG with variable preconditioning of Section 3); FP64
                             true residual confirms convergence.  Single cases only
                             (batches march SW_MIXED_FP32 lanes) */
  SW_MIXED_FP16 = 3       /* SW_MIXED_FP32 with the inner CG's direction vector stored
                             in 16 bits (bfloat16, FP32 arithmetic and accumulation):
                             the operator pass gathers it, and x += alpha p and
                             p = z + beta p use the stored values.  Single cases only */
};

/* initial guess of each step's solve */
enum {
  SW_GUESS_ZERO = 0,  /* du0 = 0 */
  SW_GUESS_POLY = 1,  /* Lagrange extrapolation of the last poly_order + 1 increments */
  SW_GUESS_MLP = 2,   /* poly extrapolation plus a learned per-DOF correction */
  SW_GUESS_PROJ = 3,  /* Galerkin projection of the step's solution onto the span of the
                         last proj_dim increments (A-norm optimal combination) */
  SW_GUESS_PROJ_MLP = 4 /* the same projection onto the span of the last proj_dim
                           increments and the network's correction w = s * y of
                           SW_GUESS_MLP (one more direction, its image A w taken
                           with one FP64 operator pass): the combination can be no
                           worse in the A-norm than either; needs a network
                           (sw_case_attach_mlp) */
};

/* operators for sw_case_apply (bit mask; the terms are summed) */
enum {
  SW_OP_M = 1,     /* consistent mass M */
  SW_OP_K = 2,     /* stiffness K */
  SW_OP_CABS = 4,  /* dashpot matrix C_abs */
  SW_OP_A = 8      /* step operator c_M M + c_K K + 2/dt C_abs (exclusive of the others) */
};

/* Message of the last failed call on this thread (never NULL). */
SW_API const char* sw_last_error(void);

/* Library version string. */
SW_API const char* sw_version(void);

/* Context on HIP device `device`; `hip_stream` is a hipStream_t (NULL = the
 * null stream) on which all work of objects made from this context runs. */
SW_API int sw_ctx_create(int device, void* hip_stream, sw_ctx** out);
SW_API int sw_ctx_destroy(sw_ctx* ctx);

/* enable != 0 (the default): CG iterations after the first chunk of each
 * solve are replayed from HIP graphs of two iterations (one per case and
 * precision, one per batch), captured on first use on a stream of the
 * library's own and launched on the context stream; 0: every kernel is
 * launched directly.  The kernels and their results are the same either
 * way; while the profiler is on, kernels are launched directly. */
SW_API int sw_ctx_set_graphs(sw_ctx* ctx, int32_t enable);

/* Workgroup count of the persistent FP32 operator passes (single case and
 * batch lanes) of objects on this context: 0 (default) = three per compute
 * unit, else at most max_workgroups (a positive multiple of 8, one run per
 * XCD), so that each workgroup walks more tiles.  A tuning and test knob;
 * results are the same to rounding.  SW_EINVAL for other values. */
SW_API int sw_ctx_set_grid_cap(sw_ctx* ctx, int32_t max_workgroups);

/* Kernel classes timed by the optional profiler: the matrix-free operator
 * (tile kernel) and the two CG vector kernels, per precision, as launched
 * inside the CG iterations of sw_case_step. */
enum {
  SW_PROF_TILE_F64 = 0, SW_PROF_TILE_F32 = 1,
  SW_PROF_UPDATE_F64 = 2, SW_PROF_UPDATE_F32 = 3,
  SW_PROF_DIR_F64 = 4, SW_PROF_DIR_F32 = 5,
  SW_PROF_KINDS = 6
};
/* enable != 0: bracket every launch of those kernels with HIP events on the
 * context stream (a few microseconds of overhead per launch) and reset the
 * totals; 0: stop.  Synchronises the stream. */
SW_API int sw_ctx_profile(sw_ctx* ctx, int32_t enable);
/* The same for the kernel classes whose bits (1 << SW_PROF_*) are set in
 * `mask` only (0: stop), and for one launch in `every` (>= 1) of each such
 * class (the first, then every `every`-th), so that the events add little to
 * the timed work.  Bits at or above SW_PROF_KINDS or every < 1 are
 * SW_EINVAL. */
SW_API int sw_ctx_profile_kinds(sw_ctx* ctx, uint32_t mask, int32_t every);
/* Total device time (ms) and launch count of one kernel class since the last
 * sw_ctx_profile call, and (optional, may be NULL) the mean duration and
 * count of its full launches: those lasting at least half the longest, which
 * leaves out launches that returned at once because the solve had already
 * converged.  Synchronises the stream. */
SW_API int sw_ctx_profile_read(sw_ctx* ctx, int32_t kind, double* total_ms, int64_t* count, double* full_mean_ms,
                               int64_t* full_count);

/* ----------------------------------------------------------------- mesh */

typedef struct {
  int64_t n_nodes, n_tets, n_faces;
  const double* xyz;          /* host, n_nodes x 3 */
  const int32_t* tet10;       /* host, n_tets x 10 */
  const int32_t* tri6;        /* host, n_faces x 6 */
  const int32_t* face_tet;    /* host, n_faces: the tet each face belongs to */
  const uint8_t* face_role;   /* host, n_faces: 1 side, 2 base */
  int32_t tile_max_nodes;     /* tile capacity of the device layout: distinct nodes per tile,
                                 64..1280 (0 = 1280) */
  int32_t tile_max_elems;     /* elements per tile, 16..1024 (0 = 512: two per work-item) */
  int32_t deterministic;      /* 1: also build, for deterministic cases, each node's list of the
                                 element and face slots that touch it (in element order;
                                 4 bytes per slot); 0: not */
} sw_mesh_desc;

/* Device workspace needed by sw_mesh_create for this mesh. */
SW_API int sw_mesh_workspace_bytes(const sw_mesh_desc* desc, size_t* bytes);
/* Validates the mesh (index ranges, positive volumes, edge nodes at edge
 * midpoints to 1e-9 relative, faces being faces of their owning tet),
 * builds the device layout and uploads it into dev_ws. */
SW_API int sw_mesh_create(sw_ctx* ctx, const sw_mesh_desc* desc, void* dev_ws, size_t ws_bytes, sw_mesh** out);
/* Tiles of the device layout and the largest tile's node count (either
 * pointer may be NULL). */
SW_API int sw_mesh_info(const sw_mesh* mesh, int32_t* n_tiles, int32_t* max_tile_nodes);
SW_API int sw_mesh_destroy(sw_mesh* mesh);

/* ----------------------------------------------------------------- case */

typedef struct {
  double dt;             /* time step, > 0 */
  double ray_alpha;      /* Rayleigh mass coefficient (1/s), >= 0 */
  double ray_beta;       /* Rayleigh stiffness coefficient (s), >= 0 */
  double rtol;           /* relative residual target, in (0, 1) */
  int32_t max_iter;      /* CG iteration cap per step (inner + outer) */
  int32_t precision;     /* SW_FP64, SW_MIXED_FP32, SW_MIXED_FP32_FLEX or SW_MIXED_FP16 */
  int32_t guess;         /* SW_GUESS_* */
  int32_t poly_order;    /* 0..3, used by SW_GUESS_POLY / SW_GUESS_MLP */
  double inner_rtol;     /* mixed precisions: floor of the inner CG relative tolerance (0 = default 1e-4) */
  int32_t n_mat;         /* rows of mat, 1..255 */
  const double* mat;     /* host, n_mat x 3 rows (Vp, Vs, rho), Vp^2 > 2 Vs^2 */
  const uint8_t* tet_mat;/* host, n_tets material ids */
  int32_t n_rec;         /* receivers (>= 0) */
  const int32_t* rec_node; /* host, n_rec node ids */
  int64_t n_steps;       /* capacity of the march (steps 1..n_steps) */
  const double* v_in;    /* host, (n_steps + 1) x 3 incident velocity at t = n dt */
  int32_t proj_dim;      /* SW_GUESS_PROJ: increments spanned, 2..16; SW_GUESS_PROJ_MLP: 2..15 (0 = 6) */
  int32_t deterministic; /* 1: bitwise reproducible march: SW_FP64 with SW_GUESS_ZERO, _POLY or
                            _PROJ, on a mesh created with deterministic = 1.  Every element's and
                            face's contribution goes to a buffer of the case (240 bytes per tet,
                            144 per face) and each node sums its own in element order, and every
                            reduction adds in a fixed order, so the same inputs give the same
                            bits on every run; slower (the default adds in arrival order).
                            0: the default */
} sw_case_desc;

SW_API int sw_case_workspace_bytes(const sw_mesh* mesh, const sw_case_desc* desc, size_t* bytes);
/* Copies the case data to the device and builds the 3x3 block-Jacobi
 * preconditioner (FP64 inverse of the diagonal blocks of A). */
SW_API int sw_case_create(sw_ctx* ctx, sw_mesh* mesh, const sw_case_desc* desc, void* dev_ws, size_t ws_bytes,
                   sw_case** out);
SW_API int sw_case_destroy(sw_case* c);

/* State (u, v, a) as host arrays of 3*n_nodes doubles and the step index;
 * set_state also clears the increment history used by the guesses.  NULL
 * pointers leave (set) or skip (get) that vector. */
SW_API int sw_case_set_state(sw_case* c, const double* u, const double* v, const double* a, int64_t step);
SW_API int sw_case_get_state(const sw_case* c, double* u, double* v, double* a, int64_t* step);

/* March n steps (synchronous on return).  Fails with SW_ESTATE beyond the
 * case's n_steps capacity. */
SW_API int sw_case_step(sw_case* c, int32_t n);

typedef struct {
  int64_t steps;             /* steps completed */
  int64_t cg_iters;          /* total CG iterations (inner iterations for mixed) */
  int64_t ir_outer;          /* total FP64 true-residual evaluations */
  double max_true_rel_res;   /* max over steps of ||b - A du|| / ||b|| (FP64) */
  int32_t flags;             /* SW_FLAG_* */
} sw_case_stats;

SW_API int sw_case_stats_get(const sw_case* c, sw_case_stats* out);
/* Per-step log for steps step0+1 .. step0+n: CG iterations and the final
 * FP64 relative residual (host arrays; either may be NULL). */
SW_API int sw_case_step_log(const sw_case* c, int64_t step0, int64_t n, int32_t* iters, double* rel_res);

/* Receiver velocities of steps step0+1 .. step0+n into host out
 * (n x n_rec x 3). */
SW_API int sw_case_waveforms(const sw_case* c, int64_t step0, int64_t n, double* out);
/* Device pointer of the waveform buffer (n_steps x n_rec x 3, FP64). */
SW_API int sw_case_waveform_device(const sw_case* c, const double** out);

/* y = op x for device vectors of 3*n_nodes doubles (op: SW_OP_*),
 * synchronous.  For testing and for callers composing their own solvers. */
SW_API int sw_case_apply(sw_case* c, int32_t op, const double* x_dev, double* y_dev);
/* Same with the FP32 operator used by the SW_MIXED_FP32 inner solve; for
 * SW_OP_A it runs the very pass an inner CG iteration launches. */
SW_API int sw_case_apply_f32(sw_case* c, int32_t op, const float* x_dev, float* y_dev);
/* Right-hand side b of the next step (from the current state) into y_dev. */
SW_API int sw_case_rhs(sw_case* c, double* y_dev);
/* Initial guess that the next step would start from (from the current
 * increment history and the case's guess kind) into y_dev. */
SW_API int sw_case_guess(sw_case* c, double* y_dev);
/* Diagonal 3x3 blocks of A, 6 doubles per node (xx yy zz yz xz xy), into y_dev. */
SW_API int sw_case_diag_blocks(sw_case* c, double* y_dev);

/* ERR of Eq. (eqerr) between device waveforms U and obs (n_steps x n_rec x
 * 3, FP64): the mean over (receiver, component) pairs of
 * ||U - obs||_2 / ||obs||_2 over time.  Pairs whose observed norm is <=
 * 1e-12 of the largest are skipped; the mean is over the pairs used
 * (*n_pairs).  dev_ws: device scratch of sw_misfit_workspace_bytes(n_rec)
 * bytes, 8-byte aligned.  Synchronous; result to host. */
SW_API int sw_misfit_workspace_bytes(int32_t n_rec, size_t* bytes);
SW_API int sw_misfit(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* U_dev, const double* obs_dev,
              void* dev_ws, size_t ws_bytes, double* err, int32_t* n_pairs);
/* The same ERR for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): no
 * workspace argument and no allocation of any kind; the per-pair scratch is
 * a static device array of the library, one per GPU, holding
 * 2 * 3 * SW_MISFIT_NOALLOC_MAX_REC + 2 doubles (about 768 KiB) for the life
 * of the process.  n_rec above SW_MISFIT_NOALLOC_MAX_REC is SW_EINVAL (no
 * device work).  All calls on one GPU share that array: calls that overlap
 * in time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Same result as sw_misfit on the same inputs;
 * synchronous; result to host. */
#define SW_MISFIT_NOALLOC_MAX_REC 16384
SW_API int sw_misfit_noalloc(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* U_dev,
                             const double* obs_dev, double* err, int32_t* n_pairs);
/* ERR of the case's recorded waveforms (steps 1..current) against obs_dev
 * (same layout, at least as many steps), using the case's own scratch. */
SW_API int sw_case_misfit(sw_case* c, const double* obs_dev, double* err, int32_t* n_pairs);

/* ------------------------------------------------------ learned guess */

/* Per-DOF network predicting each step's initial guess (the paper has no
 * network; this is the learned part added to its CG solve).  For DOF (node
 * n, component c) before the step that computes du^m:
 *   d_k   = du^{m-1-k}(n, c), k = 0..3            (last four increments)
 *   nb_k  = element-neighbour mean of du^{m-1-k}  (mean over the elements
 *           containing n of the element's mean of component c)
 *   s     = max_k(|d_k|, |nb_k|)
 *   D(a)  = (a_0, a_0 - a_1, a_0 - 2 a_1 + a_2, a_0 - 3 a_1 + 3 a_2 - a_3)
 *   x     = D(d) / s, D(nb) / s, Vs/500, rho/2000  (node means; the
 *           differences formed in FP64)
 *   y     = w3 . ReLU(W2 ReLU(W1 x + b1) + b2) + b3
 *   guess = 3 d_0 - 3 d_1 + d_2 + s y                 (0 when s = 0)
 * Parameters (SW_MLP_NPARAM floats, FP32, host order): W1[64][10], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  Inference runs in FP16 on the matrix
 * cores with FP32 accumulation.  Training rows (12 floats): the ten
 * features x, the target t = (du^m - quadratic extrapolation) / s and the
 * weight s^2; the loss is sum w (y - t)^2 / sum w, minimised with Adam
 * (beta 0.9 / 0.999, eps 1e-8) on FP32 weights. */
#define SW_MLP_NPARAM 4929
#define SW_MLP_ROW 12
/* Initial parameters for training (host, SW_MLP_NPARAM floats written):
 * Glorot-uniform hidden layers drawn from a splitmix64 stream of `seed`,
 * zero biases and a zero output layer, so that the untrained network's
 * guess is exactly the quadratic extrapolation. */
SW_API int sw_mlp_init_params(uint64_t seed, float* params);
SW_API int sw_mlp_workspace_bytes(size_t* bytes);
/* params: host, SW_MLP_NPARAM floats (copied).  Non-finite values are
 * accepted: a guess that is not finite or whose residual exceeds that of the
 * zero guess is replaced by quadratic extrapolation (SW_FLAG_GUESS_FALLBACK). */
SW_API int sw_mlp_create(sw_ctx* ctx, const float* params, void* dev_ws, size_t ws_bytes, sw_mlp** out);
SW_API int sw_mlp_destroy(sw_mlp* mlp);
SW_API int sw_mlp_get_params(sw_mlp* mlp, float* params_host);
/* y_dev[i] = network output for the features X_dev[i][0..9] (device, FP32),
 * computed by the same matrix-core path as the guess.  Synchronous. */
SW_API int sw_mlp_forward(sw_mlp* mlp, const float* X_dev, float* y_dev, int64_t n);
/* Gradient of the loss over the n rows of S_dev (device, n x 12) into
 * grad_host (SW_MLP_NPARAM doubles) and the loss into *loss (FP32 kernels).
 * Synchronous. */
SW_API int sw_mlp_gradient(sw_mlp* mlp, const float* S_dev, int64_t n, double* grad_host, double* loss);
/* `steps` Adam steps on minibatches of `batch` rows drawn with replacement
 * from the n rows of S_dev by a counter-based generator keyed on `seed`;
 * loss_host (optional, `steps` floats) receives each minibatch's loss.
 * Synchronous. */
SW_API int sw_mlp_train(sw_mlp* mlp, const float* S_dev, int64_t n, int32_t steps, int32_t batch, float lr,
                        uint64_t seed, float* loss_host);
/* Use (or with NULL stop using) the network for a case created with
 * guess SW_GUESS_MLP or SW_GUESS_PROJ_MLP; the network stays owned by the
 * caller. */
SW_API int sw_case_attach_mlp(sw_case* c, sw_mlp* mlp);
/* Record training rows while the case marches: after each step's solve,
 * per_step DOFs drawn by a counter-based generator keyed on (seed, step)
 * give one row each into the device ring buffer dev_buf (capacity rows of
 * SW_MLP_ROW floats).  Needs a case created with a non-zero guess; rows are
 * recorded once four past increments exist.  NULL stops recording. */
SW_API int sw_case_set_sampler(sw_case* c, float* dev_buf, int64_t capacity, int32_t per_step, uint64_t seed);
/* Rows recorded so far (at most the capacity). */
SW_API int sw_case_samples(const sw_case* c, int64_t* rows);

/* ------------------------------------------------------ input estimation */

/* The misfit of a candidate model with the input estimated (Section 2):
 * the input velocity along j is sum_l c_jl p(t - l dT), shifted copies of a
 * unit impulse p, and the response at the receivers is
 *     U_i^k(t) = sum_{j,l} G_ij^k(t - l dT) c_jl
 * with G_j the Green's records, i.e. the receiver velocities of three runs
 * of the model driven by p along x1, x2 and x3 (for instance the
 * waveforms of three cases whose v_in is p along one direction; the model
 * starts from rest, so a delayed impulse gives the delayed record).  The
 * coefficients minimise sum_{k,i} |U_i^k - obs_i^k|^2 / |obs_i^k|^2 (the
 * squares of the terms of ERR; silent pairs, norm <= 1e-12 of the largest,
 * carry no weight): the normal equations A c = b are formed on the GPU from
 * block inner products of the records and solved on the host with the
 * eigen-decomposition of the symmetric A, eigenvalues at or below
 * rel_cut times the largest discarded (the pseudo-inverse of Section 2).
 * ERR (Eq. eqerr) is then evaluated at that c.
 *
 * green: host array of 3 device pointers, records [n_steps][n_rec][3]
 * (FP64, step 1..n_steps); obs: device, same layout; stride: dT in time
 * steps (n_steps must be a multiple); n_shift: shifts l = 0..n_shift-1
 * (<= n_steps / stride, <= 128); ws: device workspace of
 * sw_fit_workspace_bytes, 256-byte aligned.  Outputs: c_host (3 x n_shift,
 * row j = direction), err, n_pairs (pairs used), rank (eigenvalues kept),
 * U_dev (optional, device [n_steps][n_rec][3]: the fitted response).
 * Synchronises the context stream. */
SW_API int sw_fit_workspace_bytes(int32_t n_rec, int64_t n_steps, int32_t stride, int32_t n_shift, size_t* bytes);
SW_API int sw_fit_input(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green, const double* obs,
                        int32_t stride, int32_t n_shift, double rel_cut, void* dev_ws, size_t ws_bytes,
                        double* c_host, double* err, int32_t* n_pairs, int32_t* rank, double* U_dev);

/* Several observed events of one model (Section 3: the records of several
 * earthquakes at the same site, Table of events; Section 2: the model is
 * judged by its misfit): the Green's records are the model's and are
 * computed once; the input of each event is estimated on its own exactly as
 * sw_fit_input does (the same workspace, reused event after event), and
 * the model's misfit is the largest ERR over its events (its worst event).
 * obs: host array of n_events device pointers, each [n_steps][n_rec][3].
 * Outputs (host): c_host (n_events x 3 x n_shift), err (n_events),
 * n_pairs and rank (n_events each, optional), err_max (the largest ERR; NaN
 * when an event has no usable pair, which is then the worst) and worst (its
 * event index, optional).  Synchronises the context stream. */
SW_API int sw_fit_events(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green, int32_t n_events,
                         const double* const* obs, int32_t stride, int32_t n_shift, double rel_cut, void* dev_ws,
                         size_t ws_bytes, double* c_host, double* err, int32_t* n_pairs, int32_t* rank,
                         double* err_max, int32_t* worst);

/* ----------------------------------------------------------------- batch */

/* A batch marches many candidate models together: the repeated analyses of
 * the paper (Section 3: one analysis per candidate model and input
 * direction).  Each case is a lane; every phase of a time step (right-hand
 * side, true residual, each FP32 CG iteration, Newmark update, recording)
 * is one kernel launch over all lanes, whatever their meshes, and the
 * element-by-element pass hands the lanes of one mesh tile to the same XCD
 * so that the tile's mesh data is read once per pass for all of them.
 * Each lane keeps its own convergence control: a lane whose solve has
 * converged returns from the launches at once, and its result is the same
 * (to rounding) as stepping the case alone.
 *
 * cases: n distinct cases of one context, all SW_MIXED_FP32 (SW_EINVAL
 * otherwise); any meshes, guesses, step counts.  The batch borrows them: a
 * case must outlive the batch and must not be stepped alone while a batch
 * step runs.  dev_ws: caller-owned device memory of at least the bytes
 * sw_batch_workspace_bytes gives (lane tables and work list), borrowed until
 * sw_batch_destroy.  sw_batch_step advances every case n_steps steps
 * (SW_ESTATE if one would pass its capacity or lacks its network) and
 * synchronises the context stream: each refinement round of a step decides
 * on the host, from the lanes' FP64 true residuals, which lanes run another
 * inner solve and to what tolerance, and the projection guess solves its
 * small Gram system on the host.  sw_batch_stats gives every lane's
 * statistics in lane order; logs and waveforms are read per case. */
SW_API int sw_batch_workspace_bytes(sw_case* const* cases, int32_t n, size_t* bytes);
SW_API int sw_batch_create(sw_ctx* ctx, sw_case* const* cases, int32_t n, void* dev_ws, size_t ws_bytes,
                    sw_batch** out);
SW_API int sw_batch_step(sw_batch* b, int32_t n_steps);
/* Set-up-time tuning of the schedule of the batch's FP32 lane pass (the
 * launch every inner CG iteration of sw_batch_step makes): times `reps`
 * (1..1000) passes of each candidate on the lanes' inner-solve vectors
 * (free between steps; left zero) and keeps the fastest for later steps.
 * Candidates k = 2 * order + grid: order 0 = one mesh after the other,
 * 1 = the meshes interleaved tile by tile (each with the lanes of a tile
 * adjacent); grid 0 = three workgroups per compute unit, 1 = two.  Writes
 * the chosen k and (optional) the mean pass time of each candidate (ms, 4
 * values).  Results do not depend on the schedule beyond rounding.
 * Synchronous. */
SW_API int sw_batch_autotune(sw_batch* b, int32_t reps, int32_t* choice, double* ms);
/* The same for a single case's persistent FP32 pass (mixed precisions):
 * candidates k = 0, 1, 2 are three, two and one workgroups per compute
 * unit; ms: 3 values (optional).  Synchronous. */
SW_API int sw_case_autotune(sw_case* c, int32_t reps, int32_t* choice, double* ms);
/* Statistics of every lane (out: n entries, lane order; as
 * sw_case_stats_get of each case). */
SW_API int sw_batch_stats(const sw_batch* b, sw_case_stats* out);
/* y[l] = A_l x[l] for every lane l through the batch's FP32 lane pass, the
 * very launch an inner CG iteration of sw_batch_step makes (A_l: lane l's
 * step operator; x, y: host arrays of n device pointers to 3 * n_nodes
 * floats of that lane's mesh, caller's node order).  Uses the lanes'
 * inner-solve vectors, which are free between steps.  For testing the lane
 * pass.  Synchronous. */
SW_API int sw_batch_apply_f32(sw_batch* b, const float* const* x, float* const* y);
SW_API int sw_batch_destroy(sw_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* SW_H */
