// C-ABI runtime of the implicit wave-propagation library: validation,
// workspace layout, preconditioner setup and the per-step driver.
//
// Per step (Newmark average acceleration, Section 3):
//   1. right-hand side b = F^{n+1} + M (a + (4/dt + alpha) v) - K (u - beta v)
//      + C_abs v  (one EBE pass with two inputs + one face pass)
//   2. ||b||^2, tolerance, initial guess
//   3. preconditioned CG on A du = b in chunks of iterations that run with
//      no host round trip (device-side convergence flag); FP64, or FP32 inner
//      solves inside FP64 iterative refinement
//   4. FP64 true residual ||b - A du|| / ||b|| checked against rtol
//   5. Newmark update of (u, v, a), increment history, receiver record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <stdexcept>
#include <vector>

#include "sw.h"
#include "sw_internal.h"
#include "sw_layout.h"
#include "sw_linalg.h"

using namespace sw;

// ------------------------------------------------------------ errors

static thread_local std::string g_err = "no error";

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPC(expr)                                                                                  \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess) return fail(SW_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

#define LAUNCHED()                                                                                       \
  do {                                                                                                   \
    hipError_t _e = hipGetLastError();                                                                   \
    if (_e != hipSuccess) return fail(SW_EHIP, "kernel launch failed: %s", hipGetErrorString(_e)); \
  } while (0)

extern "C" const char* sw_last_error(void) { return g_err.c_str(); }
extern "C" const char* sw_version(void) { return "sw 0.1 (gfx950)"; }

// ------------------------------------------------------------ workspace

namespace {

struct Carver {
  uint8_t* base;
  size_t off = 0;
  explicit Carver(void* b) : base((uint8_t*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

inline int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

}  // namespace

// ------------------------------------------------------------ objects

// Optional per-kernel timing with HIP events on the context stream: each
// profiled launch is bracketed by two events; elapsed times are collected
// when the event pool is full (one host synchronisation per kPool / 2
// profiled launches) and when they are read.
struct KernelProfiler {
  static constexpr int kPool = 4096;
  bool on = false;
  uint32_t mask = 0;      // kernel classes profiled (bit SW_PROF_*)
  int every = 1;          // one launch in `every` of each class is timed
  int64_t seen[SW_PROF_KINDS] = {};  // launches of each class since the start
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;  // per event pair
  int next = 0;           // next free event
  double total_ms[SW_PROF_KINDS] = {};
  int64_t count[SW_PROF_KINDS] = {};
  std::vector<float> each[SW_PROF_KINDS];  // every launch's duration (ms)
};

struct sw_ctx {
  int device;
  hipStream_t stream;
  KernelProfiler prof;
  int grid_cap = 0;  // workgroup cap of the persistent FP32 passes (0: none)
  // CG iterations after a solve's first chunk replay captured HIP graphs of
  // two iterations; they are captured on a stream of the library's own
  bool graphs = true;
  hipStream_t cap_stream = nullptr;
};

namespace {

int prof_flush(sw_ctx* ctx) {
  KernelProfiler& P = ctx->prof;
  for (int i = 0; i + 1 < P.next; i += 2) {
    float ms = 0.0f;
    HIPC(hipEventSynchronize(P.ev[i + 1]));
    HIPC(hipEventElapsedTime(&ms, P.ev[i], P.ev[i + 1]));
    P.total_ms[P.kind[i / 2]] += ms;
    P.count[P.kind[i / 2]] += 1;
    P.each[P.kind[i / 2]].push_back(ms);
  }
  P.next = 0;
  return SW_OK;
}

// returns the event index of the start marker, or -1 when not profiling
int prof_begin(sw_ctx* ctx, int kind) {
  KernelProfiler& P = ctx->prof;
  if (!P.on || !((P.mask >> kind) & 1u)) return -1;
  if (P.seen[kind]++ % P.every != 0) return -1;
  if (P.next + 2 > KernelProfiler::kPool && prof_flush(ctx) != SW_OK) return -1;
  const int i = P.next;
  P.kind[i / 2] = kind;
  P.next += 2;
  if (hipEventRecord(P.ev[i], ctx->stream) != hipSuccess) return -1;
  return i;
}

void prof_end(sw_ctx* ctx, int i) {
  if (i >= 0) (void)hipEventRecord(ctx->prof.ev[i + 1], ctx->stream);
}

}  // namespace

struct sw_mesh {
  sw_ctx* ctx;
  MeshDev dev;
  int64_t n_nodes, n_tets, n_faces;
  std::vector<int32_t> elem_order;  // internal element -> user element
  std::vector<int32_t> node_u2i;    // user node -> internal node
  std::vector<int32_t> node_i2u;
};

struct sw_case {
  sw_ctx* ctx;
  sw_mesh* mesh;
  // deterministic passes: element and face result slots (null otherwise)
  bool det = false;
  double* det_e = nullptr;
  double* det_f = nullptr;
  // parameters
  double dt, alpha, beta, rtol, inner_rtol;
  int32_t max_iter, precision, guess, poly_order, n_mat, n_rec;
  int64_t n_steps;
  double cM, cK, cC;
  // device (vectors in internal node order)
  MatDev* mats;
  uint8_t* emat;  // material per internal element
  int32_t* rec;   // internal node ids
  double* vin;
  double *u, *v, *a, *b, *x, *r, *z, *p, *q;
  double* hist;  // [4][n_dof]
  double *diag6, *pinv64, *pmax;
  __half* pinv16;  // block-Jacobi inverse / its largest diagonal entry, FP16 (FP32 CG)
  float *r32, *d32, *z32, *p32, *q32;
  uint16_t* p16;  // SW_MIXED_FP16: the inner CG's direction in bfloat16 (else null)
  // flexible outer CG (SW_MIXED_FP32_FLEX): directions and their images of
  // the current and the previous iteration (by parity), dot products
  double *fp[2] = {nullptr, nullptr}, *fq[2] = {nullptr, nullptr}, *fdots = nullptr;
  // captured pair of CG iterations (FP64, FP32) and the grid cap it was
  // captured with
  hipGraphExec_t cg_graph[2] = {nullptr, nullptr};
  int cg_graph_cap[2] = {-1, -1};
  // workgroup cap of this case's persistent FP32 pass chosen by
  // sw_case_autotune (-1: the context's)
  int grid_cap = -1;
  double* wave;
  int32_t* log_it;
  double* log_rel;
  CgCtl *ctl64, *ctl32;
  int32_t* bad;
  double* mis_buf;
  // learned guess: neighbour means of past increments, node material, network
  float* nbh = nullptr;       // [4][n_dof] ring (allocated when the guess is not zero)
  float* node_mat = nullptr;  // [n_nodes][2] (Vs, rho)
  int nb_head = 3, nb_count = 0;
  sw_mlp* mlp = nullptr;
  // training-sample collection
  float* samp = nullptr;
  int64_t samp_cap = 0, samp_rows = 0;
  int32_t samp_per_step = 0;
  uint64_t samp_seed = 0;
  // projection guess: ring of past increments X, their images Y = A X, the
  // Gram matrix X^T A X on the host
  // proj_slots = proj_dim, plus one for the network's direction (slot
  // proj_dim) with SW_GUESS_PROJ_MLP
  int proj_dim = 0, proj_slots = 0, proj_count = 0, proj_head = -1;
  double *projX = nullptr, *projY = nullptr, *proj_part = nullptr, *proj_out = nullptr, *proj_theta = nullptr;
  std::vector<double> projG, proj_h, proj_th;
  // slots stored since the last projection whose Gram rows are still to be
  // computed (with the next projection's pass over the ring), and the host
  // rows of all but the last of them
  std::vector<int> proj_pend;
  std::vector<double> proj_rows;
  // host state
  int64_t step = 0;
  int hist_head = 3, hist_count = 0;
  int last_iters = 16;
  double last_bb = 0.0;
  sw_case_stats stats{};
};

inline int case_grid_cap(const sw_case* c) { return c->grid_cap >= 0 ? c->grid_cap : c->ctx->grid_cap; }

struct sw_mlp {
  sw_ctx* ctx;
  float *theta, *m, *v;  // FP32 master weights, Adam moments
  double* grad;          // un-normalised gradient accumulator
  double* loss2;         // sum w e^2, sum w
  int64_t adam_step = 0;
};

// Cases marched together.  Lane l is cases[l]; every phase of a step is one
// launch over all lanes (see the lane kernels), the host keeps each lane's
// refinement decisions.
struct sw_batch {
  sw_ctx* ctx;
  std::vector<sw_case*> cases;
  hipGraphExec_t cg_graph = nullptr;  // captured pair of FP32 CG iterations
  int cg_graph_cap = -1;
  int grid_cap = -1;                  // chosen by sw_batch_autotune (-1: the context's)
  int schedule = 0;                   // work-item order (see batch_items)
  int n = 0;
  int64_t max_nodes = 0;
  int max_tile_nodes = 0;
  int n_work = 0;
  // device tables (in the caller's workspace)
  LaneDev* d_lanes = nullptr;
  LaneState* d_st = nullptr;
  LaneInfo* d_info = nullptr;
  TileLane<double>* d_rhs1 = nullptr;
  TileLane<double>* d_rhs2 = nullptr;
  TileLane<double>* d_true = nullptr;
  TileLane<float>* d_cg32 = nullptr;
  int2* d_work = nullptr;
  int2* d_items = nullptr;  // (lane, tile), tile-major, for the persistent FP32 pass
  int n_items = 0;
  // host copies
  std::vector<LaneDev> lanes;
  std::vector<LaneState> st;
  std::vector<LaneInfo> info;
  std::vector<TileLane<double>> rhs1;
};

inline int batch_grid_cap(const sw_batch* b) { return b->grid_cap >= 0 ? b->grid_cap : b->ctx->grid_cap; }

// the case's guess uses the network (and so the neighbour-mean history)
inline bool learned(const sw_case* c) { return c->guess == SW_GUESS_MLP || c->guess == SW_GUESS_PROJ_MLP; }
inline bool needs_mlp(const sw_case* c) { return learned(c) && !c->mlp; }

static int static_scratch_init(int device);

extern "C" int sw_ctx_create(int device, void* hip_stream, sw_ctx** out) {
  if (!out) return fail(SW_EINVAL, "out is NULL");
  int n = 0;
  HIPC(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(SW_EINVAL, "device %d out of range (%d devices)", device, n);
  HIPC(hipSetDevice(device));
  if (int rc = static_scratch_init(device)) return rc;
  sw_ctx* c = new sw_ctx{device, (hipStream_t)hip_stream, {}, 0};
  *out = c;
  return SW_OK;
}

extern "C" int sw_ctx_destroy(sw_ctx* ctx) {
  if (ctx) {
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  }
  delete ctx;
  return SW_OK;
}

extern "C" int sw_ctx_set_graphs(sw_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(SW_EINVAL, "NULL context");
  ctx->graphs = enable != 0;
  return SW_OK;
}

extern "C" int sw_ctx_set_grid_cap(sw_ctx* ctx, int32_t max_workgroups) {
  if (!ctx) return fail(SW_EINVAL, "NULL context");
  if (max_workgroups < 0 || max_workgroups % 8)
    return fail(SW_EINVAL, "grid cap %d is not 0 or a positive multiple of 8", max_workgroups);
  ctx->grid_cap = max_workgroups;
  return SW_OK;
}

extern "C" int sw_ctx_profile(sw_ctx* ctx, int32_t enable) {
  return sw_ctx_profile_kinds(ctx, enable ? (1u << SW_PROF_KINDS) - 1u : 0u, 1);
}

extern "C" int sw_ctx_profile_kinds(sw_ctx* ctx, uint32_t mask, int32_t every) {
  if (!ctx) return fail(SW_EINVAL, "NULL context");
  if (mask >> SW_PROF_KINDS) return fail(SW_EINVAL, "profile mask 0x%x has bits past the %d kernel classes", mask,
                                         (int)SW_PROF_KINDS);
  if (every < 1) return fail(SW_EINVAL, "profile sampling every %d launches", (int)every);
  const bool enable = mask != 0;
  HIPC(hipSetDevice(ctx->device));
  KernelProfiler& P = ctx->prof;
  if (enable && P.ev.empty()) {
    P.ev.resize(KernelProfiler::kPool);
    P.kind.assign(KernelProfiler::kPool / 2, 0);
    for (auto& e : P.ev) HIPC(hipEventCreate(&e));
  }
  HIPC(hipStreamSynchronize(ctx->stream));
  int rc = prof_flush(ctx);
  if (rc) return rc;
  for (int k = 0; k < SW_PROF_KINDS; ++k) {
    P.total_ms[k] = 0.0;
    P.count[k] = 0;
    P.each[k].clear();
    P.seen[k] = 0;
  }
  P.on = enable;
  P.mask = mask;
  P.every = every;
  return SW_OK;
}

extern "C" int sw_ctx_profile_read(sw_ctx* ctx, int32_t kind, double* total_ms, int64_t* count,
                                   double* full_mean_ms, int64_t* full_count) {
  if (!ctx || !total_ms || !count) return fail(SW_EINVAL, "NULL argument");
  if (kind < 0 || kind >= SW_PROF_KINDS) return fail(SW_EINVAL, "unknown kernel kind %d", kind);
  HIPC(hipStreamSynchronize(ctx->stream));
  int rc = prof_flush(ctx);
  if (rc) return rc;
  *total_ms = ctx->prof.total_ms[kind];
  *count = ctx->prof.count[kind];
  const std::vector<float>& e = ctx->prof.each[kind];
  float mx = 0.0f;
  for (float v : e) mx = std::max(mx, v);
  double sum = 0.0;
  int64_t n = 0;
  for (float v : e)
    if (v >= 0.5f * mx) {
      sum += v;
      ++n;
    }
  if (full_mean_ms) *full_mean_ms = n ? sum / (double)n : 0.0;
  if (full_count) *full_count = n;
  return SW_OK;
}

// ------------------------------------------------------------ mesh

static int validate_mesh(const sw_mesh_desc* d) {
  if (!d) return fail(SW_EINVAL, "mesh desc is NULL");
  if (d->n_nodes <= 0 || d->n_tets <= 0 || d->n_faces < 0)
    return fail(SW_EINVAL, "bad mesh sizes (nodes %lld tets %lld faces %lld)", (long long)d->n_nodes,
                (long long)d->n_tets, (long long)d->n_faces);
  if (d->n_nodes > (int64_t)INT32_MAX / 3) return fail(SW_EINVAL, "too many nodes for int32 indexing");
  if (!d->xyz || !d->tet10 || (d->n_faces > 0 && (!d->tri6 || !d->face_tet || !d->face_role)))
    return fail(SW_EINVAL, "NULL mesh array");
  if (d->tile_max_nodes != 0 && (d->tile_max_nodes < 64 || d->tile_max_nodes > TILE_MAX_NODES))
    return fail(SW_EINVAL, "tile_max_nodes %d outside 64..%d (0: default)", d->tile_max_nodes, TILE_MAX_NODES);
  if (d->tile_max_elems != 0 && (d->tile_max_elems < 16 || d->tile_max_elems > TILE_MAX_ELEMS))
    return fail(SW_EINVAL, "tile_max_elems %d outside 16..%d (0: default)", d->tile_max_elems, TILE_MAX_ELEMS);
  if (d->deterministic != 0 && d->deterministic != 1) return fail(SW_EINVAL, "deterministic must be 0 or 1");
  if (d->deterministic && (d->n_tets > (int64_t)INT32_MAX / 10 || d->n_faces > (int64_t)INT32_MAX / 6))
    return fail(SW_EINVAL, "too many elements for the int32 slot lists of deterministic passes");
  for (int64_t i = 0; i < 3 * d->n_nodes; ++i)
    if (!std::isfinite(d->xyz[i])) return fail(SW_EMESH, "non-finite coordinate at node %lld", (long long)(i / 3));
  static const int EA[6] = {0, 1, 0, 0, 1, 2}, EB[6] = {1, 2, 2, 3, 3, 3};
  for (int64_t e = 0; e < d->n_tets; ++e) {
    const int32_t* t = d->tet10 + 10 * e;
    for (int k = 0; k < 10; ++k)
      if (t[k] < 0 || t[k] >= d->n_nodes)
        return fail(SW_EMESH, "tet %lld node %d index %d out of range", (long long)e, k, t[k]);
    const double* X[4];
    for (int k = 0; k < 4; ++k) X[k] = d->xyz + 3 * (int64_t)t[k];
    double c1[3], c2[3], c3[3];
    for (int q = 0; q < 3; ++q) {
      c1[q] = X[1][q] - X[0][q];
      c2[q] = X[2][q] - X[0][q];
      c3[q] = X[3][q] - X[0][q];
    }
    const double det = c1[0] * (c2[1] * c3[2] - c2[2] * c3[1]) - c1[1] * (c2[0] * c3[2] - c2[2] * c3[0]) +
                       c1[2] * (c2[0] * c3[1] - c2[1] * c3[0]);
    if (!(det > 0.0)) return fail(SW_EMESH, "tet %lld has non-positive volume (%g)", (long long)e, det / 6.0);
    for (int k = 0; k < 6; ++k) {
      const double* A = X[EA[k]];
      const double* B = X[EB[k]];
      const double* M = d->xyz + 3 * (int64_t)t[4 + k];
      double len2 = 0.0, err2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        len2 += (B[q] - A[q]) * (B[q] - A[q]);
        const double m = 0.5 * (A[q] + B[q]) - M[q];
        err2 += m * m;
      }
      if (err2 > 1e-18 * len2)
        return fail(SW_EMESH, "tet %lld edge node %d is not at its edge midpoint", (long long)e, 4 + k);
    }
  }
  for (int64_t f = 0; f < d->n_faces; ++f) {
    const int32_t* tr = d->tri6 + 6 * f;
    const int32_t ow = d->face_tet[f];
    if (ow < 0 || ow >= d->n_tets) return fail(SW_EMESH, "face %lld owner %d out of range", (long long)f, ow);
    if (d->face_role[f] != 1 && d->face_role[f] != 2)
      return fail(SW_EMESH, "face %lld has role %d (expected 1 or 2)", (long long)f, (int)d->face_role[f]);
    const int32_t* t = d->tet10 + 10 * (int64_t)ow;
    for (int k = 0; k < 6; ++k) {
      bool found = false;
      for (int j = 0; j < 10; ++j) found |= (t[j] == tr[k]);
      if (!found) return fail(SW_EMESH, "face %lld node %d is not a node of its tet", (long long)f, k);
      if (k < 3) {
        bool vert = false;
        for (int j = 0; j < 4; ++j) vert |= (t[j] == tr[k]);
        if (!vert) return fail(SW_EMESH, "face %lld vertex %d is not a vertex of its tet", (long long)f, k);
      }
    }
  }
  return SW_OK;
}


namespace {

// FNV-1a-style digest (over 8-byte words, then the tail bytes) of a mesh's
// arrays: the layout cache below is keyed by the contents, not by the
// addresses, which a freed and reallocated array of the same size can take
// again.
uint64_t mesh_digest(const sw_mesh_desc* d) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const uint8_t* b = (const uint8_t*)p;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
      uint64_t w;
      std::memcpy(&w, b + i, 8);
      h = (h ^ w) * 1099511628211ull;
    }
    for (; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(d->xyz, 24 * (size_t)d->n_nodes);
  mix(d->tet10, 40 * (size_t)d->n_tets);
  if (d->n_faces > 0) {
    mix(d->tri6, 24 * (size_t)d->n_faces);
    mix(d->face_tet, 4 * (size_t)d->n_faces);
    mix(d->face_role, (size_t)d->n_faces);
  }
  return h;
}

// The tiled layout of the last mesh sized by sw_mesh_workspace_bytes, so the
// create call that normally follows does not rebuild it.
struct LayoutCache {
  uint64_t digest = 0;
  int64_t n_nodes = -1, n_tets = -1, n_faces = -1;
  int32_t cap_nodes = -1, cap_elems = -1;
  HostLayout L;
  bool matches(const sw_mesh_desc* d, uint64_t dig) const {
    return digest == dig && n_nodes == d->n_nodes && n_tets == d->n_tets && n_faces == d->n_faces &&
           cap_nodes == d->tile_max_nodes && cap_elems == d->tile_max_elems;
  }
};
thread_local LayoutCache g_layout;

const HostLayout& layout_for(const sw_mesh_desc* d) {
  const uint64_t dig = mesh_digest(d);
  if (!g_layout.matches(d, dig)) {
    build_layout(d->n_nodes, d->n_tets, d->n_faces, d->xyz, d->tet10, d->tri6, d->face_tet, d->face_role,
                 g_layout.L, d->tile_max_nodes ? d->tile_max_nodes : TILE_MAX_NODES,
                 d->tile_max_elems ? d->tile_max_elems : TILE_DEFAULT_ELEMS);
    g_layout.cap_nodes = d->tile_max_nodes;
    g_layout.cap_elems = d->tile_max_elems;
    g_layout.digest = dig;
    g_layout.n_nodes = d->n_nodes;
    g_layout.n_tets = d->n_tets;
    g_layout.n_faces = d->n_faces;
  }
  return g_layout.L;
}

size_t mesh_layout(const HostLayout& L, bool det, Carver& cv, MeshDev* md) {
  const int32_t nT = L.n_tiles;
  auto conn_loc = cv.take<uint16_t>(10 * L.tet_stride);
  auto teo = cv.take<int32_t>(nT + 1);
  auto tno = cv.take<int32_t>(nT + 1);
  auto tn = cv.take<int32_t>(std::max<size_t>(L.tile_nodes.size(), 1));
  auto tib = cv.take<int32_t>(nT);
  auto tni = cv.take<int32_t>(nT);
  auto tfo = cv.take<int32_t>(nT + 1);
  auto xyz = cv.take<double>(3 * L.n_nodes);
  auto geo32 = cv.take<float>(10 * L.tet_stride);
  auto geo64 = cv.take<double>(10 * L.tet_stride);
  auto fconn = cv.take<int32_t>(6 * L.face_stride);
  auto fconn_loc = cv.take<uint16_t>(6 * L.face_stride);
  auto fel = cv.take<int32_t>(L.face_stride);
  auto frole = cv.take<uint8_t>(L.face_stride);
  auto u2i = cv.take<int32_t>(L.n_nodes);
  auto i2u = cv.take<int32_t>(L.n_nodes);
  auto inv_val = cv.take<float>(L.n_nodes);
  // incidence lists of the deterministic passes (sizes known from the counts)
  int32_t *inc_off = nullptr, *inc = nullptr, *finc_off = nullptr, *finc = nullptr;
  if (det) {
    inc_off = cv.take<int32_t>(L.n_nodes + 1);
    inc = cv.take<int32_t>(10 * L.n_tets);
    finc_off = cv.take<int32_t>(L.n_nodes + 1);
    finc = cv.take<int32_t>(std::max<int64_t>(6 * L.n_faces, 1));
  }
  if (md) {
    md->n_nodes = L.n_nodes;
    md->n_tets = L.n_tets;
    md->n_faces = L.n_faces;
    md->n_tiles = nT;
    md->max_tile_nodes = L.max_tile_nodes;
    md->n_interior = L.n_interior;
    md->tet_stride = L.tet_stride;
    md->face_stride = L.face_stride;
    md->conn_loc = conn_loc;
    md->tile_elem_off = teo;
    md->tile_node_off = tno;
    md->tile_nodes = tn;
    md->tile_int_base = tib;
    md->tile_nint = tni;
    md->tile_face_off = tfo;
    md->xyz = xyz;
    md->geo32 = geo32;
    md->geo64 = geo64;
    md->fconn = fconn;
    md->fconn_loc = fconn_loc;
    md->face_elem = fel;
    md->face_role = frole;
    md->node_u2i = u2i;
    md->node_i2u = i2u;
    md->inv_valence = inv_val;
    md->inc_off = inc_off;
    md->inc = inc;
    md->finc_off = finc_off;
    md->finc = finc;
  }
  return cv.off;
}

template <typename T>
hipError_t up(const T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

namespace {

// The host-side layout allocates; no C++ exception may cross the C-ABI.
template <typename F>
int host_guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(SW_EINVAL, "host memory exhausted while building the mesh layout");
  } catch (const std::exception& e) {
    return fail(SW_EINVAL, "mesh layout: %s", e.what());
  }
}

int mesh_workspace_bytes(const sw_mesh_desc* d, size_t* bytes) {
  if (!d || !bytes) return fail(SW_EINVAL, "NULL argument");
  int rc = validate_mesh(d);
  if (rc) return rc;
  Carver cv(nullptr);
  *bytes = mesh_layout(layout_for(d), d->deterministic != 0, cv, nullptr);
  return SW_OK;
}

int mesh_create(sw_ctx* ctx, const sw_mesh_desc* d, void* ws, size_t ws_bytes, sw_mesh** out) {
  if (!ctx || !out) return fail(SW_EINVAL, "NULL argument");
  int rc = validate_mesh(d);
  if (rc) return rc;
  const HostLayout& L = layout_for(d);
  if (L.max_tile_nodes > TILE_MAX_NODES) return fail(SW_EMESH, "tile exceeds the LDS node capacity");
  const bool det = d->deterministic != 0;
  Carver dry(nullptr);
  const size_t need = mesh_layout(L, det, dry, nullptr);
  if (!ws || ((uintptr_t)ws & 255)) return fail(SW_ENOWS, "mesh workspace NULL or not 256-byte aligned");
  if (ws_bytes < need) return fail(SW_ENOWS, "mesh workspace %zu bytes < %zu needed", ws_bytes, need);
  HIPC(hipSetDevice(ctx->device));
  Carver cv(ws);
  MeshDev md;
  mesh_layout(L, det, cv, &md);
  hipStream_t s = ctx->stream;
  HIPC(up(md.conn_loc, L.conn_loc, s));
  HIPC(up(md.tile_elem_off, L.tile_elem_off, s));
  HIPC(up(md.tile_node_off, L.tile_node_off, s));
  HIPC(up(md.tile_nodes, L.tile_nodes, s));
  HIPC(up(md.tile_int_base, L.tile_int_base, s));
  HIPC(up(md.tile_nint, L.tile_nint, s));
  HIPC(up(md.tile_face_off, L.tile_face_off, s));
  HIPC(up(md.xyz, L.xyz, s));
  HIPC(up(md.fconn, L.fconn, s));
  HIPC(up(md.fconn_loc, L.fconn_loc, s));
  HIPC(up(md.face_elem, L.face_elem, s));
  HIPC(up(md.face_role, L.face_role, s));
  HIPC(up(md.node_u2i, L.node_u2i, s));
  HIPC(up(md.node_i2u, L.node_i2u, s));
  HIPC(up(md.inv_valence, L.inv_valence, s));
  if (det) {
    Incidence I;
    build_incidence(L, I);
    HIPC(up(md.inc_off, I.elem_off, s));
    HIPC(up(md.inc, I.elem, s));
    HIPC(up(md.finc_off, I.face_off, s));
    HIPC(up(md.finc, I.face, s));
    // the uploads read the host lists: finish them before I goes away
    HIPC(hipStreamSynchronize(s));
  }
  launch_geom(md, (float*)md.geo32, (double*)md.geo64, s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  sw_mesh* m = new sw_mesh{ctx, md, d->n_nodes, d->n_tets, d->n_faces, L.elem_order, L.node_u2i, L.node_i2u};
  *out = m;
  return SW_OK;
}

}  // namespace

extern "C" int sw_mesh_workspace_bytes(const sw_mesh_desc* d, size_t* bytes) {
  return host_guarded([&] { return mesh_workspace_bytes(d, bytes); });
}

extern "C" int sw_mesh_create(sw_ctx* ctx, const sw_mesh_desc* d, void* ws, size_t ws_bytes, sw_mesh** out) {
  return host_guarded([&] { return mesh_create(ctx, d, ws, ws_bytes, out); });
}

extern "C" int sw_mesh_info(const sw_mesh* m, int32_t* n_tiles, int32_t* max_tile_nodes) {
  if (!m) return fail(SW_EINVAL, "NULL mesh");
  if (n_tiles) *n_tiles = (int32_t)m->dev.n_tiles;
  if (max_tile_nodes) *max_tile_nodes = (int32_t)m->dev.max_tile_nodes;
  return SW_OK;
}

extern "C" int sw_mesh_destroy(sw_mesh* m) {
  delete m;
  return SW_OK;
}

// ------------------------------------------------------------ case

static size_t case_layout(const sw_mesh* m, const sw_case_desc* d, Carver& cv, sw_case* c) {
  const int64_t nn = m->n_nodes, nd = 3 * nn;
  const bool mixed = d->precision != SW_FP64;
  const bool flex = d->precision == SW_MIXED_FP32_FLEX;
  auto mats = cv.take<MatDev>(d->n_mat);
  auto em = cv.take<uint8_t>(m->n_tets);
  auto rec = cv.take<int32_t>(std::max(d->n_rec, 1));
  auto vin = cv.take<double>(3 * (d->n_steps + 1));
  double* vec[9];
  for (int i = 0; i < 9; ++i) vec[i] = cv.take<double>(nd);
  auto hist = cv.take<double>(4 * nd);
  auto diag6 = cv.take<double>(6 * nn);
  auto pinv64 = cv.take<double>(6 * nn);
  auto pinv16 = cv.take<__half>(6 * nn);
  auto pmax = cv.take<double>(1);
  float* f32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  if (mixed)
    for (int i = 0; i < 5; ++i) f32[i] = cv.take<float>(nd);
  uint16_t* p16 = d->precision == SW_MIXED_FP16 ? cv.take<uint16_t>(nd) : nullptr;
  double* fvec[4] = {nullptr, nullptr, nullptr, nullptr};
  double* fdots = nullptr;
  if (flex) {
    for (int i = 0; i < 4; ++i) fvec[i] = cv.take<double>(nd);
    fdots = cv.take<double>(8);
  }
  auto wave = cv.take<double>(std::max<int64_t>(d->n_steps * 3 * d->n_rec, 1));
  auto log_it = cv.take<int32_t>(d->n_steps);
  auto log_rel = cv.take<double>(d->n_steps);
  auto ctl = cv.take<CgCtl>(2);
  auto bad = cv.take<int32_t>(1);
  auto mis_buf = cv.take<double>(2 * 3 * std::max(d->n_rec, 1) + 2);
  float* nbh = nullptr;
  float* node_mat = nullptr;
  if (d->guess == SW_GUESS_POLY || d->guess == SW_GUESS_MLP || d->guess == SW_GUESS_PROJ_MLP) {
    nbh = cv.take<float>(4 * nd);
    node_mat = cv.take<float>(2 * nn);
  }
  double *det_e = nullptr, *det_f = nullptr;
  if (d->deterministic) {
    det_e = cv.take<double>(30 * m->n_tets);
    det_f = cv.take<double>(18 * std::max<int64_t>(m->n_faces, 1));
  }
  double *pX = nullptr, *pY = nullptr, *ppart = nullptr, *pout = nullptr, *pth = nullptr;
  const bool proj_guess = d->guess == SW_GUESS_PROJ || d->guess == SW_GUESS_PROJ_MLP;
  const int L = proj_guess ? (d->proj_dim > 0 ? d->proj_dim : 6) : 0;
  const int LS = L + (d->guess == SW_GUESS_PROJ_MLP ? 1 : 0);
  if (L > 0) {
    pX = cv.take<double>((size_t)LS * nd);
    pY = cv.take<double>((size_t)LS * nd);
    ppart = cv.take<double>((size_t)PROJ_BLOCKS * 2 * LS);
    pout = cv.take<double>(2 * LS);
    pth = cv.take<double>(LS);
  }
  if (c) {
    c->mats = mats;
    c->emat = em;
    c->rec = rec;
    c->vin = vin;
    c->u = vec[0];
    c->v = vec[1];
    c->a = vec[2];
    c->b = vec[3];
    c->x = vec[4];
    c->r = vec[5];
    c->z = vec[6];
    c->p = vec[7];
    c->q = vec[8];
    c->hist = hist;
    c->diag6 = diag6;
    c->pinv64 = pinv64;
    c->pinv16 = pinv16;
    c->pmax = pmax;
    c->r32 = f32[0];
    c->d32 = f32[1];
    c->z32 = f32[2];
    c->p32 = f32[3];
    c->q32 = f32[4];
    c->p16 = p16;
    c->fp[0] = fvec[0];
    c->fp[1] = fvec[1];
    c->fq[0] = fvec[2];
    c->fq[1] = fvec[3];
    c->fdots = fdots;
    c->wave = wave;
    c->log_it = log_it;
    c->log_rel = log_rel;
    c->ctl64 = ctl;
    c->ctl32 = ctl ? ctl + 1 : nullptr;
    c->bad = bad;
    c->mis_buf = mis_buf;
    c->nbh = nbh;
    c->node_mat = node_mat;
    c->det = d->deterministic != 0;
    c->det_e = det_e;
    c->det_f = det_f;
    c->proj_dim = L;
    c->proj_slots = LS;
    c->projX = pX;
    c->projY = pY;
    c->proj_part = ppart;
    c->proj_out = pout;
    c->proj_theta = pth;
  }
  return cv.off;
}

static int validate_case(const sw_mesh* m, const sw_case_desc* d) {
  if (!m || !d) return fail(SW_EINVAL, "NULL argument");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(SW_EINVAL, "dt must be > 0");
  if (!(d->ray_alpha >= 0.0) || !(d->ray_beta >= 0.0)) return fail(SW_EINVAL, "Rayleigh coefficients must be >= 0");
  if (!(d->rtol > 0.0 && d->rtol < 1.0)) return fail(SW_EINVAL, "rtol must be in (0, 1)");
  if (d->max_iter <= 0) return fail(SW_EINVAL, "max_iter must be > 0");
  if (d->precision != SW_FP64 && d->precision != SW_MIXED_FP32 && d->precision != SW_MIXED_FP32_FLEX &&
      d->precision != SW_MIXED_FP16)
    return fail(SW_EINVAL, "unknown precision %d", d->precision);
  if (d->guess != SW_GUESS_ZERO && d->guess != SW_GUESS_POLY && d->guess != SW_GUESS_MLP &&
      d->guess != SW_GUESS_PROJ && d->guess != SW_GUESS_PROJ_MLP)
    return fail(SW_EINVAL, "unknown guess kind %d", d->guess);
  if (d->guess == SW_GUESS_PROJ && d->proj_dim != 0 && (d->proj_dim < 2 || d->proj_dim > PROJ_MAX))
    return fail(SW_EINVAL, "proj_dim must be 0 or 2..%d", PROJ_MAX);
  if (d->guess == SW_GUESS_PROJ_MLP && d->proj_dim != 0 && (d->proj_dim < 2 || d->proj_dim > PROJ_MAX - 1))
    return fail(SW_EINVAL, "proj_dim must be 0 or 2..%d with the network's direction", PROJ_MAX - 1);
  if (d->poly_order < 0 || d->poly_order > 3) return fail(SW_EINVAL, "poly_order must be 0..3");
  if (d->deterministic != 0 && d->deterministic != 1) return fail(SW_EINVAL, "deterministic must be 0 or 1");
  if (d->deterministic) {
    if (d->precision != SW_FP64) return fail(SW_EINVAL, "deterministic cases need SW_FP64");
    if (d->guess != SW_GUESS_ZERO && d->guess != SW_GUESS_POLY && d->guess != SW_GUESS_PROJ)
      return fail(SW_EINVAL, "deterministic cases take the zero, polynomial or projection guess");
    if (!m->dev.inc) return fail(SW_EINVAL, "deterministic cases need a mesh created with deterministic = 1");
  }
  if (!(d->inner_rtol >= 0.0 && d->inner_rtol < 1.0)) return fail(SW_EINVAL, "inner_rtol must be in [0, 1)");
  if (d->n_mat < 1 || d->n_mat > 255 || !d->mat) return fail(SW_EINVAL, "n_mat must be 1..255 with a table");
  for (int i = 0; i < d->n_mat; ++i) {
    const double vp = d->mat[3 * i], vs = d->mat[3 * i + 1], rho = d->mat[3 * i + 2];
    if (!(vp > 0 && vs > 0 && rho > 0) || !(vp * vp > 4.0 / 3.0 * vs * vs))
      return fail(SW_EINVAL, "material %d (Vp %g Vs %g rho %g) is not a valid elastic solid", i, vp, vs, rho);
  }
  if (!d->tet_mat) return fail(SW_EINVAL, "tet_mat is NULL");
  for (int64_t e = 0; e < m->n_tets; ++e)
    if (d->tet_mat[e] >= d->n_mat) return fail(SW_EINVAL, "tet %lld material %d >= n_mat", (long long)e, d->tet_mat[e]);
  if (d->n_rec < 0 || (d->n_rec > 0 && !d->rec_node)) return fail(SW_EINVAL, "bad receivers");
  for (int i = 0; i < d->n_rec; ++i)
    if (d->rec_node[i] < 0 || d->rec_node[i] >= m->n_nodes) return fail(SW_EINVAL, "receiver %d node out of range", i);
  if (d->n_steps < 1 || !d->v_in) return fail(SW_EINVAL, "n_steps must be >= 1 with a v_in array");
  for (int64_t i = 0; i < 3 * (d->n_steps + 1); ++i)
    if (!std::isfinite(d->v_in[i])) return fail(SW_EINVAL, "non-finite v_in");
  return SW_OK;
}


extern "C" int sw_case_workspace_bytes(const sw_mesh* m, const sw_case_desc* d, size_t* bytes) {
  if (!m || !d || !bytes) return fail(SW_EINVAL, "NULL argument");
  if (d->n_mat < 1 || d->n_rec < 0 || d->n_steps < 1) return fail(SW_EINVAL, "bad case sizes");
  Carver cv(nullptr);
  *bytes = case_layout(m, d, cv, nullptr);
  return SW_OK;
}

namespace {

void op_scales(const sw_case* c, int op, double* sM, double* sK, double* sC) {
  if (op == SW_OP_A) {
    *sM = c->cM;
    *sK = c->cK;
    *sC = c->cC;
  } else {
    *sM = (op & SW_OP_M) ? 1.0 : 0.0;
    *sK = (op & SW_OP_K) ? 1.0 : 0.0;
    *sC = (op & SW_OP_CABS) ? 1.0 : 0.0;
  }
}

// y = op x (internal order).  y's shared-node entries must be zero on entry
// (interior entries are overwritten).
int apply_f64(sw_case* c, int op, const double* x, double* y, CgCtl* ctl, int iter, hipStream_t s) {
  TileArgs<double> A{};
  op_scales(c, op, &A.sM, &A.sK, &A.sC);
  A.x1 = x;
  A.a1 = 1.0;
  A.xf = x;
  A.y = y;
  A.eout = c->det_e;
  A.fout = c->det_f;
  launch_tile_f64(c->mesh->dev, c->emat, c->mats, A, ctl, iter, s);
  LAUNCHED();
  return SW_OK;
}
int apply_f64(sw_case* c, int op, const double* x, double* y, CgCtl* ctl, int iter) {
  return apply_f64(c, op, x, y, ctl, iter, c->ctx->stream);
}

int apply_f32(sw_case* c, int op, const float* x, float* y, CgCtl* ctl, int iter, hipStream_t s) {
  TileArgs<float> A{};
  double sM, sK, sC;
  op_scales(c, op, &sM, &sK, &sC);
  A.sM = (float)sM;
  A.sK = (float)sK;
  A.sC = (float)sC;
  A.x1 = x;
  A.a1 = 1.0f;
  A.xf = x;
  A.y = y;
  A.n_mat = c->n_mat;
  launch_tile_f32(c->mesh->dev, c->emat, c->mats, A, ctl, iter, case_grid_cap(c), s);
  LAUNCHED();
  return SW_OK;
}
int apply_f32(sw_case* c, int op, const float* x, float* y, CgCtl* ctl, int iter) {
  return apply_f32(c, op, x, y, ctl, iter, c->ctx->stream);
}

// y = A x with x in bfloat16 (the SW_MIXED_FP16 inner CG's direction)
int apply_f32_h(sw_case* c, const uint16_t* x, float* y, CgCtl* ctl, int iter, hipStream_t s) {
  TileArgs<float> A{};
  A.sM = (float)c->cM;
  A.sK = (float)c->cK;
  A.sC = (float)c->cC;
  A.x1h = x;
  A.a1 = 1.0f;
  A.y = y;
  A.n_mat = c->n_mat;
  launch_tile_f32(c->mesh->dev, c->emat, c->mats, A, ctl, iter, case_grid_cap(c), s);
  LAUNCHED();
  return SW_OK;
}

// Right-hand side of step c->step -> c->step + 1 (internal order) into y:
// y = M (a + (4/dt + alpha) v) + C_abs v + F  then  y += -K (u - beta v).
int build_rhs(sw_case* c, double* y) {
  hipStream_t s = c->ctx->stream;
  const int64_t nd = 3 * c->mesh->n_nodes;
  // the first pass stores the interior nodes and adds into the shared ones
  const int64_t ni3 = 3 * c->mesh->dev.n_interior;
  launch_fill_f64(nd - ni3, y + ni3, 0.0, s);
  TileArgs<double> A{};
  A.sM = 1.0;
  A.sK = 0.0;
  A.sC = 1.0;
  A.x1 = c->a;
  A.a1 = 1.0;
  A.x2 = c->v;
  A.a2 = 4.0 / c->dt + c->alpha;
  A.xf = c->v;
  A.vin = c->vin + 3 * (c->step + 1);
  A.y = y;
  A.accumulate = 0;
  A.eout = c->det_e;
  A.fout = c->det_f;
  launch_tile_f64(c->mesh->dev, c->emat, c->mats, A, nullptr, -1, s);
  TileArgs<double> B{};
  B.sM = 0.0;
  B.sK = -1.0;
  B.sC = 0.0;
  B.x1 = c->u;
  B.a1 = 1.0;
  B.x2 = c->v;
  B.a2 = -c->beta;
  B.y = y;
  B.accumulate = 1;
  B.eout = c->det_e;
  B.fout = c->det_f;
  launch_tile_f64(c->mesh->dev, c->emat, c->mats, B, nullptr, -1, s);
  LAUNCHED();
  return SW_OK;
}

}  // namespace

extern "C" int sw_case_create(sw_ctx* ctx, sw_mesh* m, const sw_case_desc* d, void* ws, size_t ws_bytes,
                              sw_case** out) {
  if (!ctx || !out) return fail(SW_EINVAL, "NULL argument");
  int rc = validate_case(m, d);
  if (rc) return rc;
  Carver dry(nullptr);
  const size_t need = case_layout(m, d, dry, nullptr);
  if (!ws || ((uintptr_t)ws & 255)) return fail(SW_ENOWS, "case workspace NULL or not 256-byte aligned");
  if (ws_bytes < need) return fail(SW_ENOWS, "case workspace %zu bytes < %zu needed", ws_bytes, need);
  HIPC(hipSetDevice(ctx->device));
  sw_case* c = new sw_case();
  c->ctx = ctx;
  c->mesh = m;
  c->dt = d->dt;
  c->alpha = d->ray_alpha;
  c->beta = d->ray_beta;
  c->rtol = d->rtol;
  c->inner_rtol = d->inner_rtol > 0.0 ? d->inner_rtol : 1e-4;
  c->max_iter = d->max_iter;
  c->precision = d->precision;
  c->guess = d->guess;
  c->poly_order = d->poly_order;
  c->n_mat = d->n_mat;
  c->n_rec = d->n_rec;
  c->n_steps = d->n_steps;
  c->cM = 4.0 / (d->dt * d->dt) + 2.0 * d->ray_alpha / d->dt;
  c->cK = 1.0 + 2.0 * d->ray_beta / d->dt;
  c->cC = 2.0 / d->dt;
  Carver cv(ws);
  case_layout(m, d, cv, c);
  hipStream_t s = ctx->stream;
  std::vector<MatDev> mats(d->n_mat);
  for (int i = 0; i < d->n_mat; ++i) {
    const double vp = d->mat[3 * i], vs = d->mat[3 * i + 1], rho = d->mat[3 * i + 2];
    mats[i].mu = rho * vs * vs;
    mats[i].lam = rho * vp * vp - 2.0 * mats[i].mu;
    mats[i].rho = rho;
    mats[i].zp = rho * vp;
    mats[i].zs = rho * vs;
  }
  std::vector<uint8_t> em(m->n_tets);
  for (int64_t i = 0; i < m->n_tets; ++i) em[i] = d->tet_mat[m->elem_order[i]];
  std::vector<int32_t> rec(std::max(d->n_rec, 1), 0);
  for (int i = 0; i < d->n_rec; ++i) rec[i] = m->node_u2i[d->rec_node[i]];
  const int64_t nn = m->n_nodes, nd = 3 * nn;
  auto cleanup = [&](int code) {
    delete c;
    return code;
  };
#define HIPX(expr)                                                                                       \
  do {                                                                                                   \
    hipError_t _e = (expr);                                                                              \
    if (_e != hipSuccess) return cleanup(fail(SW_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e))); \
  } while (0)
  HIPX(hipMemcpyAsync(c->mats, mats.data(), mats.size() * sizeof(MatDev), hipMemcpyHostToDevice, s));
  HIPX(hipMemcpyAsync(c->emat, em.data(), em.size(), hipMemcpyHostToDevice, s));
  HIPX(hipMemcpyAsync(c->rec, rec.data(), 4 * rec.size(), hipMemcpyHostToDevice, s));
  HIPX(hipMemcpyAsync(c->vin, d->v_in, 8 * 3 * (size_t)(d->n_steps + 1), hipMemcpyHostToDevice, s));
  double* zero_vecs[] = {c->u, c->v, c->a, c->b, c->x, c->r, c->z, c->p, c->q};
  for (double* zv : zero_vecs) launch_fill_f64(nd, zv, 0.0, s);
  launch_fill_f64(4 * nd, c->hist, 0.0, s);
  if (c->precision != SW_FP64) {
    float* zf[] = {c->r32, c->d32, c->z32, c->p32, c->q32};
    for (float* zv : zf) launch_fill_f32(nd, zv, 0.0f, s);
    if (c->p16) HIPX(hipMemsetAsync(c->p16, 0, 2 * (size_t)nd, s));
  }
  if (c->precision == SW_MIXED_FP32_FLEX) {
    double* zf[] = {c->fp[0], c->fp[1], c->fq[0], c->fq[1]};
    for (double* zv : zf) launch_fill_f64(nd, zv, 0.0, s);
    launch_fill_f64(8, c->fdots, 0.0, s);
  }
  launch_fill_f64(std::max<int64_t>(c->n_steps * 3 * c->n_rec, 1), c->wave, 0.0, s);
  launch_fill_f64((int64_t)(2 * sizeof(CgCtl) / 8), (double*)c->ctl64, 0.0, s);
  launch_fill_f64(c->n_steps, c->log_rel, 0.0, s);
  HIPX(hipMemsetAsync(c->log_it, 0, 4 * (size_t)c->n_steps, s));
  // preconditioner: inverse 3x3 diagonal blocks of A
  launch_fill_f64(6 * nn, c->diag6, 0.0, s);
  HIPX(hipMemsetAsync(c->bad, 0, 4, s));
  launch_tile_diag(m->dev, c->emat, c->mats, c->cM, c->cK, c->cC, c->diag6, s, c->det_e, c->det_f);
  launch_invert_blocks(nn, c->diag6, c->pinv64, c->pinv16, c->pmax, c->bad, s);
  HIPX(hipGetLastError());
  int32_t bad = 0;
  HIPX(hipMemcpyAsync(&bad, c->bad, 4, hipMemcpyDeviceToHost, s));
  HIPX(hipStreamSynchronize(s));
  if (bad) return cleanup(fail(SW_EINVAL, "a diagonal block of the step operator is not positive definite"));
  if (c->proj_dim > 0) {
    launch_fill_f64((int64_t)c->proj_slots * nd, c->projX, 0.0, s);
    launch_fill_f64((int64_t)c->proj_slots * nd, c->projY, 0.0, s);
    c->projG.assign((size_t)c->proj_dim * c->proj_dim, 0.0);
    c->proj_h.assign(2 * (size_t)c->proj_slots, 0.0);
    c->proj_th.assign(c->proj_slots, 0.0);
    c->proj_rows.assign((size_t)c->proj_dim * c->proj_dim, 0.0);
    c->proj_pend.clear();
    HIPX(hipGetLastError());
  }
  if (c->nbh) {
    launch_fill_f32(4 * nd, c->nbh, 0.0f, s);
    launch_fill_f32(2 * nn, c->node_mat, 0.0f, s);
    launch_node_material(m->dev, c->emat, c->mats, c->node_mat, s);
    HIPX(hipGetLastError());
    HIPX(hipStreamSynchronize(s));
  }
#undef HIPX
  *out = c;
  return SW_OK;
}

extern "C" int sw_case_destroy(sw_case* c) {
  if (c)
    for (hipGraphExec_t g : c->cg_graph)
      if (g) (void)hipGraphExecDestroy(g);
  delete c;
  return SW_OK;
}

extern "C" int sw_case_set_state(sw_case* c, const double* u, const double* v, const double* a, int64_t step) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (step < 0 || step > c->n_steps) return fail(SW_EINVAL, "step %lld out of range", (long long)step);
  HIPC(hipSetDevice(c->ctx->device));
  const int64_t nn = c->mesh->n_nodes;
  hipStream_t s = c->ctx->stream;
  std::vector<double> tmp(3 * nn);
  const double* src[3] = {u, v, a};
  double* dst[3] = {c->u, c->v, c->a};
  for (int k = 0; k < 3; ++k) {
    if (!src[k]) continue;
    for (int64_t i = 0; i < nn; ++i) {
      const int64_t j = c->mesh->node_u2i[i];
      for (int d = 0; d < 3; ++d) tmp[3 * j + d] = src[k][3 * i + d];
    }
    HIPC(hipMemcpyAsync(dst[k], tmp.data(), 8 * tmp.size(), hipMemcpyHostToDevice, s));
    HIPC(hipStreamSynchronize(s));
  }
  launch_fill_f64(4 * 3 * nn, c->hist, 0.0, s);
  LAUNCHED();
  HIPC(hipStreamSynchronize(s));
  c->step = step;
  c->hist_count = 0;
  c->hist_head = 3;
  c->nb_count = 0;
  c->nb_head = 3;
  c->proj_count = 0;
  c->proj_head = -1;
  c->proj_pend.clear();
  if (c->proj_dim > 0) std::fill(c->projG.begin(), c->projG.end(), 0.0);
  return SW_OK;
}

extern "C" int sw_case_get_state(const sw_case* c, double* u, double* v, double* a, int64_t* step) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  HIPC(hipSetDevice(c->ctx->device));
  const int64_t nn = c->mesh->n_nodes;
  hipStream_t s = c->ctx->stream;
  std::vector<double> tmp(3 * nn);
  double* dst[3] = {u, v, a};
  const double* src[3] = {c->u, c->v, c->a};
  for (int k = 0; k < 3; ++k) {
    if (!dst[k]) continue;
    HIPC(hipMemcpyAsync(tmp.data(), src[k], 8 * tmp.size(), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nn; ++i) {
      const int64_t j = c->mesh->node_u2i[i];
      for (int d = 0; d < 3; ++d) dst[k][3 * i + d] = tmp[3 * j + d];
    }
  }
  if (step) *step = c->step;
  return SW_OK;
}

// ------------------------------------------------------------ solver

namespace {

int read_ctl(sw_case* c, CgCtl* dev, CgCtl* host) {
  HIPC(hipMemcpyAsync(host, dev, sizeof(CgCtl), hipMemcpyDeviceToHost, c->ctx->stream));
  HIPC(hipStreamSynchronize(c->ctx->stream));
  return c->ctx->prof.on ? prof_flush(c->ctx) : SW_OK;
}

// Runs CG iterations of the solve in `ctl` until its done flag is set.  The
// first chunk is sized from the previous solve's count; later ones are short
// so that few launches are spent after convergence.
// One CG iteration of the single-case solve on stream s: the operator pass
// (iteration `iter` of the solve: parity and the first-iteration test), the
// update and the direction kernels (iter_abs: the iteration's index in the
// step, or -1 to take it from the control block).
template <bool F32>
int cg_iteration(sw_case* c, CgCtl* ctl, int iter, int iter_abs, hipStream_t s, bool prof) {
  const int64_t nn = c->mesh->n_nodes;
  sw_ctx* cx = c->ctx;
  int rc;
  if (F32) {
    int ev = prof ? prof_begin(cx, SW_PROF_TILE_F32) : -1;
    rc = c->p16 ? apply_f32_h(c, c->p16, c->q32, ctl, iter, s) : apply_f32(c, SW_OP_A, c->p32, c->q32, ctl, iter, s);
    if (prof) prof_end(cx, ev);
    if (rc) return rc;
    ev = prof ? prof_begin(cx, SW_PROF_UPDATE_F32) : -1;
    launch_cg_update_f32(nn, c->mesh->dev.n_interior, iter & 1, c->pinv16, c->r32, c->z32, c->q32, ctl, s);
    if (prof) prof_end(cx, ev);
    ev = prof ? prof_begin(cx, SW_PROF_DIR_F32) : -1;
    if (c->p16)
      launch_cg_dir_h(nn, iter & 1, iter_abs, c->max_iter, c->z32, c->p16, c->d32, ctl, s);
    else
      launch_cg_dir_f32(nn, iter & 1, iter_abs, c->max_iter, c->z32, c->p32, c->d32, ctl, s);
    if (prof) prof_end(cx, ev);
  } else {
    int ev = prof ? prof_begin(cx, SW_PROF_TILE_F64) : -1;
    rc = apply_f64(c, SW_OP_A, c->p, c->q, ctl, iter, s);
    if (prof) prof_end(cx, ev);
    if (rc) return rc;
    ev = prof ? prof_begin(cx, SW_PROF_UPDATE_F64) : -1;
    launch_cg_update_f64(nn, iter & 1, c->pinv64, c->r, c->z, c->q, ctl, s, c->det);
    if (prof) prof_end(cx, ev);
    ev = prof ? prof_begin(cx, SW_PROF_DIR_F64) : -1;
    launch_cg_dir_f64(nn, iter & 1, iter_abs, c->max_iter, c->z, c->p, c->x, ctl, s);
    if (prof) prof_end(cx, ev);
  }
  LAUNCHED();
  return SW_OK;
}

// The capture stream of a context (created on first use; default priority).
int capture_stream(sw_ctx* cx, hipStream_t* out) {
  if (!cx->cap_stream) HIPC(hipStreamCreateWithFlags(&cx->cap_stream, hipStreamNonBlocking));
  *out = cx->cap_stream;
  return SW_OK;
}

// Instantiated graph of two CG iterations of this case's solve (an even
// iteration then an odd one, past the first: the direction kernels take
// the iteration index from the control block), captured once per case and
// precision (again when the grid cap changes).  The captured kernels read
// and write only the case's vectors and control block, so every replay
// continues the solve in the control block.  *out stays null if capture is
// not available (the caller then launches the kernels directly).
template <bool F32>
int cg_pair_graph(sw_case* c, CgCtl* ctl, hipGraphExec_t* out) {
  const int slot = F32 ? 1 : 0;
  if (c->cg_graph[slot] && c->cg_graph_cap[slot] == case_grid_cap(c)) {
    *out = c->cg_graph[slot];
    return SW_OK;
  }
  if (c->cg_graph[slot]) {
    HIPC(hipGraphExecDestroy(c->cg_graph[slot]));
    c->cg_graph[slot] = nullptr;
  }
  hipStream_t cs;
  int rc = capture_stream(c->ctx, &cs);
  if (rc) return rc;
  HIPC(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < 2 && !rc; ++k) rc = cg_iteration<F32>(c, ctl, 2 + k, -1, cs, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc) return rc;
  if (e != hipSuccess) return fail(SW_EHIP, "CG graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return fail(SW_EHIP, "CG graph instantiation failed: %s", hipGetErrorString(e2));
  c->cg_graph[slot] = ex;
  c->cg_graph_cap[slot] = case_grid_cap(c);
  *out = ex;
  return SW_OK;
}

template <bool F32>
int cg_loop(sw_case* c, CgCtl* ctl, int iter_base, int first_chunk, int* iters_out) {
  const int64_t nn = c->mesh->n_nodes;
  hipStream_t s = c->ctx->stream;
  sw_ctx* cx = c->ctx;
  int it = 0;
  // the first chunk has an even count, so that the chunks of two that follow
  // start at even iterations (the parity a captured pair assumes)
  int chunk = std::max(2, first_chunk + (first_chunk & 1));
  CgCtl h;
  for (;;) {
    hipGraphExec_t g = nullptr;
    if (it > 0 && chunk == 2 && cx->graphs && !cx->prof.on) {
      int rc = cg_pair_graph<F32>(c, ctl, &g);
      if (rc) return rc;
    }
    if (g) {
      HIPC(hipGraphLaunch(g, s));
    } else {
      for (int k = 0; k < chunk; ++k) {
        int rc = cg_iteration<F32>(c, ctl, it + k, iter_base + it + k, s, true);
        if (rc) return rc;
      }
    }
    LAUNCHED();
    it += chunk;
    int rc = read_ctl(c, ctl, &h);
    if (rc) return rc;
    if (h.done) break;
    chunk = 2;
  }
  *iters_out = h.iters - iter_base > 0 ? h.iters - iter_base : 0;
  return SW_OK;
}

// FP64 true residual of x: q = A x, r = b - q, rr_true into ctl64.  q keeps
// A x unless zero_q is set; then its shared nodes are cleared, which is all
// the next operator pass into q needs (it stores the interior nodes and
// adds into the shared ones).
int true_residual(sw_case* c, CgCtl* hctl, bool zero_q) {
  hipStream_t s = c->ctx->stream;
  const int64_t nd = 3 * c->mesh->n_nodes;
  launch_fill_f64(1, &c->ctl64->rr_true, 0.0, s);
  int rc = apply_f64(c, SW_OP_A, c->x, c->q, nullptr, -1);
  if (rc) return rc;
  launch_true_residual(nd, c->b, c->q, c->r, c->ctl64, s, c->det);
  if (zero_q) {
    const int64_t ni3 = 3 * c->mesh->dev.n_interior;
    launch_fill_f64(nd - ni3, c->q + ni3, 0.0, s);
  }
  LAUNCHED();
  return read_ctl(c, c->ctl64, hctl);
}

MlpFeat mlp_features(const sw_case* c) {
  MlpFeat F;
  F.n_dof = 3 * c->mesh->n_nodes;
  F.hist = c->hist;
  F.head = c->hist_head;
  F.nbh = c->nbh;
  F.nb_head = c->nb_head;
  F.node_mat = c->node_mat;
  return F;
}

// GUESS_PROJ_NET: the projection with the network's correction as one more
// direction (SW_GUESS_PROJ_MLP once the network has its four increments)
enum { GUESS_NONE = 0, GUESS_EXTRAP = 1, GUESS_NET = 2, GUESS_PROJ = 3, GUESS_PROJ_NET = 4 };

inline bool projected(int g) { return g == GUESS_PROJ || g == GUESS_PROJ_NET; }

// The network's direction for GUESS_PROJ_NET: its correction w = s * y into
// the extra slot X_L and the image A w into Y_L (one FP64 operator pass).
int proj_net_direction(sw_case* c) {
  hipStream_t s = c->ctx->stream;
  const int L = c->proj_dim;
  const int64_t nd = 3 * c->mesh->n_nodes;
  double* Xw = c->projX + (size_t)L * nd;
  double* Yw = c->projY + (size_t)L * nd;
  launch_mlp_guess(mlp_features(c), c->mlp->theta, Xw, c->ctl64, true, s);
  launch_fill_f64(nd, Yw, 0.0, s);
  LAUNCHED();
  return apply_f64(c, SW_OP_A, Xw, Yw, nullptr, -1);
}

// Projection guess, first half: X_i . b for the ring, copied to the host,
// together with the Gram rows X_i . A X_s = X_i . Y_s of the slots stored
// since the last projection (the last of them in the same pass over the
// ring as X_i . b).  extra: the network's direction in slot L joins, with
// X_i . b and X_i . Y_L over all L + 1 slots in one pass (the ring's new
// rows then each take a pass of their own).
int proj_begin(sw_case* c, bool extra = false) {
  hipStream_t s = c->ctx->stream;
  const int L = c->proj_dim;
  const int64_t nd = 3 * c->mesh->n_nodes;
  const int np = (int)c->proj_pend.size();
  for (int k = 0; k + (extra ? 0 : 1) < np; ++k) {
    const int p = c->proj_pend[k];
    launch_proj_dots(L, nd, c->projX, c->projY + (size_t)p * nd, nullptr, c->proj_part, c->proj_out, s);
    HIPC(hipMemcpyAsync(c->proj_rows.data() + (size_t)p * L, c->proj_out, L * sizeof(double),
                        hipMemcpyDeviceToHost, s));
  }
  int nout;
  if (extra) {
    launch_proj_dots2(L + 1, nd, c->projX, c->b, c->projY + (size_t)L * nd, c->proj_part, c->proj_out, s);
    nout = 2 * (L + 1);
  } else if (np > 0) {
    const int p = c->proj_pend[np - 1];
    launch_proj_dots2(L, nd, c->projX, c->b, c->projY + (size_t)p * nd, c->proj_part, c->proj_out, s);
    nout = 2 * L;
  } else {
    launch_proj_dots(L, nd, c->projX, c->b, nullptr, c->proj_part, c->proj_out, s);
    nout = L;
  }
  LAUNCHED();
  HIPC(hipMemcpyAsync(c->proj_h.data(), c->proj_out, nout * sizeof(double), hipMemcpyDeviceToHost, s));
  return SW_OK;
}

// Second half (after a synchronisation): theta from the Gram matrix of the
// filled slots (and the network's direction with extra), x = X theta;
// with_res: also r = b - Y theta and its norm in ctl64->rr_true (the
// residual of x from the stored images).
int proj_finish(sw_case* c, bool with_res, bool extra = false) {
  hipStream_t s = c->ctx->stream;
  const int L = c->proj_dim;
  const int64_t nd = 3 * c->mesh->n_nodes;
  // Gram rows and columns of the newly stored slots (A is symmetric and the
  // images are exact, so X_i . A X_p = X_p . A X_i)
  const int np = (int)c->proj_pend.size();
  for (int k = 0; k < np; ++k) {
    const int p = c->proj_pend[k];
    const double* row = (extra || k + 1 < np) ? c->proj_rows.data() + (size_t)p * L : c->proj_h.data() + L;
    for (int i = 0; i < L; ++i) {
      c->projG[(size_t)i * L + p] = row[i];
      c->projG[(size_t)p * L + i] = row[i];
    }
  }
  c->proj_pend.clear();
  int idx[PROJ_MAX];
  const int m = c->proj_count;
  for (int j = 0; j < m; ++j) idx[j] = ((c->proj_head - j) % L + L) % L;
  // with extra the system gains row and column m: the network's direction
  // (its right-hand side X_L . b and Gram entries X_i . Y_L from the pass)
  const int M = m + (extra ? 1 : 0);
  const int LS = L + 1;
  double Gs[PROJ_MAX * PROJ_MAX], hs[PROJ_MAX], ts[PROJ_MAX];
  for (int i = 0; i < m; ++i) {
    hs[i] = c->proj_h[idx[i]];
    for (int j = 0; j < m; ++j) Gs[i * M + j] = c->projG[(size_t)idx[i] * L + idx[j]];
  }
  if (extra) {
    const double* hb = c->proj_h.data();       // X_i . b, i = 0..L
    const double* hw = c->proj_h.data() + LS;  // X_i . Y_L, i = 0..L
    hs[m] = hb[L];
    for (int i = 0; i < m; ++i) Gs[i * M + m] = Gs[m * M + i] = hw[idx[i]];
    Gs[m * M + m] = hw[L];
  }
  // directions are kept down to FP64 resolution of the unit-diagonal Gram
  // matrix: the increments of a smooth march are nearly dependent, and the
  // step's new component lies in the directions of smallest energy
  psd_solve(M, Gs, M, hs, ts, 1e-16);
  std::fill(c->proj_th.begin(), c->proj_th.end(), 0.0);
  for (int i = 0; i < m; ++i) c->proj_th[idx[i]] = std::isfinite(ts[i]) ? ts[i] : 0.0;
  if (extra) c->proj_th[L] = std::isfinite(ts[m]) ? ts[m] : 0.0;
  const int K = extra ? LS : L;
  HIPC(hipMemcpyAsync(c->proj_theta, c->proj_th.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
  if (with_res)
    launch_proj_combine_res(K, nd, c->projX, c->projY, c->proj_theta, c->b, c->x, c->r, c->proj_part,
                            &c->ctl64->rr_true, s);
  else
    launch_proj_combine(K, nd, c->projX, c->proj_theta, c->x, s);
  LAUNCHED();
  return SW_OK;
}

// After a converged step (x = du, r = b - A du): du and A du = b - r enter
// the ring; the slot's Gram row waits for the next projection.
int proj_record(sw_case* c) {
  hipStream_t s = c->ctx->stream;
  const int L = c->proj_dim;
  const int64_t nd = 3 * c->mesh->n_nodes;
  const int sl = (c->proj_head + 1) % L;
  double* Xs = c->projX + (size_t)sl * nd;
  double* Ys = c->projY + (size_t)sl * nd;
  launch_proj_store(nd, c->x, c->b, c->r, Xs, Ys, s);
  LAUNCHED();
  auto& pend = c->proj_pend;
  pend.erase(std::remove(pend.begin(), pend.end(), sl), pend.end());
  pend.push_back(sl);
  c->proj_head = sl;
  c->proj_count = std::min(c->proj_count + 1, L);
  return SW_OK;
}

// Guess kind for the coming step of c.
int guess_kind(const sw_case* c) {
  const bool net = c->mlp && c->hist_count >= 4 && c->nb_count >= 4;
  if (c->guess == SW_GUESS_PROJ_MLP && c->proj_count >= 2) return net ? GUESS_PROJ_NET : GUESS_PROJ;
  if (c->guess == SW_GUESS_PROJ && c->proj_count >= 2) return GUESS_PROJ;
  if (c->guess == SW_GUESS_MLP && net) return GUESS_NET;
  if (c->guess != SW_GUESS_ZERO && c->hist_count > 0) return GUESS_EXTRAP;
  return GUESS_NONE;
}

// Writes the initial guess of kind g into c->x (the projection reads c->b;
// with_res: it also leaves its residual in c->r and ctl64->rr_true).
int set_guess(sw_case* c, int g, bool with_res = false) {
  hipStream_t s = c->ctx->stream;
  const int64_t nd = 3 * c->mesh->n_nodes;
  if (projected(g)) {
    const bool extra = g == GUESS_PROJ_NET;
    int rc = extra ? proj_net_direction(c) : SW_OK;
    if (!rc) rc = proj_begin(c, extra);
    if (rc) return rc;
    HIPC(hipStreamSynchronize(s));
    return proj_finish(c, with_res, extra);
  }
  if (g == GUESS_NET) {
    launch_mlp_guess(mlp_features(c), c->mlp->theta, c->x, c->ctl64, false, s);
  } else if (g == GUESS_EXTRAP) {
    const int order = std::min(c->poly_order, c->hist_count - 1);
    launch_guess_poly(nd, c->hist, c->hist_head, order, c->x, c->ctl64, s);
  } else {
    launch_fill_f64(nd, c->x, 0.0, s);
  }
  LAUNCHED();
  return SW_OK;
}

int solve_step(sw_case* c, int* iters, int* outer, double* relres, int* flags) {
  hipStream_t s = c->ctx->stream;
  const int64_t nn = c->mesh->n_nodes, nd = 3 * nn;
  *iters = 0;
  *outer = 0;
  *flags = 0;
  int rc = build_rhs(c, c->b);
  if (rc) return rc;
  launch_fill_f64(1, &c->ctl64->bb, 0.0, s);
  launch_norm2(nd, c->b, &c->ctl64->bb, s, c->det);
  launch_ctl_prepare(c->ctl64, c->rtol, s);
  // guess: the projection needs two past increments, the network four and
  // their neighbour means, extrapolation one; otherwise zero
  int g = guess_kind(c);
  rc = set_guess(c, g, c->precision != SW_FP64);
  if (rc) return rc;
  CgCtl h;
  if (c->precision == SW_FP64) {
    for (int attempt = 0;; ++attempt) {
      if (g != GUESS_NONE) {
        rc = apply_f64(c, SW_OP_A, c->x, c->q, nullptr, -1);
        if (rc) return rc;
        launch_cg_init_f64(nn, c->b, c->q, c->pinv64, c->r, c->z, c->p, c->q, c->ctl64, s, c->det);
      } else {
        launch_cg_init_f64(nn, c->b, nullptr, c->pinv64, c->r, c->z, c->p, nullptr, c->ctl64, s, c->det);
      }
      LAUNCHED();
      if ((g != GUESS_NET && !projected(g)) || attempt > 0) break;
      // reject a learned or projected guess whose residual exceeds that of
      // the zero guess
      rc = read_ctl(c, c->ctl64, &h);
      if (rc) return rc;
      double rr0 = 0.0;
      for (int k = 0; k < NSLOT; ++k) rr0 += h.rr[0][k];
      if (rr0 <= h.bb) break;
      *flags |= SW_FLAG_GUESS_FALLBACK;
      g = GUESS_EXTRAP;
      launch_ctl_prepare(c->ctl64, c->rtol, s);
      rc = set_guess(c, g);
      if (rc) return rc;
    }
    for (;;) {
      int it = 0;
      rc = cg_loop<false>(c, c->ctl64, *iters, c->last_iters - *iters - 1, &it);
      if (rc) return rc;
      *iters += it;
      rc = true_residual(c, &h, false);
      if (rc) return rc;
      ++*outer;
      bool stop = false;
      if (!(h.rr_true == h.rr_true)) {
        *flags |= SW_FLAG_NONFINITE;
        stop = true;
      } else if (h.rr_true <= c->rtol * c->rtol * h.bb) {
        stop = true;
      } else if (*iters >= c->max_iter) {
        *flags |= SW_FLAG_NOCONV;
        stop = true;
      }
      if (stop) {
        launch_fill_f64(nd, c->q, 0.0, s);
        LAUNCHED();
        break;
      }
      // restart CG from the current iterate on the true residual b - A x
      launch_ctl_prepare(c->ctl64, c->rtol, s);
      launch_cg_init_f64(nn, c->b, c->q, c->pinv64, c->r, c->z, c->p, c->q, c->ctl64, s, c->det);
      LAUNCHED();
    }
  } else {
    // FP32 inner CG, either inside FP64 iterative refinement (each round
    // adds the inner solution and takes the true residual), or as the
    // variable preconditioner of an FP64 flexible CG (Section 3 names CG with
    // variable preconditioning): each outer iteration applies A to the inner
    // solution z, makes the direction A-orthogonal to the previous one
    // (truncation to one) and updates x and r by the recurrence; the true
    // residual confirms convergence and restarts the recurrence if it
    // disagrees.
    const bool flex = c->precision == SW_MIXED_FP32_FLEX;
    const int64_t ni3 = 3 * c->mesh->dev.n_interior;
    int inner_est = std::max(1, c->last_iters / 2);
    bool first = true;
    // a projected guess comes with its residual from the stored images
    bool image_res = projected(g);
    bool recursive = false;  // residual from the flexible recurrence
    int k = 0;               // flexible iterations since the last true residual
    for (;;) {
      const bool from_images = image_res;
      const bool from_rec = recursive;
      image_res = false;
      recursive = false;
      if (from_images || from_rec) {
        rc = read_ctl(c, c->ctl64, &h);
      } else {
        rc = true_residual(c, &h, true);
        k = 0;
      }
      if (rc) return rc;
      ++*outer;
      if (first && (g == GUESS_NET || projected(g)) && !(h.rr_true <= h.bb)) {
        // reject a learned or projected guess whose residual exceeds that of
        // the zero guess
        *flags |= SW_FLAG_GUESS_FALLBACK;
        g = GUESS_EXTRAP;
        rc = set_guess(c, g);
        if (rc) return rc;
        continue;
      }
      first = false;
      if (!(h.rr_true == h.rr_true)) {
        *flags |= SW_FLAG_NONFINITE;
        break;
      }
      if (h.rr_true <= c->rtol * c->rtol * h.bb) {
        if (from_images || from_rec) continue;  // confirm with an operator pass
        break;
      }
      if (*iters >= c->max_iter) {
        *flags |= SW_FLAG_NOCONV;
        break;
      }
      // inner tolerance: the fixed inner_rtol, or less work when the target
      // needs only a smaller reduction of the current residual
      const double need = c->rtol * std::sqrt(h.bb / h.rr_true);
      const double tol = std::min(0.5, std::max(c->inner_rtol, 0.9 * need));
      launch_fill_f64(sizeof(CgCtl) / 8, (double*)c->ctl32, 0.0, s);
      launch_fill_f64(1, &c->ctl32->bb, 1.0, s);
      launch_ctl_prepare(c->ctl32, tol, s);
      launch_ir_begin(nn, c->r, c->pinv16, c->r32, c->z32, c->p32, c->p16, c->d32, c->ctl64, c->ctl32, s);
      LAUNCHED();
      int it = 0;
      rc = cg_loop<true>(c, c->ctl32, *iters, inner_est - 1, &it);
      if (rc) return rc;
      *iters += it;
      inner_est = std::max(1, it);
      if (!flex) {
        launch_ir_update(nd, c->x, c->d32, c->ctl64, s);
        LAUNCHED();
        continue;
      }
      const int par = k & 1;
      const bool prev = k > 0;
      launch_fill_f64(2, c->fdots, 0.0, s);
      launch_fill_f64(1, c->fdots + 2 + par, 0.0, s);
      launch_fcg_begin(nd, c->d32, c->ctl64, prev ? c->fq[par ^ 1] : nullptr, c->z, c->fdots, s);
      // w = A z into q (its shared nodes are clear between passes)
      rc = apply_f64(c, SW_OP_A, c->z, c->q, nullptr, -1);
      if (rc) return rc;
      launch_fcg_dir(nd, c->z, c->q, c->r, prev ? c->fp[par ^ 1] : nullptr, prev ? c->fq[par ^ 1] : nullptr,
                     c->fp[par], c->fq[par], c->fdots, par, s);
      launch_fill_f64(1, &c->ctl64->rr_true, 0.0, s);
      launch_fcg_update(nd, c->x, c->r, c->fp[par], c->fq[par], c->fdots, par, c->ctl64, s);
      launch_fill_f64(nd - ni3, c->q + ni3, 0.0, s);
      LAUNCHED();
      ++k;
      recursive = true;
    }
  }
  *relres = h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
  c->last_bb = h.bb;
  return SW_OK;
}

}  // namespace

extern "C" int sw_case_step(sw_case* c, int32_t n) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (n < 0) return fail(SW_EINVAL, "negative step count");
  if (c->step + n > c->n_steps)
    return fail(SW_ESTATE, "stepping to %lld exceeds the case capacity of %lld steps", (long long)(c->step + n),
                (long long)c->n_steps);
  if (needs_mlp(c)) return fail(SW_ESTATE, "SW_GUESS_MLP and SW_GUESS_PROJ_MLP need sw_case_attach_mlp first");
  HIPC(hipSetDevice(c->ctx->device));
  hipStream_t s = c->ctx->stream;
  const int64_t nd = 3 * c->mesh->n_nodes;
  // the steps follow each other on the stream without a host
  // synchronisation between them (the solves synchronise where they read
  // their control blocks); the call returns once the last step is done
  for (int k = 0; k < n; ++k) {
    int iters, outer, flags;
    double rel;
    int rc = solve_step(c, &iters, &outer, &rel, &flags);
    if (rc) return rc;
    if (c->samp && c->hist_count >= 4 && c->nb_count >= 4) {
      launch_mlp_collect(mlp_features(c), c->x, c->samp_per_step, c->samp_seed, c->step, c->samp_rows, c->samp_cap,
                         c->samp, s);
      c->samp_rows += c->samp_per_step;
    }
    const bool rec_proj = c->proj_dim > 0 && c->last_bb > 0.0 && !(flags & SW_FLAG_NONFINITE);
    if (rec_proj && (rc = proj_record(c))) return rc;
    const int head = (c->hist_head + 1) & 3;
    launch_newmark(nd, c->dt, c->x, c->u, c->v, c->a, c->hist + head * nd, s);
    launch_record(c->n_rec, c->rec, c->v, c->wave + c->step * 3 * c->n_rec, s);
    LAUNCHED();
    c->hist_head = head;
    c->hist_count = std::min(c->hist_count + 1, 4);
    if (c->nbh && (learned(c) || c->samp)) {
      const int nh = (c->nb_head + 1) & 3;
      launch_fill_f32(nd, c->nbh + nh * nd, 0.0f, s);
      launch_neighbour_mean(c->mesh->dev, c->hist + head * nd, c->nbh + nh * nd, s);
      LAUNCHED();
      c->nb_head = nh;
      c->nb_count = std::min(c->nb_count + 1, 4);
    }
    launch_log_step(c->log_it + c->step, iters, c->log_rel + c->step, rel, s);
    LAUNCHED();
    c->step += 1;
    c->last_iters = std::max(2, iters);
    c->stats.steps += 1;
    c->stats.cg_iters += iters;
    c->stats.ir_outer += outer;
    c->stats.max_true_rel_res = std::max(c->stats.max_true_rel_res, rel);
    c->stats.flags |= flags;
  }
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_stats_get(const sw_case* c, sw_case_stats* out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  *out = c->stats;
  return SW_OK;
}

extern "C" int sw_case_step_log(const sw_case* c, int64_t step0, int64_t n, int32_t* iters, double* rel) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (step0 < 0 || n < 0 || step0 + n > c->step) return fail(SW_EINVAL, "log range outside the completed steps");
  if (n == 0) return SW_OK;
  HIPC(hipSetDevice(c->ctx->device));
  hipStream_t s = c->ctx->stream;
  if (iters) HIPC(hipMemcpyAsync(iters, c->log_it + step0, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
  if (rel) HIPC(hipMemcpyAsync(rel, c->log_rel + step0, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_waveforms(const sw_case* c, int64_t step0, int64_t n, double* out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  if (step0 < 0 || n < 0 || step0 + n > c->n_steps) return fail(SW_EINVAL, "waveform range out of bounds");
  if (n == 0 || c->n_rec == 0) return SW_OK;
  HIPC(hipSetDevice(c->ctx->device));
  HIPC(hipMemcpyAsync(out, c->wave + step0 * 3 * c->n_rec, 8 * 3 * (size_t)c->n_rec * n, hipMemcpyDeviceToHost,
                      c->ctx->stream));
  HIPC(hipStreamSynchronize(c->ctx->stream));
  return SW_OK;
}

extern "C" int sw_case_waveform_device(const sw_case* c, const double** out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  *out = c->wave;
  return SW_OK;
}

// The user-order entry points below borrow the case's CG work vectors
// (p, q, r, z), which hold no state between steps.
extern "C" int sw_case_apply(sw_case* c, int32_t op, const double* x, double* y) {
  if (!c || !x || !y) return fail(SW_EINVAL, "NULL argument");
  if (!(op == SW_OP_A || (op > 0 && op < 8))) return fail(SW_EINVAL, "bad operator mask %d", op);
  HIPC(hipSetDevice(c->ctx->device));
  const int64_t nn = c->mesh->n_nodes;
  hipStream_t s = c->ctx->stream;
  launch_permute_f64(nn, 3, x, c->mesh->dev.node_i2u, c->p, s);
  launch_fill_f64(3 * nn, c->q, 0.0, s);
  int rc = apply_f64(c, op, c->p, c->q, nullptr, -1);
  if (rc) return rc;
  launch_permute_f64(nn, 3, c->q, c->mesh->dev.node_u2i, y, s);
  launch_fill_f64(3 * nn, c->q, 0.0, s);
  LAUNCHED();
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_apply_f32(sw_case* c, int32_t op, const float* x, float* y) {
  if (!c || !x || !y) return fail(SW_EINVAL, "NULL argument");
  if (!(op == SW_OP_A || (op > 0 && op < 8))) return fail(SW_EINVAL, "bad operator mask %d", op);
  HIPC(hipSetDevice(c->ctx->device));
  const int64_t nn = c->mesh->n_nodes;
  hipStream_t s = c->ctx->stream;
  float* xi = (float*)c->r;  // FP64 vectors hold twice the floats needed
  float* yi = (float*)c->z;
  launch_permute_f32(nn, 3, x, c->mesh->dev.node_i2u, xi, s);
  launch_fill_f32(3 * nn, yi, 0.0f, s);
  int rc;
  if (op == SW_OP_A) {
    // as in an inner CG iteration (past the first): a fresh control block,
    // so the pass runs in full (the case's inner control block is free
    // between steps)
    launch_fill_f64(sizeof(CgCtl) / 8, (double*)c->ctl32, 0.0, s);
    rc = apply_f32(c, op, xi, yi, c->ctl32, 1);
  } else {
    rc = apply_f32(c, op, xi, yi, nullptr, -1);
  }
  if (rc) return rc;
  launch_permute_f32(nn, 3, yi, c->mesh->dev.node_u2i, y, s);
  LAUNCHED();
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_rhs(sw_case* c, double* y) {
  if (!c || !y) return fail(SW_EINVAL, "NULL argument");
  if (c->step >= c->n_steps) return fail(SW_ESTATE, "no further step in the case capacity");
  HIPC(hipSetDevice(c->ctx->device));
  int rc = build_rhs(c, c->r);
  if (rc) return rc;
  launch_permute_f64(c->mesh->n_nodes, 3, c->r, c->mesh->dev.node_u2i, y, c->ctx->stream);
  LAUNCHED();
  HIPC(hipStreamSynchronize(c->ctx->stream));
  return SW_OK;
}

extern "C" int sw_case_guess(sw_case* c, double* y) {
  if (!c || !y) return fail(SW_EINVAL, "NULL argument");
  if (c->step >= c->n_steps) return fail(SW_ESTATE, "no further step in the case capacity");
  if (needs_mlp(c)) return fail(SW_ESTATE, "SW_GUESS_MLP and SW_GUESS_PROJ_MLP need sw_case_attach_mlp first");
  HIPC(hipSetDevice(c->ctx->device));
  hipStream_t s = c->ctx->stream;
  const int64_t nd = 3 * c->mesh->n_nodes;
  int rc = build_rhs(c, c->b);
  if (rc) return rc;
  launch_fill_f64(1, &c->ctl64->bb, 0.0, s);
  launch_norm2(nd, c->b, &c->ctl64->bb, s, c->det);
  rc = set_guess(c, guess_kind(c));
  if (rc) return rc;
  launch_permute_f64(c->mesh->n_nodes, 3, c->x, c->mesh->dev.node_u2i, y, s);
  LAUNCHED();
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_diag_blocks(sw_case* c, double* y) {
  if (!c || !y) return fail(SW_EINVAL, "NULL argument");
  HIPC(hipSetDevice(c->ctx->device));
  launch_permute_f64(c->mesh->n_nodes, 6, c->diag6, c->mesh->dev.node_u2i, y, c->ctx->stream);
  LAUNCHED();
  HIPC(hipStreamSynchronize(c->ctx->stream));
  return SW_OK;
}

// ------------------------------------------------------------ misfit

extern "C" int sw_misfit_workspace_bytes(int32_t n_rec, size_t* bytes) {
  if (!bytes || n_rec <= 0) return fail(SW_EINVAL, "bad arguments");
  *bytes = 8 * (2 * 3 * (size_t)n_rec + 2);
  return SW_OK;
}

static int misfit_run(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* U, const double* obs, double* buf,
                      double* err, int32_t* n_pairs) {
  launch_misfit(n_rec, n_steps, U, obs, buf, buf + 2 * 3 * n_rec, ctx->stream);
  LAUNCHED();
  double h[2];
  HIPC(hipMemcpyAsync(h, buf + 2 * 3 * n_rec, 16, hipMemcpyDeviceToHost, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  *err = h[0];
  if (n_pairs) *n_pairs = (int32_t)h[1];
  return SW_OK;
}

extern "C" int sw_misfit(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* U, const double* obs,
                         void* dev_ws, size_t ws_bytes, double* err, int32_t* n_pairs) {
  if (!ctx || !U || !obs || !err) return fail(SW_EINVAL, "NULL argument");
  if (n_rec <= 0 || n_steps <= 0) return fail(SW_EINVAL, "n_rec and n_steps must be > 0");
  if ((int64_t)n_rec * 3 > (1 << 30)) return fail(SW_EINVAL, "too many receivers");
  size_t need = 0;
  sw_misfit_workspace_bytes(n_rec, &need);
  if (!dev_ws || ((uintptr_t)dev_ws & 7) || ws_bytes < need)
    return fail(SW_ENOWS, "misfit workspace NULL, misaligned or smaller than %zu bytes", need);
  HIPC(hipSetDevice(ctx->device));
  return misfit_run(ctx, n_rec, n_steps, U, obs, (double*)dev_ws, err, n_pairs);
}

extern "C" int sw_case_misfit(sw_case* c, const double* obs, double* err, int32_t* n_pairs) {
  if (!c || !obs || !err) return fail(SW_EINVAL, "NULL argument");
  if (c->n_rec <= 0 || c->step <= 0) return fail(SW_ESTATE, "no recorded waveforms");
  HIPC(hipSetDevice(c->ctx->device));
  return misfit_run(c->ctx, c->n_rec, c->step, c->wave, obs, c->mis_buf, err, n_pairs);
}

// ------------------------------------------- misfit without a workspace
//
// For callers that cannot allocate device memory: the pair sums and the two
// results live in a file-scope device array, one copy per GPU, whose device
// address is looked up once per device when the first context on it is
// created.  Host code uses only that looked-up address: the array's name is
// a host-side stand-in, not a device pointer.  Every call on a GPU reuses
// that GPU's array, so calls on one GPU that overlap in time (two streams or
// two threads) race.  The kernels overwrite every value they later read, so
// nothing has to be cleared between calls.

static constexpr int kStaticScratchDoubles = 2 * 3 * SW_MISFIT_NOALLOC_MAX_REC + 2;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

static int static_scratch_init(int device) {
  if (device >= kMaxDevices) return fail(SW_EINVAL, "device %d beyond the %d supported", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return SW_OK;
  void* ptr = nullptr;
  HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));  // the calling thread has `device` current
  if (!ptr) return fail(SW_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
  g_scratch_dev[device] = (double*)ptr;
  return SW_OK;
}

extern "C" int sw_misfit_noalloc(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* U, const double* obs,
                                 double* err, int32_t* n_pairs) {
  if (!ctx || !U || !obs || !err) return fail(SW_EINVAL, "NULL argument");
  if (n_rec <= 0 || n_steps <= 0) return fail(SW_EINVAL, "n_rec and n_steps must be > 0");
  if (n_rec > SW_MISFIT_NOALLOC_MAX_REC)
    return fail(SW_EINVAL, "n_rec %d exceeds the static scratch limit of %d receivers (use sw_misfit)", n_rec,
                (int)SW_MISFIT_NOALLOC_MAX_REC);
  double* buf = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    buf = g_scratch_dev[ctx->device];
  }
  if (!buf) return fail(SW_ESTATE, "static scratch of device %d not set up", ctx->device);
  HIPC(hipSetDevice(ctx->device));
  return misfit_run(ctx, n_rec, n_steps, U, obs, buf, err, n_pairs);
}

// ------------------------------------------------------------ network

// ------------------------------------------------------- input estimation

namespace {

struct FitWs {
  double *o2, *w, *C, *c, *U, *mis, *out2;
};

constexpr int FIT_MAX_SHIFT = 128;

size_t fit_layout(int32_t n_rec, int64_t n_steps, int32_t stride, Carver& cv, FitWs* f) {
  const int np = 3 * n_rec;
  const int64_t nb = n_steps / stride;
  FitWs t{};
  t.o2 = cv.take<double>(np);
  t.w = cv.take<double>(np);
  t.C = cv.take<double>((size_t)(4 * nb) * (4 * nb));
  t.c = cv.take<double>(3 * FIT_MAX_SHIFT);
  t.U = cv.take<double>((size_t)n_steps * np);
  t.mis = cv.take<double>(2 * np + 2);
  t.out2 = cv.take<double>(2);
  if (f) *f = t;
  return cv.off + 256;
}

int fit_check(int32_t n_rec, int64_t n_steps, int32_t stride, int32_t n_shift) {
  if (n_rec < 1 || n_steps < 1) return fail(SW_EINVAL, "need receivers and steps");
  if (stride < 1 || n_steps % stride) return fail(SW_EINVAL, "n_steps must be a positive multiple of the stride");
  if (n_shift < 1 || n_shift > n_steps / stride || n_shift > FIT_MAX_SHIFT)
    return fail(SW_EINVAL, "n_shift must be in 1..min(n_steps / stride, %d)", FIT_MAX_SHIFT);
  return SW_OK;
}

}  // namespace

extern "C" int sw_fit_workspace_bytes(int32_t n_rec, int64_t n_steps, int32_t stride, int32_t n_shift,
                                      size_t* bytes) {
  if (!bytes) return fail(SW_EINVAL, "bytes is NULL");
  int rc = fit_check(n_rec, n_steps, stride, n_shift);
  if (rc) return rc;
  Carver cv(nullptr);
  *bytes = fit_layout(n_rec, n_steps, stride, cv, nullptr);
  return SW_OK;
}

static int fit_one(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green, const double* obs,
                   int32_t stride, int32_t n_shift, double rel_cut, void* ws, double* c_host, double* err,
                   int32_t* n_pairs, int32_t* rank, double* U_dev);

extern "C" int sw_fit_input(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green,
                            const double* obs, int32_t stride, int32_t n_shift, double rel_cut, void* ws,
                            size_t ws_bytes, double* c_host, double* err, int32_t* n_pairs, int32_t* rank,
                            double* U_dev) {
  if (!ctx || !green || !obs || !c_host || !err) return fail(SW_EINVAL, "NULL argument");
  for (int j = 0; j < 3; ++j)
    if (!green[j]) return fail(SW_EINVAL, "Green's record %d is NULL", j);
  int rc = fit_check(n_rec, n_steps, stride, n_shift);
  if (rc) return rc;
  if (!(rel_cut >= 0.0 && rel_cut < 1.0)) return fail(SW_EINVAL, "rel_cut must be in [0, 1)");
  {
    Carver dry(nullptr);
    const size_t need = fit_layout(n_rec, n_steps, stride, dry, nullptr);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
      return fail(SW_ENOWS, "fit workspace needs %zu bytes, 256-byte aligned", need);
  }
  HIPC(hipSetDevice(ctx->device));
  return fit_one(ctx, n_rec, n_steps, green, obs, stride, n_shift, rel_cut, ws, c_host, err, n_pairs, rank, U_dev);
}

extern "C" int sw_fit_events(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green,
                             int32_t n_events, const double* const* obs, int32_t stride, int32_t n_shift,
                             double rel_cut, void* ws, size_t ws_bytes, double* c_host, double* err,
                             int32_t* n_pairs, int32_t* rank, double* err_max, int32_t* worst) {
  if (!ctx || !green || !obs || !c_host || !err || !err_max) return fail(SW_EINVAL, "NULL argument");
  if (n_events < 1) return fail(SW_EINVAL, "n_events must be >= 1");
  for (int j = 0; j < 3; ++j)
    if (!green[j]) return fail(SW_EINVAL, "Green's record %d is NULL", j);
  for (int e = 0; e < n_events; ++e)
    if (!obs[e]) return fail(SW_EINVAL, "observed record of event %d is NULL", e);
  int rc = fit_check(n_rec, n_steps, stride, n_shift);
  if (rc) return rc;
  if (!(rel_cut >= 0.0 && rel_cut < 1.0)) return fail(SW_EINVAL, "rel_cut must be in [0, 1)");
  {
    Carver dry(nullptr);
    const size_t need = fit_layout(n_rec, n_steps, stride, dry, nullptr);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
      return fail(SW_ENOWS, "fit workspace needs %zu bytes, 256-byte aligned", need);
  }
  HIPC(hipSetDevice(ctx->device));
  // the Green's records are the model's; each event is fitted on its own
  // (the weights 1/|obs|^2 of the normal equations are the event's), and
  // the model's misfit is that of its worst event
  int w = -1;
  double mx = 0.0;
  for (int e = 0; e < n_events; ++e) {
    rc = fit_one(ctx, n_rec, n_steps, green, obs[e], stride, n_shift, rel_cut, ws, c_host + (size_t)e * 3 * n_shift,
                 err + e, n_pairs ? n_pairs + e : nullptr, rank ? rank + e : nullptr, nullptr);
    if (rc) return rc;
    if (err[e] != err[e]) {  // an event with no usable pair: the model's misfit is undefined
      w = e;
      mx = err[e];
      break;
    }
    if (w < 0 || err[e] > mx) {
      w = e;
      mx = err[e];
    }
  }
  *err_max = mx;
  if (worst) *worst = w;
  return SW_OK;
}

static int fit_one(sw_ctx* ctx, int32_t n_rec, int64_t n_steps, const double* const* green, const double* obs,
                   int32_t stride, int32_t n_shift, double rel_cut, void* ws, double* c_host, double* err,
                   int32_t* n_pairs, int32_t* rank, double* U_dev) {
  hipStream_t s = ctx->stream;
  FitWs f;
  Carver cv(ws);
  fit_layout(n_rec, n_steps, stride, cv, &f);
  const int np = 3 * n_rec, nb = (int)(n_steps / stride), L = n_shift, ncol = 4 * nb;
  launch_fit_weights(np, n_steps, obs, f.o2, f.w, s);
  launch_fit_gram(green, obs, np, stride, nb, f.w, f.C, s);
  LAUNCHED();
  std::vector<double> C((size_t)ncol * ncol);
  HIPC(hipMemcpyAsync(C.data(), f.C, C.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  // normal equations from block inner products (shift l delays by l blocks)
  const int n = 3 * L;
  std::vector<double> A((size_t)n * n, 0.0), bv(n, 0.0), V, w, cvec(n);
  for (int j = 0; j < 3; ++j)
    for (int l = 0; l < L; ++l) {
      double acc = 0.0;
      for (int b = l; b < nb; ++b) acc += C[(size_t)(j * nb + b - l) * ncol + 3 * nb + b];
      bv[j * L + l] = acc;
      for (int j2 = 0; j2 < 3; ++j2)
        for (int l2 = 0; l2 < L; ++l2) {
          double a = 0.0;
          for (int b = std::max(l, l2); b < nb; ++b) a += C[(size_t)(j * nb + b - l) * ncol + j2 * nb + b - l2];
          A[(size_t)(j * L + l) * n + j2 * L + l2] = a;
        }
    }
  sym_eig(n, A, V, w);
  const int kept = truncated_solve(n, V, w, bv.data(), cvec.data(), rel_cut);
  for (int i = 0; i < n; ++i) c_host[i] = cvec[i];
  if (rank) *rank = kept;
  // response to the fitted input and its misfit
  double* U = U_dev ? U_dev : f.U;
  HIPC(hipMemcpyAsync(f.c, cvec.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  launch_fit_response(green, np, stride, L, n_steps, f.c, U, s);
  launch_misfit(n_rec, n_steps, U, obs, f.mis, f.out2, s);
  LAUNCHED();
  double out2[2];
  HIPC(hipMemcpyAsync(out2, f.out2, sizeof out2, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  *err = out2[0];
  if (n_pairs) *n_pairs = (int32_t)out2[1];
  return SW_OK;
}

static size_t mlp_layout(Carver& cv, sw_mlp* o) {
  auto th = cv.take<float>(MLP_NP);
  auto m = cv.take<float>(MLP_NP);
  auto v = cv.take<float>(MLP_NP);
  auto g = cv.take<double>(MLP_NP);
  auto l2 = cv.take<double>(4);
  if (o) {
    o->theta = th;
    o->m = m;
    o->v = v;
    o->grad = g;
    o->loss2 = l2;
  }
  return cv.off;
}

extern "C" int sw_mlp_init_params(uint64_t seed, float* params) {
  if (!params) return fail(SW_EINVAL, "params is NULL");
  uint64_t state = seed;
  auto next = [&state]() {  // splitmix64
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto uniform = [&next](double a) { return (float)(a * (2.0 * (double)(next() >> 11) * 0x1.0p-53 - 1.0)); };
  const double a1 = std::sqrt(6.0 / (MLP_IN + MLP_H)), a2 = std::sqrt(6.0 / (MLP_H + MLP_H));
  for (int i = 0; i < MLP_NP; ++i) params[i] = 0.0f;
  for (int i = 0; i < MLP_H * MLP_IN; ++i) params[MLP_OFF_W1 + i] = uniform(a1);
  for (int i = 0; i < MLP_H * MLP_H; ++i) params[MLP_OFF_W2 + i] = uniform(a2);
  return SW_OK;
}

extern "C" int sw_mlp_workspace_bytes(size_t* bytes) {
  if (!bytes) return fail(SW_EINVAL, "NULL argument");
  Carver cv(nullptr);
  *bytes = mlp_layout(cv, nullptr);
  return SW_OK;
}

extern "C" int sw_mlp_create(sw_ctx* ctx, const float* params, void* ws, size_t ws_bytes, sw_mlp** out) {
  if (!ctx || !params || !out) return fail(SW_EINVAL, "NULL argument");
  Carver dry(nullptr);
  const size_t need = mlp_layout(dry, nullptr);
  if (!ws || ((uintptr_t)ws & 255)) return fail(SW_ENOWS, "network workspace NULL or not 256-byte aligned");
  if (ws_bytes < need) return fail(SW_ENOWS, "network workspace %zu bytes < %zu needed", ws_bytes, need);
  HIPC(hipSetDevice(ctx->device));
  sw_mlp* o = new sw_mlp();
  o->ctx = ctx;
  Carver cv(ws);
  mlp_layout(cv, o);
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemcpyAsync(o->theta, params, 4 * (size_t)MLP_NP, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    delete o;
    return fail(SW_EHIP, "parameter upload failed: %s", hipGetErrorString(e));
  }
  launch_fill_f32(MLP_NP, o->m, 0.0f, s);
  launch_fill_f32(MLP_NP, o->v, 0.0f, s);
  launch_fill_f64(MLP_NP, o->grad, 0.0, s);
  launch_fill_f64(4, o->loss2, 0.0, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete o;
    return fail(SW_EHIP, "network set-up failed: %s", hipGetErrorString(e));
  }
  *out = o;
  return SW_OK;
}

extern "C" int sw_mlp_destroy(sw_mlp* o) {
  delete o;
  return SW_OK;
}

extern "C" int sw_mlp_get_params(sw_mlp* o, float* out) {
  if (!o || !out) return fail(SW_EINVAL, "NULL argument");
  HIPC(hipSetDevice(o->ctx->device));
  HIPC(hipMemcpyAsync(out, o->theta, 4 * (size_t)MLP_NP, hipMemcpyDeviceToHost, o->ctx->stream));
  HIPC(hipStreamSynchronize(o->ctx->stream));
  return SW_OK;
}

extern "C" int sw_mlp_forward(sw_mlp* o, const float* X, float* y, int64_t n) {
  if (!o || (n > 0 && (!X || !y)) || n < 0) return fail(SW_EINVAL, "bad arguments");
  HIPC(hipSetDevice(o->ctx->device));
  launch_mlp_forward(n, X, o->theta, y, o->ctx->stream);
  LAUNCHED();
  HIPC(hipStreamSynchronize(o->ctx->stream));
  return SW_OK;
}

extern "C" int sw_mlp_gradient(sw_mlp* o, const float* S, int64_t n, double* grad, double* loss) {
  if (!o || !S || n <= 0 || !grad) return fail(SW_EINVAL, "bad arguments");
  HIPC(hipSetDevice(o->ctx->device));
  hipStream_t s = o->ctx->stream;
  launch_fill_f64(MLP_NP, o->grad, 0.0, s);
  launch_fill_f64(4, o->loss2, 0.0, s);
  launch_mlp_grad(S, n, 0, 0, 0, o->theta, o->grad, o->loss2, s);
  LAUNCHED();
  double l2[2];
  HIPC(hipMemcpyAsync(grad, o->grad, 8 * (size_t)MLP_NP, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(l2, o->loss2, 16, hipMemcpyDeviceToHost, s));
  launch_fill_f64(MLP_NP, o->grad, 0.0, s);
  HIPC(hipStreamSynchronize(s));
  if (l2[1] > 0.0)
    for (int j = 0; j < MLP_NP; ++j) grad[j] /= l2[1];
  if (loss) *loss = l2[1] > 0.0 ? l2[0] / l2[1] : 0.0;
  return SW_OK;
}

extern "C" int sw_mlp_train(sw_mlp* o, const float* S, int64_t n, int32_t steps, int32_t batch, float lr,
                            uint64_t seed, float* loss) {
  if (!o || !S || n <= 0 || steps < 0 || batch <= 0 || !(lr > 0.0f)) return fail(SW_EINVAL, "bad arguments");
  HIPC(hipSetDevice(o->ctx->device));
  hipStream_t s = o->ctx->stream;
  for (int k = 0; k < steps; ++k) {
    launch_fill_f64(4, o->loss2, 0.0, s);
    launch_mlp_grad(S, n, batch, seed, o->adam_step, o->theta, o->grad, o->loss2, s);
    o->adam_step += 1;
    launch_mlp_adam(o->theta, o->m, o->v, o->grad, o->loss2, o->adam_step, lr, s);
    LAUNCHED();
    if (loss) {
      double l2[2];
      HIPC(hipMemcpyAsync(l2, o->loss2, 16, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      loss[k] = l2[1] > 0.0 ? (float)(l2[0] / l2[1]) : 0.0f;
    }
  }
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_case_attach_mlp(sw_case* c, sw_mlp* o) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (o && o->ctx->device != c->ctx->device) return fail(SW_EINVAL, "network on another device");
  if (o && !c->nbh) return fail(SW_ESTATE, "the case was created with the zero guess (no feature buffers)");
  c->mlp = o;
  return SW_OK;
}

extern "C" int sw_case_set_sampler(sw_case* c, float* buf, int64_t capacity, int32_t per_step, uint64_t seed) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (buf && (capacity <= 0 || per_step <= 0 || per_step > capacity)) return fail(SW_EINVAL, "bad sampler sizes");
  if (buf && !c->nbh) return fail(SW_ESTATE, "the case was created with the zero guess (no feature buffers)");
  if (buf && c->nb_count < 4 && c->step > 0 && !learned(c))
    c->nb_count = 0;  // neighbour means start accumulating now
  c->samp = buf;
  c->samp_cap = capacity;
  c->samp_per_step = per_step;
  c->samp_seed = seed;
  c->samp_rows = 0;
  return SW_OK;
}

extern "C" int sw_case_samples(const sw_case* c, int64_t* rows) {
  if (!c || !rows) return fail(SW_EINVAL, "NULL argument");
  *rows = std::min(c->samp_rows, c->samp_cap);
  return SW_OK;
}

// ------------------------------------------------------------ batch

namespace {

// Work items of the batched operator pass: (lane, tile) pairs.  Lanes that
// share a mesh form a group; within a group the lanes of tile t get work
// items whose index is congruent to t modulo 8 and adjacent in dispatch
// order, so that (with workgroups handed to the 8 XCDs round-robin) one XCD
// runs every lane of a tile at about the same time and reads the tile's mesh
// data once into its L2.  Each group's range is padded to a multiple of 8.
std::vector<int2> batch_work(sw_case* const* cases, int n) {
  std::vector<int2> work;
  std::vector<const sw_mesh*> meshes;
  for (int l = 0; l < n; ++l)
    if (std::find(meshes.begin(), meshes.end(), cases[l]->mesh) == meshes.end()) meshes.push_back(cases[l]->mesh);
  for (const sw_mesh* m : meshes) {
    std::vector<int> lanes;
    for (int l = 0; l < n; ++l)
      if (cases[l]->mesh == m) lanes.push_back(l);
    const int nt = m->dev.n_tiles, K = (int)lanes.size();
    for (int r = 0; r < (nt + 7) / 8; ++r)
      for (int li = 0; li < K; ++li)
        for (int x = 0; x < 8; ++x) {
          const int t = 8 * r + x;
          work.push_back(t < nt ? make_int2(lanes[li], t) : make_int2(-1, -1));
        }
  }
  return work;
}

// Items of the persistent FP32 pass, tile by tile with the lanes of one
// mesh adjacent (they share the tile's mesh data).  schedule 0: one mesh
// after the other; 1: the meshes interleaved tile by tile (tile t of every
// mesh, then tile t + 1), which spreads each mesh over all XCDs.
std::vector<int2> batch_items(sw_case* const* cases, int n, int schedule = 0) {
  std::vector<int2> items;
  std::vector<const sw_mesh*> meshes;
  for (int l = 0; l < n; ++l)
    if (std::find(meshes.begin(), meshes.end(), cases[l]->mesh) == meshes.end()) meshes.push_back(cases[l]->mesh);
  if (schedule == 0) {
    for (const sw_mesh* m : meshes)
      for (int t = 0; t < m->dev.n_tiles; ++t)
        for (int l = 0; l < n; ++l)
          if (cases[l]->mesh == m) items.push_back(make_int2(l, t));
  } else {
    int tmax = 0;
    for (const sw_mesh* m : meshes) tmax = std::max(tmax, (int)m->dev.n_tiles);
    for (int t = 0; t < tmax; ++t)
      for (const sw_mesh* m : meshes)
        if (t < m->dev.n_tiles)
          for (int l = 0; l < n; ++l)
            if (cases[l]->mesh == m) items.push_back(make_int2(l, t));
  }
  return items;
}

size_t batch_layout(int n, int n_work, int n_items, Carver& cv, sw_batch* b) {
  b->d_lanes = cv.take<LaneDev>(n);
  b->d_st = cv.take<LaneState>(n);
  b->d_info = cv.take<LaneInfo>(n);
  b->d_rhs1 = cv.take<TileLane<double>>(n);
  b->d_rhs2 = cv.take<TileLane<double>>(n);
  b->d_true = cv.take<TileLane<double>>(n);
  b->d_cg32 = cv.take<TileLane<float>>(n);
  b->d_work = cv.take<int2>(n_work);
  b->d_items = cv.take<int2>(n_items);
  return cv.off + 256;
}

int batch_check(sw_ctx* ctx, sw_case* const* cases, int32_t n) {
  if (!cases || n <= 0) return fail(SW_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    if (!cases[i]) return fail(SW_EINVAL, "case %d is NULL", i);
    if (ctx && cases[i]->ctx != ctx) return fail(SW_EINVAL, "case %d belongs to another context", i);
    if (cases[i]->ctx != cases[0]->ctx) return fail(SW_EINVAL, "cases of one batch must share a context");
    if (cases[i]->precision != SW_MIXED_FP32)
      return fail(SW_EINVAL, "case %d: batches march SW_MIXED_FP32 cases only", i);
    for (int j = 0; j < i; ++j)
      if (cases[j] == cases[i]) return fail(SW_EINVAL, "case %d appears twice in the batch", i);
  }
  return SW_OK;
}

template <typename T>
TileLane<T> tile_lane(const sw_case* c) {
  TileLane<T> t{};
  t.m = c->mesh->dev;
  t.emat = c->emat;
  t.mats = c->mats;
  return t;
}

int batch_upload(sw_batch* b, void* dst, const void* src, size_t bytes) {
  HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->ctx->stream));
  return SW_OK;
}

int batch_gather(sw_batch* b) {
  hipStream_t s = b->ctx->stream;
  launch_lanes(LANE_GATHER, b->n, b->max_nodes, b->d_lanes, nullptr, b->d_info, s);
  LAUNCHED();
  HIPC(hipMemcpyAsync(b->info.data(), b->d_info, b->n * sizeof(LaneInfo), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  return b->ctx->prof.on ? prof_flush(b->ctx) : SW_OK;
}

// One FP32 CG iteration of every refining lane on stream s (dev_index: the
// direction kernels take the iteration index from the lanes' control
// blocks, as in a captured pair).
void batch_cg_iteration(sw_batch* b, int i, bool dev_index, hipStream_t s, bool prof) {
  sw_ctx* cx = b->ctx;
  const int n = b->n;
  int ev = prof ? prof_begin(cx, SW_PROF_TILE_F32) : -1;
  launch_tile_lanes_pipe_f32(b->d_cg32, b->d_items, b->n_items, b->max_tile_nodes, b->d_st, i, batch_grid_cap(b), s);
  if (prof) prof_end(cx, ev);
  ev = prof ? prof_begin(cx, SW_PROF_UPDATE_F32) : -1;
  launch_lanes_cg(true, false, n, b->max_nodes, b->d_lanes, b->d_st, i, s, dev_index);
  if (prof) prof_end(cx, ev);
  ev = prof ? prof_begin(cx, SW_PROF_DIR_F32) : -1;
  launch_lanes_cg(true, true, n, b->max_nodes, b->d_lanes, b->d_st, i, s, dev_index);
  if (prof) prof_end(cx, ev);
}

// The batch's captured pair of FP32 CG iterations (see cg_pair_graph).
int batch_pair_graph(sw_batch* b, hipGraphExec_t* out) {
  if (b->cg_graph && b->cg_graph_cap == batch_grid_cap(b)) {
    *out = b->cg_graph;
    return SW_OK;
  }
  if (b->cg_graph) {
    HIPC(hipGraphExecDestroy(b->cg_graph));
    b->cg_graph = nullptr;
  }
  hipStream_t cs;
  int rc = capture_stream(b->ctx, &cs);
  if (rc) return rc;
  HIPC(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < 2; ++k) batch_cg_iteration(b, 2 + k, true, cs, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess) return fail(SW_EHIP, "batch CG graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return fail(SW_EHIP, "batch CG graph instantiation failed: %s", hipGetErrorString(e2));
  b->cg_graph = ex;
  b->cg_graph_cap = batch_grid_cap(b);
  *out = ex;
  return SW_OK;
}

// One time step of every lane (mixed precision: FP32 inner CG inside FP64
// refinement), the same arithmetic as solve_step + sw_case_step per case.
int batch_step_once(sw_batch* b) {
  sw_ctx* cx = b->ctx;
  hipStream_t s = cx->stream;
  const int n = b->n;
  std::vector<int> g(n), iters(n, 0), outer(n, 0), flags(n, 0), est(n), stopped(n, 0), first(n, 1);
  std::vector<double> rel(n, 0.0);
  for (int l = 0; l < n; ++l) {
    sw_case* c = b->cases[l];
    g[l] = guess_kind(c);
    LaneDev& L = b->lanes[l];
    L.step = c->step;
    L.hist_head = c->hist_head;
    L.guess_order = (g[l] == GUESS_NET || projected(g[l]))
                        ? -2
                        : (g[l] == GUESS_EXTRAP ? std::min(c->poly_order, c->hist_count - 1) : -1);
    b->rhs1[l].A.vin = c->vin + 3 * (c->step + 1);
    est[l] = std::max(1, c->last_iters / 2);
  }
  int rc = batch_upload(b, b->d_lanes, b->lanes.data(), n * sizeof(LaneDev));
  if (!rc) rc = batch_upload(b, b->d_rhs1, b->rhs1.data(), n * sizeof(TileLane<double>));
  if (rc) return rc;
  // right-hand side, its norm, tolerance, initial guess
  launch_lanes(LANE_BEGIN_STEP, n, b->max_nodes, b->d_lanes, nullptr, nullptr, s);
  launch_tile_lanes_f64(b->d_rhs1, b->d_work, b->n_work, b->max_tile_nodes, nullptr, -1, s);
  launch_tile_lanes_f64(b->d_rhs2, b->d_work, b->n_work, b->max_tile_nodes, nullptr, -1, s);
  launch_lanes(LANE_NORM2_B, n, b->max_nodes, b->d_lanes, nullptr, nullptr, s);
  launch_lanes(LANE_PREPARE64, n, b->max_nodes, b->d_lanes, nullptr, nullptr, s);
  launch_lanes(LANE_GUESS, n, b->max_nodes, b->d_lanes, nullptr, nullptr, s);
  LAUNCHED();
  bool any_proj = false;
  for (int l = 0; l < n; ++l) {
    if (g[l] == GUESS_NET && (rc = set_guess(b->cases[l], GUESS_NET))) return rc;
    if (projected(g[l])) {
      const bool extra = g[l] == GUESS_PROJ_NET;
      if (extra && (rc = proj_net_direction(b->cases[l]))) return rc;
      if ((rc = proj_begin(b->cases[l], extra))) return rc;
      any_proj = true;
    }
  }
  // a projected guess comes with its residual from the stored images
  std::vector<char> image_res(n, 0);
  if (any_proj) {
    HIPC(hipStreamSynchronize(s));
    for (int l = 0; l < n; ++l)
      if (projected(g[l])) {
        if ((rc = proj_finish(b->cases[l], true, g[l] == GUESS_PROJ_NET))) return rc;
        image_res[l] = 1;
      }
  }
  // refinement rounds
  for (;;) {
    for (int l = 0; l < n; ++l) {
      b->st[l].active = !stopped[l] && !image_res[l];
      b->st[l].zero_q = 1;
    }
    if ((rc = batch_upload(b, b->d_st, b->st.data(), n * sizeof(LaneState)))) return rc;
    launch_lanes(LANE_RRTRUE_RESET, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
    launch_tile_lanes_f64(b->d_true, b->d_work, b->n_work, b->max_tile_nodes, b->d_st, -1, s);
    launch_lanes(LANE_TRUE_RES, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
    LAUNCHED();
    if ((rc = batch_gather(b))) return rc;
    bool any_inner = false, any_open = false;
    for (int l = 0; l < n; ++l) {
      LaneState& S = b->st[l];
      if (stopped[l]) {
        S.active = 0;
        continue;
      }
      sw_case* c = b->cases[l];
      const LaneInfo& h = b->info[l];
      const bool from_images = image_res[l];
      image_res[l] = 0;
      ++outer[l];
      S.active = 0;
      if (first[l] && (g[l] == GUESS_NET || projected(g[l])) && !(h.rr_true <= h.bb)) {
        // reject a learned or projected guess whose residual exceeds that of
        // the zero guess; the lane's true residual is taken again next round
        flags[l] |= SW_FLAG_GUESS_FALLBACK;
        g[l] = GUESS_EXTRAP;
        first[l] = 0;
        if ((rc = set_guess(c, GUESS_EXTRAP))) return rc;
        any_open = true;
        continue;
      }
      first[l] = 0;
      bool stop = false;
      if (!(h.rr_true == h.rr_true)) {
        flags[l] |= SW_FLAG_NONFINITE;
        stop = true;
      } else if (h.rr_true <= c->rtol * c->rtol * h.bb) {
        if (from_images) {  // confirm with an operator pass next round
          any_open = true;
          continue;
        }
        stop = true;
      } else if (iters[l] >= c->max_iter) {
        flags[l] |= SW_FLAG_NOCONV;
        stop = true;
      }
      if (stop) {
        stopped[l] = 1;
        rel[l] = h.bb > 0.0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
        continue;
      }
      const double need = c->rtol * std::sqrt(h.bb / h.rr_true);
      S.tol = std::min(0.5, std::max(c->inner_rtol, 0.9 * need));
      S.iter_base = iters[l];
      S.active = 1;
      any_inner = any_open = true;
    }
    if (!any_open) break;
    if (!any_inner) continue;
    if ((rc = batch_upload(b, b->d_st, b->st.data(), n * sizeof(LaneState)))) return rc;
    launch_lanes(LANE_TO_F32, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
    launch_lanes(LANE_CG_INIT32, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
    LAUNCHED();
    // inner CG of every refining lane in lockstep; converged lanes' work
    // items return at once.  The first chunk has an even count; the chunks
    // of two after it replay the batch's captured pair of iterations.
    int chunk = 2;
    for (int l = 0; l < n; ++l)
      if (b->st[l].active) chunk = std::max(chunk, est[l] + (est[l] & 1));
    for (int it = 0;;) {
      hipGraphExec_t g = nullptr;
      if (it > 0 && chunk == 2 && cx->graphs && !cx->prof.on && (rc = batch_pair_graph(b, &g))) return rc;
      if (g) {
        HIPC(hipGraphLaunch(g, s));
      } else {
        for (int k = 0; k < chunk; ++k) batch_cg_iteration(b, it + k, false, s, true);
      }
      LAUNCHED();
      it += chunk;
      if ((rc = batch_gather(b))) return rc;
      bool all = true;
      for (int l = 0; l < n; ++l)
        if (b->st[l].active && !b->info[l].done32) all = false;
      if (all) break;
      chunk = 2;
    }
    for (int l = 0; l < n; ++l) {
      if (!b->st[l].active) continue;
      const int itl = std::max(0, b->info[l].iters32 - b->st[l].iter_base);
      iters[l] += itl;
      est[l] = std::max(1, itl);
    }
    launch_lanes(LANE_IR_UPDATE, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
    LAUNCHED();
  }
  // training samples, projection ring, Newmark update, receivers, logs
  for (int l = 0; l < n; ++l) {
    sw_case* c = b->cases[l];
    if (c->samp && c->hist_count >= 4 && c->nb_count >= 4) {
      launch_mlp_collect(mlp_features(c), c->x, c->samp_per_step, c->samp_seed, c->step, c->samp_rows, c->samp_cap,
                         c->samp, s);
      c->samp_rows += c->samp_per_step;
    }
    c->last_bb = b->info[l].bb;
    const bool rec_proj = c->proj_dim > 0 && c->last_bb > 0.0 && !(flags[l] & SW_FLAG_NONFINITE);
    if (rec_proj && (rc = proj_record(c))) return rc;
    b->st[l].active = 1;
    b->st[l].iters = iters[l];
    b->st[l].rel = rel[l];
  }
  if ((rc = batch_upload(b, b->d_st, b->st.data(), n * sizeof(LaneState)))) return rc;
  launch_lanes(LANE_NEWMARK, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
  launch_lanes(LANE_RECORD, n, b->max_nodes, b->d_lanes, b->d_st, nullptr, s);
  LAUNCHED();
  for (int l = 0; l < n; ++l) {
    sw_case* c = b->cases[l];
    const int64_t nd = 3 * c->mesh->n_nodes;
    const int head = (c->hist_head + 1) & 3;
    c->hist_head = head;
    c->hist_count = std::min(c->hist_count + 1, 4);
    if (c->nbh && (learned(c) || c->samp)) {
      const int nh = (c->nb_head + 1) & 3;
      launch_fill_f32(nd, c->nbh + nh * nd, 0.0f, s);
      launch_neighbour_mean(c->mesh->dev, c->hist + head * nd, c->nbh + nh * nd, s);
      LAUNCHED();
      c->nb_head = nh;
      c->nb_count = std::min(c->nb_count + 1, 4);
    }
  }
  HIPC(hipStreamSynchronize(s));
  for (int l = 0; l < n; ++l) {
    sw_case* c = b->cases[l];
    c->step += 1;
    c->last_iters = std::max(2, iters[l]);
    c->stats.steps += 1;
    c->stats.cg_iters += iters[l];
    c->stats.ir_outer += outer[l];
    c->stats.max_true_rel_res = std::max(c->stats.max_true_rel_res, rel[l]);
    c->stats.flags |= flags[l];
  }
  return SW_OK;
}

}  // namespace

extern "C" int sw_batch_workspace_bytes(sw_case* const* cases, int32_t n, size_t* bytes) {
  if (!bytes) return fail(SW_EINVAL, "bytes is NULL");
  int rc = batch_check(nullptr, cases, n);
  if (rc) return rc;
  const std::vector<int2> work = batch_work(cases, n);
  const std::vector<int2> items = batch_items(cases, n);
  sw_batch tmp;
  Carver cv(nullptr);
  *bytes = batch_layout(n, (int)work.size(), (int)items.size(), cv, &tmp);
  return SW_OK;
}

extern "C" int sw_batch_create(sw_ctx* ctx, sw_case* const* cases, int32_t n, void* ws, size_t ws_bytes,
                               sw_batch** out) {
  if (!ctx || !out) return fail(SW_EINVAL, "bad batch arguments");
  int rc = batch_check(ctx, cases, n);
  if (rc) return rc;
  const std::vector<int2> work = batch_work(cases, n);
  const std::vector<int2> items = batch_items(cases, n);
  size_t need = 0;
  {
    sw_batch tmp;
    Carver cv(nullptr);
    need = batch_layout(n, (int)work.size(), (int)items.size(), cv, &tmp);
  }
  if (!ws || ws_bytes < need) return fail(SW_ENOWS, "batch workspace needs %zu bytes, got %zu", need, ws_bytes);
  HIPC(hipSetDevice(ctx->device));
  sw_batch* b = new sw_batch();
  b->ctx = ctx;
  b->cases.assign(cases, cases + n);
  b->n = n;
  b->n_work = (int)work.size();
  b->n_items = (int)items.size();
  Carver cv(ws);
  batch_layout(n, b->n_work, b->n_items, cv, b);
  b->lanes.resize(n);
  b->st.assign(n, LaneState{});
  b->info.resize(n);
  b->rhs1.resize(n);
  std::vector<TileLane<double>> rhs2(n), tru(n);
  std::vector<TileLane<float>> cg32(n);
  for (int l = 0; l < n; ++l) {
    sw_case* c = cases[l];
    b->max_nodes = std::max(b->max_nodes, c->mesh->n_nodes);
    b->max_tile_nodes = std::max(b->max_tile_nodes, c->mesh->dev.max_tile_nodes);
    LaneDev& L = b->lanes[l];
    L = LaneDev{};
    L.n_nodes = c->mesh->n_nodes;
    L.dt = c->dt;
    L.u = c->u;
    L.v = c->v;
    L.a = c->a;
    L.b = c->b;
    L.x = c->x;
    L.r = c->r;
    L.z = c->z;
    L.p = c->p;
    L.q = c->q;
    L.hist = c->hist;
    L.pinv64 = c->pinv64;
    L.pinv16 = c->pinv16;
    L.n_interior = c->mesh->dev.n_interior;
    L.r32 = c->r32;
    L.d32 = c->d32;
    L.z32 = c->z32;
    L.p32 = c->p32;
    L.q32 = c->q32;
    L.ctl64 = c->ctl64;
    L.ctl32 = c->ctl32;
    L.rec = c->rec;
    L.wave = c->wave;
    L.log_it = c->log_it;
    L.log_rel = c->log_rel;
    L.rtol = c->rtol;
    L.n_rec = c->n_rec;
    L.max_iter = c->max_iter;
    // right-hand side: M (a + (4/dt + alpha) v) + C_abs v + F, then -K (u - beta v)
    TileLane<double>& r1 = b->rhs1[l];
    r1 = tile_lane<double>(c);
    r1.A.sM = 1.0;
    r1.A.sC = 1.0;
    r1.A.x1 = c->a;
    r1.A.a1 = 1.0;
    r1.A.x2 = c->v;
    r1.A.a2 = 4.0 / c->dt + c->alpha;
    r1.A.xf = c->v;
    r1.A.y = c->b;
    TileLane<double>& r2 = rhs2[l];
    r2 = tile_lane<double>(c);
    r2.A.sK = -1.0;
    r2.A.x1 = c->u;
    r2.A.a1 = 1.0;
    r2.A.x2 = c->v;
    r2.A.a2 = -c->beta;
    r2.A.y = c->b;
    r2.A.accumulate = 1;
    // q = A x (FP64) and q32 = A p32 (FP32 CG iterations)
    TileLane<double>& t = tru[l];
    t = tile_lane<double>(c);
    t.A.sM = c->cM;
    t.A.sK = c->cK;
    t.A.sC = c->cC;
    t.A.x1 = c->x;
    t.A.a1 = 1.0;
    t.A.xf = c->x;
    t.A.y = c->q;
    TileLane<float>& f = cg32[l];
    f = tile_lane<float>(c);
    f.A.sM = (float)c->cM;
    f.A.sK = (float)c->cK;
    f.A.sC = (float)c->cC;
    f.A.x1 = c->p32;
    f.A.a1 = 1.0f;
    f.A.xf = c->p32;
    f.A.y = c->q32;
    f.ctl = c->ctl32;
  }
  rc = batch_upload(b, b->d_rhs2, rhs2.data(), n * sizeof(TileLane<double>));
  if (!rc) rc = batch_upload(b, b->d_true, tru.data(), n * sizeof(TileLane<double>));
  if (!rc) rc = batch_upload(b, b->d_cg32, cg32.data(), n * sizeof(TileLane<float>));
  if (!rc) rc = batch_upload(b, b->d_work, work.data(), work.size() * sizeof(int2));
  if (!rc) rc = batch_upload(b, b->d_items, items.data(), items.size() * sizeof(int2));
  if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = fail(SW_EHIP, "batch upload failed");
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return SW_OK;
}

extern "C" int sw_batch_apply_f32(sw_batch* b, const float* const* x, float* const* y) {
  if (!b || !x || !y) return fail(SW_EINVAL, "NULL argument");
  for (int l = 0; l < b->n; ++l)
    if (!x[l] || !y[l]) return fail(SW_EINVAL, "NULL vector of lane %d", l);
  HIPC(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  // every lane's inner-solve vectors and control block are free between
  // steps: the input goes into p32, q32 is cleared whole, and a fresh
  // control block makes every work item run in full (an iteration past the
  // first, as in an inner CG iteration)
  for (int l = 0; l < b->n; ++l) {
    sw_case* c = b->cases[l];
    const int64_t nn = c->mesh->n_nodes;
    launch_permute_f32(nn, 3, x[l], c->mesh->dev.node_i2u, c->p32, s);
    launch_fill_f32(3 * nn, c->q32, 0.0f, s);
    launch_fill_f64(sizeof(CgCtl) / 8, (double*)c->ctl32, 0.0, s);
    b->st[l].active = 1;
  }
  LAUNCHED();
  int rc = batch_upload(b, b->d_st, b->st.data(), b->n * sizeof(LaneState));
  if (rc) return rc;
  launch_tile_lanes_pipe_f32(b->d_cg32, b->d_items, b->n_items, b->max_tile_nodes, b->d_st, 1, batch_grid_cap(b),
                             s);
  for (int l = 0; l < b->n; ++l) {
    sw_case* c = b->cases[l];
    launch_permute_f32(c->mesh->n_nodes, 3, c->q32, c->mesh->dev.node_u2i, y[l], s);
  }
  LAUNCHED();
  HIPC(hipStreamSynchronize(s));
  return SW_OK;
}

extern "C" int sw_batch_stats(const sw_batch* b, sw_case_stats* out) {
  if (!b || !out) return fail(SW_EINVAL, "NULL argument");
  for (int l = 0; l < b->n; ++l) {
    int rc = sw_case_stats_get(b->cases[l], out + l);
    if (rc) return rc;
  }
  return SW_OK;
}

namespace {

int cu_count(int device, int* out) {
  int v = 0;
  HIPC(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
  *out = v > 0 ? v : 256;
  return SW_OK;
}

// Mean duration (ms) of `reps` launches of fn after one untimed launch.
template <typename F>
int time_launches(hipStream_t s, int reps, F&& fn, double* ms) {
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  fn();
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) fn();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(SW_EHIP, "autotune timing failed: %s", hipGetErrorString(e));
  *ms = (double)t / reps;
  return SW_OK;
}

}  // namespace

extern "C" int sw_case_autotune(sw_case* c, int32_t reps, int32_t* choice, double* ms_out) {
  if (!c) return fail(SW_EINVAL, "NULL case");
  if (c->precision == SW_FP64) return fail(SW_EINVAL, "autotune tunes the FP32 pass of the mixed precisions");
  if (reps < 1 || reps > 1000) return fail(SW_EINVAL, "reps must be in 1..1000");
  HIPC(hipSetDevice(c->ctx->device));
  hipStream_t s = c->ctx->stream;
  int n_cu = 0;
  if (int rc = cu_count(c->ctx->device, &n_cu)) return rc;
  const int64_t nd = 3 * c->mesh->n_nodes;
  // zero input (the same work as any other), fresh control block so every
  // launch runs in full; the inner-solve vectors are free between steps
  launch_fill_f32(nd, c->p32, 0.0f, s);
  launch_fill_f32(nd, c->q32, 0.0f, s);
  const int caps[3] = {0, 8 * std::max(1, 2 * n_cu / 8), 8 * std::max(1, n_cu / 8)};
  double ms[3];
  int best = 0;
  for (int k = 0; k < 3; ++k) {
    c->grid_cap = caps[k];
    launch_fill_f64(sizeof(CgCtl) / 8, (double*)c->ctl32, 0.0, s);
    int rc = time_launches(s, reps, [&] { apply_f32(c, SW_OP_A, c->p32, c->q32, c->ctl32, 1); }, &ms[k]);
    if (rc) return rc;
    if (ms[k] < ms[best]) best = k;
  }
  LAUNCHED();
  c->grid_cap = caps[best];
  if (choice) *choice = best;
  if (ms_out)
    for (int k = 0; k < 3; ++k) ms_out[k] = ms[k];
  return SW_OK;
}

extern "C" int sw_batch_autotune(sw_batch* b, int32_t reps, int32_t* choice, double* ms_out) {
  if (!b) return fail(SW_EINVAL, "NULL batch");
  if (reps < 1 || reps > 1000) return fail(SW_EINVAL, "reps must be in 1..1000");
  HIPC(hipSetDevice(b->ctx->device));
  hipStream_t s = b->ctx->stream;
  int n_cu = 0;
  if (int rc = cu_count(b->ctx->device, &n_cu)) return rc;
  for (int l = 0; l < b->n; ++l) {
    sw_case* c = b->cases[l];
    const int64_t nd = 3 * c->mesh->n_nodes;
    launch_fill_f32(nd, c->p32, 0.0f, s);
    launch_fill_f32(nd, c->q32, 0.0f, s);
    launch_fill_f64(sizeof(CgCtl) / 8, (double*)c->ctl32, 0.0, s);
    b->st[l].active = 1;
  }
  LAUNCHED();
  int rc = batch_upload(b, b->d_st, b->st.data(), b->n * sizeof(LaneState));
  if (rc) return rc;
  const int caps[2] = {0, 8 * std::max(1, 2 * n_cu / 8)};
  double ms[4];
  int best = 0;
  for (int sch = 0; sch < 2; ++sch) {
    const std::vector<int2> items = batch_items(b->cases.data(), b->n, sch);
    if ((rc = batch_upload(b, b->d_items, items.data(), items.size() * sizeof(int2)))) return rc;
    for (int g = 0; g < 2; ++g) {
      const int k = 2 * sch + g;
      rc = time_launches(s, reps, [&] {
        launch_tile_lanes_pipe_f32(b->d_cg32, b->d_items, b->n_items, b->max_tile_nodes, b->d_st, 1, caps[g], s);
      }, &ms[k]);
      if (rc) return rc;
      if (ms[k] < ms[best]) best = k;
    }
  }
  LAUNCHED();
  b->schedule = best / 2;
  b->grid_cap = caps[best % 2];
  const std::vector<int2> items = batch_items(b->cases.data(), b->n, b->schedule);
  if ((rc = batch_upload(b, b->d_items, items.data(), items.size() * sizeof(int2)))) return rc;
  HIPC(hipStreamSynchronize(s));
  if (choice) *choice = best;
  if (ms_out)
    for (int k = 0; k < 4; ++k) ms_out[k] = ms[k];
  return SW_OK;
}

extern "C" int sw_batch_step(sw_batch* b, int32_t n_steps) {
  if (!b) return fail(SW_EINVAL, "NULL batch");
  if (n_steps < 0) return fail(SW_EINVAL, "negative step count");
  for (sw_case* c : b->cases) {
    if (c->step + n_steps > c->n_steps) return fail(SW_ESTATE, "a case would exceed its step capacity");
    if (needs_mlp(c)) return fail(SW_ESTATE, "SW_GUESS_MLP and SW_GUESS_PROJ_MLP need sw_case_attach_mlp first");
  }
  HIPC(hipSetDevice(b->ctx->device));
  for (int k = 0; k < n_steps; ++k) {
    int rc = batch_step_once(b);
    if (rc) return rc;
  }
  return SW_OK;
}

extern "C" int sw_batch_destroy(sw_batch* b) {
  if (b && b->cg_graph) (void)hipGraphExecDestroy(b->cg_graph);
  delete b;
  return SW_OK;
}
