// LDS-tiled element-by-element kernels (gfx950).
//
// One workgroup per tile (see sw_mesh.cpp): it gathers the tile's node
// values into LDS, applies every element of the tile (and the boundary
// faces owned by those elements) with LDS atomics into a per-tile
// accumulator, then writes the tile's interior nodes with plain coalesced
// stores and its shared nodes with one global atomic per value.  Against a
// scatter of every element entry to global memory this cuts global atomics
// from 30 per tet to about 2 per tet, and the ones left are address-sorted.
#include <hip/hip_runtime.h>

#include "sw_bf16.h"
#include "sw_device.h"
#include "sw_elem.h"
#include "sw_internal.h"
#include "sw_layout.h"

#include <algorithm>

#ifndef SW_PIPE_PF
#define SW_PIPE_PF false
#endif

namespace sw {

// Load through the constant address space: with a uniform index this is a
// scalar load, which is not counted with the vector loads (those complete
// in order, so waiting for one waits for every older one).  For the
// per-tile offsets and counts, constant during a kernel.
template <typename U>
__device__ __forceinline__ U ldc(const U* p, int64_t i) {
  return ((const __attribute__((address_space(4))) U*)p)[i];
}

// Input value i of a pass (x1), and of its dashpot term (xf): in the 16-bit
// passes of the SW_MIXED_FP16 inner CG both come from the bfloat16 input
// x1h (x1 and xf null), so every term of A acts on the same stored values.
template <typename T>
__device__ __forceinline__ T x1_at(const TileArgs<T>& A, int64_t i) {
  return A.x1[i];
}
template <>
__device__ __forceinline__ float x1_at<float>(const TileArgs<float>& A, int64_t i) {
  return A.x1h ? bf16_value(A.x1h[i]) : A.x1[i];
}
template <typename T>
__device__ __forceinline__ T xf_at(const TileArgs<T>& A, int64_t i) {
  return A.xf[i];
}
template <>
__device__ __forceinline__ float xf_at<float>(const TileArgs<float>& A, int64_t i) {
  return A.x1h ? bf16_value(A.x1h[i]) : A.xf[i];
}

// Per-element inputs fetched from global memory: tile-local connectivity
// (stored as 3 x the local index: the offset of the node's first value in
// the tile's 3-value-per-node LDS arrays, which saves the address
// arithmetic), material id, and the precomputed barycentric gradients and
// volume in the pass's precision (coalesced streams, no dependent gather).
template <typename T>
struct ElemIn {
  int ln[10];
  T geo[10];
  int mid;
};

template <typename T>
__device__ __forceinline__ const T* geo_of(const MeshDev& m);
template <>
__device__ __forceinline__ const float* geo_of<float>(const MeshDev& m) {
  return m.geo32;
}
template <>
__device__ __forceinline__ const double* geo_of<double>(const MeshDev& m) {
  return m.geo64;
}

template <typename T>
__device__ __forceinline__ void load_elem(const MeshDev& m, const uint8_t* __restrict__ emat, int e, ElemIn<T>& o) {
  const T* __restrict__ geo = geo_of<T>(m);
#pragma unroll
  for (int k = 0; k < 10; ++k) o.ln[k] = m.conn_loc[k * m.tet_stride + e];
#pragma unroll
  for (int k = 0; k < 10; ++k) o.geo[k] = geo[k * m.tet_stride + e];
  o.mid = emat[e];
}

// g_0 = -(g_1 + g_2 + g_3), summed in the order tet_geometry uses, so the
// FP64 operator is the one computed from the coordinates bit for bit
template <typename T>
__device__ __forceinline__ void elem_geometry(const ElemIn<T>& in, Geo<T>& G) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    G.g[1][d] = in.geo[d];
    G.g[2][d] = in.geo[3 + d];
    G.g[3][d] = in.geo[6 + d];
    G.g[0][d] = -(in.geo[d] + in.geo[3 + d] + in.geo[6 + d]);
  }
  G.vol = in.geo[9];
}

// Element work of tile t on the values gathered in LDS (xs, node ids gid),
// accumulated into ys (x.A x, which CG passes need, is taken afterwards from
// the tile's node values: tile_scatter).  Work-item i takes the tile's
// element i, i + NT, ...: the layout has grouped the elements of each
// half-wavefront and numbered the tile's interior nodes so that the nodes one
// LDS instruction reaches rarely share a bank (and rarely coincide), while
// the element loads stay coalesced.  PF: software
// pipeline, the next element's connectivity, geometry and material are
// loaded before the current one is computed (FP32; in FP64 the registers
// would halve the occupancy).  STIFF / MASS / DYN: which operator terms are
// on, and whether each element checks its coefficients (element_apply).
// hook() runs once, right after the first element's loads are issued (the
// pipelined pass issues its next tile's gather there, behind them).  MATL:
// the material constants come from an LDS copy (matl: lam, mu, rho per
// material) rather than from global memory, a load that would wait on the
// element's material id.  DET: each element's ten nodal results go to its
// slots of A.eout instead of the LDS accumulator.
template <typename T, int NT, bool PF, bool STIFF, bool MASS, bool DYN, bool MATL, bool DET, typename Hook>
__device__ __forceinline__ void tile_element_loop(const MeshDev& m, const uint8_t* __restrict__ emat,
                                                  const MatDev* __restrict__ mats, const float* matl,
                                                  const TileArgs<T>& A, int t, const int32_t* gid, const T* xs,
                                                  double* ys, Hook&& hook) {
  const int eb = ldc(m.tile_elem_off, t);
  const int n_e = ldc(m.tile_elem_off, t + 1) - eb;
  auto elem_of = [&](int i) { return eb + i; };
  ElemIn<T> nx;
  int i = threadIdx.x;
  if (i < n_e) load_elem<T>(m, emat, elem_of(i), nx);
  hook();
  constexpr bool kPrefetch = PF;
  for (; i < n_e; i += NT) {
    if (!kPrefetch && i != (int)threadIdx.x) load_elem<T>(m, emat, elem_of(i), nx);
    const ElemIn<T> cur = nx;
    if (kPrefetch && i + NT < n_e) load_elem<T>(m, emat, elem_of(i + NT), nx);
    const int* ln = cur.ln;
    Geo<T> G;
    elem_geometry(cur, G);
    T lam, mu, rho;
    if constexpr (MATL) {
      lam = matl[3 * cur.mid];
      mu = matl[3 * cur.mid + 1];
      rho = matl[3 * cur.mid + 2];
    } else {
      const MatDev& mt = mats[cur.mid];
      lam = (T)mt.lam;
      mu = (T)mt.mu;
      rho = (T)mt.rho;
    }
    T w[10][3];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) w[k][c] = xs[ln[k] + c];
    }
    // each node's force goes to the LDS accumulator as soon as it is
    // complete (no 30-value force array held in registers)
    element_apply<T, STIFF, MASS, DYN>(G, lam, mu, A.sK, A.sM * rho * G.vol, w,
                                  [&](int k, T f0, T f1, T f2) {
                                    if constexpr (DET) {
                                      double* eo = A.eout + (size_t)elem_of(i) * 30 + 3 * k;
                                      eo[0] = (double)f0;
                                      eo[1] = (double)f1;
                                      eo[2] = (double)f2;
                                    } else {
                                      double* yk = &ys[ln[k]];
                                      atomicAdd(yk, (double)f0);
                                      atomicAdd(yk + 1, (double)f1);
                                      atomicAdd(yk + 2, (double)f2);
                                    }
                                  });
  }
}

// Element and face work of tile t (see tile_element_loop), plus the
// boundary faces owned by the tile's elements (DET: their results to the
// face slots of A.fout).
template <typename T, int NT, bool PF, bool MATL, bool DET, typename Hook>
__device__ __forceinline__ void tile_elements(const MeshDev& m, const uint8_t* __restrict__ emat,
                                              const MatDev* __restrict__ mats, const float* matl,
                                              const TileArgs<T>& A, int t, const int32_t* gid, const T* xs,
                                              double* ys, Hook&& hook) {
  if constexpr (sizeof(T) == 8) {
    // FP64: per-element checks (the branch-free form needs more registers
    // than the FP64 passes can spare; measured slower)
    if (A.sK != (T)0 || A.sM != (T)0)
      tile_element_loop<T, NT, PF, true, true, true, MATL, DET>(m, emat, mats, matl, A, t, gid, xs, ys,
                                                                        hook);
    else
      hook();
  } else {
    if (A.sK != (T)0 && A.sM != (T)0)
      tile_element_loop<T, NT, PF, true, true, false, MATL, false>(m, emat, mats, matl, A, t, gid, xs, ys,
                                                                           hook);
    else if (A.sK != (T)0)
      tile_element_loop<T, NT, PF, true, false, false, MATL, false>(m, emat, mats, matl, A, t, gid, xs, ys,
                                                                            hook);
    else if (A.sM != (T)0)
      tile_element_loop<T, NT, PF, false, true, false, MATL, false>(m, emat, mats, matl, A, t, gid, xs, ys,
                                                                            hook);
    else
      hook();
  }
  if (A.sC != (T)0 || A.vin != nullptr) {
    const int f1 = ldc(m.tile_face_off, t + 1);
    for (int f = ldc(m.tile_face_off, t) + threadIdx.x; f < f1; f += NT) {
      int ln[6];
      int64_t gn[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        ln[k] = m.fconn_loc[k * m.face_stride + f];
        gn[k] = m.fconn[k * m.face_stride + f];
      }
      double P[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int d = 0; d < 3; ++d) P[k][d] = m.xyz[3 * gn[k] + d];
      }
      const FaceGeo g = face_geometry(P);
      const MatDev mt = mats[emat[m.face_elem[f]]];
      T out[6][3];
#pragma unroll
      for (int k = 0; k < 6; ++k) out[k][0] = out[k][1] = out[k][2] = (T)0;
      if (A.sC != (T)0) {
        T w[6][3];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
#pragma unroll
          for (int c = 0; c < 3; ++c) w[k][c] = xf_at(A, 3 * gn[k] + c);
        }
        const T n[3] = {(T)g.n[0], (T)g.n[1], (T)g.n[2]};
        face_dashpot_apply<T>(n, (T)g.area, (T)mt.zp, (T)mt.zs, A.sC, w, out);
      }
      if (A.vin != nullptr && m.face_role[f] == 2) {
        // incident wave: traction 2 Z v_in, consistent load A/3 on the edge nodes
        const double nv = g.n[0] * A.vin[0] + g.n[1] * A.vin[1] + g.n[2] * A.vin[2];
        const double w3 = g.area / 3.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T f3 = (T)(w3 * 2.0 * (mt.zs * A.vin[c] + (mt.zp - mt.zs) * nv * g.n[c]));
          out[3][c] += f3;
          out[4][c] += f3;
          out[5][c] += f3;
        }
      }
      if constexpr (DET) {
        double* fo = A.fout + (size_t)f * 18;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
#pragma unroll
          for (int c = 0; c < 3; ++c) fo[3 * k + c] = (double)out[k][c];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
#pragma unroll
          for (int c = 0; c < 3; ++c) atomicAdd(&ys[3 * ln[k] + c], (double)out[k][c]);
        }
      }
    }
  }
}

template <typename T, int NT, bool PF>
__device__ __forceinline__ void tile_elements(const MeshDev& m, const uint8_t* __restrict__ emat,
                                              const MatDev* __restrict__ mats, const TileArgs<T>& A, int t,
                                              const int32_t* gid, const T* xs, double* ys) {
  tile_elements<T, NT, PF, false, false>(m, emat, mats, nullptr, A, t, gid, xs, ys, [] {});
}

// Results of tile t: interior nodes (one contiguous range) with plain
// stores, shared nodes with address-sorted global atomics.  Returns this
// work-item's share of the tile's x.(A x)_tile = sum over the tile's nodes
// of the input value times the tile's partial sum: summed over the tiles it
// is x.A x (a node's full value is the sum of its tiles' partials), with one
// product per node value instead of one per element entry.
template <typename T, int NT>
__device__ __forceinline__ double tile_scatter(const MeshDev& m, const TileArgs<T>& A, int t, const int32_t* gid,
                                               const T* xs, const double* ys) {
  const int nt = ldc(m.tile_node_off, t + 1) - ldc(m.tile_node_off, t);
  const int nint = ldc(m.tile_nint, t);
  const int64_t ib3 = 3 * (int64_t)ldc(m.tile_int_base, t);
  T* __restrict__ y = A.y;
  double energy = 0.0;
  for (int k = threadIdx.x; k < 3 * nint; k += NT) {
    const double v = ys[k];
    energy += (double)xs[k] * v;
    if (A.accumulate)
      y[ib3 + k] += (T)v;
    else
      y[ib3 + k] = (T)v;
  }
  // shared nodes: address-sorted global atomics
  for (int k = 3 * nint + threadIdx.x; k < 3 * nt; k += NT) {
    const int j = k / 3;
    const double v = ys[k];
    energy += (double)xs[k] * v;
    atomic_add(&y[3 * (int64_t)gid[j] + (k - 3 * j)], (T)v);
  }
  return energy;
}

// One workgroup's share of an operator pass: tile t of mesh m.  smem_raw is
// the dynamic LDS (sized for m.max_tile_nodes), sh NT/64 doubles.  DET: the
// element and face results go to their slots (no scatter, no energy; the
// node pass and a fixed-order dot product follow).
template <typename T, int NT, bool DET = false>
__device__ __forceinline__ void tile_body(const MeshDev& m, const uint8_t* __restrict__ emat,
                                          const MatDev* __restrict__ mats, const TileArgs<T>& A, CgCtl* ctl,
                                          int iter, int t, unsigned char* smem_raw, double* sh) {
  // LDS: FP64 accumulators (LDS FP64 atomics are much faster than FP32 ones
  // on this target), then the tile's input values in T
  double* ys = reinterpret_cast<double*>(smem_raw);
  int32_t* gid = reinterpret_cast<int32_t*>(ys + 3 * m.max_tile_nodes);
  T* xs = reinterpret_cast<T*>(gid + m.max_tile_nodes + (m.max_tile_nodes & 1));
  // CG-iteration protocol: exit when the solve is done; on the first
  // iteration end a solve whose initial residual meets the tolerance; the
  // workgroup of tile 0 clears the scalar slots the next update kernel
  // accumulates into.
  if (iter >= 0) {
    const int par = iter & 1;
    if (ctl->done) return;
    if (iter == 0 && slot_sum<NSLOT>(ctl->rr[0]) <= ctl->tol2) {
      if (t == 0 && threadIdx.x == 0) ctl->done = 1;
      return;
    }
    if (t == 0 && threadIdx.x < NSLOT) {
      ctl->rz[par ^ 1][threadIdx.x] = 0.0;
      ctl->rr[par ^ 1][threadIdx.x] = 0.0;
    }
  }
  const int n0 = ldc(m.tile_node_off, t);
  const int nt = ldc(m.tile_node_off, t + 1) - n0;
  const int nint = ldc(m.tile_nint, t);
  const int64_t ib3 = 3 * (int64_t)ldc(m.tile_int_base, t);

  // gather xe = a1 x1 + a2 x2 for the tile's nodes and clear the
  // accumulator, issued behind the first element's loads (the hook of
  // tile_elements): the interior nodes are one contiguous range; the shared
  // ones take their ids from the tile's node list (kept in LDS for the
  // scatter)
  auto gather = [&] {
    for (int k = threadIdx.x; k < 3 * nint; k += NT) {
      T v = A.a1 * x1_at(A, ib3 + k);
      if (A.x2 != nullptr) v += A.a2 * A.x2[ib3 + k];
      xs[k] = v;
      ys[k] = 0.0;
    }
    for (int j = nint + threadIdx.x; j < nt; j += NT) {
      const int32_t g = m.tile_nodes[n0 + j];
      gid[j] = g;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t gi = 3 * (int64_t)g + c;
        T v = A.a1 * x1_at(A, gi);
        if (A.x2 != nullptr) v += A.a2 * A.x2[gi];
        xs[3 * j + c] = v;
        ys[3 * j + c] = 0.0;
      }
    }
    __syncthreads();
  };
  tile_elements<T, NT, sizeof(T) == 4, false, DET>(m, emat, mats, nullptr, A, t, gid, xs, ys, gather);
  if constexpr (DET) return;
  __syncthreads();
  const double energy = tile_scatter<T, NT>(m, A, t, gid, xs, ys);
  if (iter >= 0) {
    const double s = block_sum_n<NT>(energy, sh);
    if (threadIdx.x == 0) atomic_add(&ctl->pAp[t % NSLOT], s);
  }
}

template <typename T, int NT, bool DET = false>
__global__ __launch_bounds__(NT) void k_tile(MeshDev m, const uint8_t* __restrict__ emat,
                                              const MatDev* __restrict__ mats, TileArgs<T> A, CgCtl* ctl, int iter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[NT / 64];
  tile_body<T, NT, DET>(m, emat, mats, A, ctl, iter, blockIdx.x, smem_raw, sh);
}

// Deterministic node pass: y[ystride * i + yoff + c] (= or +=) the sum over
// node i's element slots, then its face slots, in increasing slot order
// (elems / faces: whether the pass wrote them).  A CG iteration (iter >= 0)
// whose solve is done does nothing.
__global__ __launch_bounds__(TPB) void k_node_gather(MeshDev m, const double* __restrict__ eout,
                                                     const double* __restrict__ fout, double* __restrict__ y,
                                                     int ystride, int yoff, int accumulate, int elems, int faces,
                                                     const CgCtl* ctl, int iter) {
  if (iter >= 0 && ctl->done) return;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < m.n_nodes; i += (int64_t)gridDim.x * TPB) {
    double a[3] = {0.0, 0.0, 0.0};
    if (elems)
      for (int j = m.inc_off[i]; j < m.inc_off[i + 1]; ++j) {
        const double* e = eout + 3 * (size_t)m.inc[j];
        a[0] += e[0];
        a[1] += e[1];
        a[2] += e[2];
      }
    if (faces)
      for (int j = m.finc_off[i]; j < m.finc_off[i + 1]; ++j) {
        const double* f = fout + 3 * (size_t)m.finc[j];
        a[0] += f[0];
        a[1] += f[1];
        a[2] += f[2];
      }
    double* yi = y + (int64_t)ystride * i + yoff;
#pragma unroll
    for (int c = 0; c < 3; ++c) yi[c] = accumulate ? yi[c] + a[c] : a[c];
  }
}

// slots[b] = workgroup b's share of x.y, one workgroup per slot (a
// fixed-order sum); nothing when the CG solve in ctl is done.
__global__ __launch_bounds__(TPB) void k_dot_slots(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ y, double* __restrict__ slots,
                                                   const CgCtl* ctl) {
  __shared__ double sh[2 * TPB / 64];
  if (ctl->done) return;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n; k += (int64_t)gridDim.x * TPB) acc += x[k] * y[k];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) slots[blockIdx.x] = acc;
}

// The same pass for several cases (lanes) in one launch: work item b is
// (lane, tile) = work[b] (lane < 0: padding), lanes whose state is inactive
// return at once.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_tile_lanes(const TileLane<T>* __restrict__ lanes,
                                                    const int2* __restrict__ work,
                                                    const LaneState* __restrict__ st, int iter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[NT / 64];
  const int2 w = work[blockIdx.x];
  if (w.x < 0) return;
  if (st != nullptr && !st[w.x].active) return;
  const TileLane<T>& L = lanes[w.x];
  tile_body<T, NT>(L.m, L.emat, L.mats, L.A, L.ctl, iter, w.y, smem_raw, sh);
}

// Largest material table the pipelined pass copies into LDS.
constexpr int PIPE_MATS = 32;

// FP32 operator pass of a CG iteration (input scaled by 1, no second input),
// persistent and software-pipelined.  Each workgroup walks a run of tiles;
// while it computes tile t it already loads the input values of its next
// tile into registers (node by node, 12 contiguous bytes per node), so a
// tile's gather latency hides behind the element work of the one before.
// Order of the loads, since a wait for a vector load also waits for every
// older one: the node ids of tile t+1 are loaded at the end of tile t-1;
// tile t's first element data goes out before the values of tile t+1, so
// the element work waits only for its own data; per-tile offsets and counts
// are scalar loads; the material constants come from an LDS copy.
// XCD-aware: workgroup b runs on XCD b mod 8 (workgroups are dealt to the 8
// XCDs round-robin) and takes its tiles from that XCD's contiguous eighth of
// the tile list, so neighbouring tiles, which share nodes, meet in the same
// L2.  NPT * NT must cover the largest tile; at most PIPE_MATS materials.
template <int NT, int NPT, bool PF, bool H16 = false>
__global__ __launch_bounds__(NT) void k_tile_pipe(MeshDev m, const uint8_t* __restrict__ emat,
                                                   const MatDev* __restrict__ mats, TileArgs<float> A, CgCtl* ctl,
                                                   int iter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[NT / 64];
  double* ys = reinterpret_cast<double*>(smem_raw);
  int32_t* gid = reinterpret_cast<int32_t*>(ys + 3 * m.max_tile_nodes);
  float* xs = reinterpret_cast<float*>(gid + m.max_tile_nodes + (m.max_tile_nodes & 1));
  // CG-iteration protocol (as in tile_body; workgroup 0 leads)
  const int par = iter & 1;
  if (ctl->done) return;
  if (iter == 0 && slot_sum<NSLOT>(ctl->rr[0]) <= ctl->tol2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x < NSLOT) {
    ctl->rz[par ^ 1][threadIdx.x] = 0.0;
    ctl->rr[par ^ 1][threadIdx.x] = 0.0;
  }
  const int xcd = blockIdx.x & 7, slots = gridDim.x >> 3, slot = blockIdx.x >> 3;
  const int lo = (int)(((int64_t)m.n_tiles * xcd) >> 3);
  const int hi = (int)(((int64_t)m.n_tiles * (xcd + 1)) >> 3);
  int t = lo + slot;
  if (t >= hi) return;
  // the input: FP32, or bfloat16 (H16: the 16-bit passes)
  const float* __restrict__ x = A.x1;
  const uint16_t* __restrict__ xh = A.x1h;
  auto in = [&](int64_t i) -> float {
    if constexpr (H16)
      return bf16_value(xh[i]);
    else
      return x[i];
  };
  // the material table, rounded to FP32, into LDS
  __shared__ float matl[3 * PIPE_MATS];
  for (int i = threadIdx.x; i < A.n_mat; i += NT) {
    matl[3 * i] = (float)mats[i].lam;
    matl[3 * i + 1] = (float)mats[i].mu;
    matl[3 * i + 2] = (float)mats[i].rho;
  }
  {
    // first tile: node ids and values straight into LDS
    const int n0 = ldc(m.tile_node_off, t), nt = ldc(m.tile_node_off, t + 1) - n0;
    for (int j = threadIdx.x; j < nt; j += NT) {
      const int32_t g = m.tile_nodes[n0 + j];
      gid[j] = g;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xs[3 * j + c] = in(3 * (int64_t)g + c);
        ys[3 * j + c] = 0.0;
      }
    }
  }
  // node ids of tile tn (0 past the tile: a valid index, loaded and unused)
  int32_t pg[NPT];
  auto load_ids = [&](int tn, int& ntn) {
    ntn = 0;
    int n0 = 0;
    if (tn < hi) {
      n0 = ldc(m.tile_node_off, tn);
      ntn = ldc(m.tile_node_off, tn + 1) - n0;
    }
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int j = threadIdx.x + q * NT;
      pg[q] = j < ntn ? m.tile_nodes[n0 + j] : 0;
    }
  };
  int ntn;
  load_ids(t + slots, ntn);
  __syncthreads();
  double energy = 0.0;
  for (;;) {
    const int tn = t + slots;
    const bool more = tn < hi;
    // the next tile's values: loaded behind the first element's loads, so
    // that the element work waits only for its own data
    float px[NPT][3];
    auto gather_next = [&] {
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const int64_t g3 = 3 * (int64_t)pg[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) px[q][c] = in(g3 + c);
      }
    };
    tile_elements<float, NT, PF, true, false>(m, emat, mats, matl, A, t, gid, xs, ys, gather_next);
    __syncthreads();
    energy += tile_scatter<float, NT>(m, A, t, gid, xs, ys);
    __syncthreads();
    if (!more) break;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int j = threadIdx.x + q * NT;
      if (j < ntn) {
        gid[j] = pg[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xs[3 * j + c] = px[q][c];
          ys[3 * j + c] = 0.0;
        }
      }
    }
    // ids of the tile after next: their latency overlaps the barrier and
    // the next tile's first element loads
    load_ids(tn + slots, ntn);
    __syncthreads();
    t = tn;
  }
  const double e = block_sum_n<NT>(energy, sh);
  if (threadIdx.x == 0) atomic_add(&ctl->pAp[blockIdx.x % NSLOT], e);
}

// The same persistent pipeline over the (lane, tile) items of several cases:
// items[k] = (lane, tile), tile-major with the lanes of a tile adjacent (they
// share the tile's mesh data through L2); XCD x owns the contiguous eighth
// [k_x, k_{x+1}) of the list.  An item is skipped when its lane is inactive or
// its solve is done (or, on the first iteration, already converged): every
// workgroup evaluates the same condition, so a skipped lane's output is left
// untouched; on the first iteration the workgroup whose scan passes the
// tile-0 item of an already converged lane marks that lane done (every item
// is visited by exactly one workgroup's scan).  nmax: the largest tile over
// the lanes (LDS layout).

template <int NT, int NPT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_tile_lanes_pipe(
    const TileLane<float>* __restrict__ lanes, const int2* __restrict__ items, int n_items, int nmax,
    const LaneState* __restrict__ st, int iter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[NT / 64];
  double* ys = reinterpret_cast<double*>(smem_raw);
  int32_t* gid = reinterpret_cast<int32_t*>(ys + 3 * nmax);
  float* xs = reinterpret_cast<float*>(gid + nmax + (nmax & 1));
  const int par = iter & 1;
  const int xcd = blockIdx.x & 7, slots = gridDim.x >> 3, slot = blockIdx.x >> 3;
  const int lo = (int)(((int64_t)n_items * xcd) >> 3);
  const int hi = (int)(((int64_t)n_items * (xcd + 1)) >> 3);
  // work item k, the same in every lane of the workgroup: readfirstlane
  // tells the compiler so, which keeps the item's lane and tile indices and
  // the lane's pointers in scalar registers (without it the kernel spilled
  // 29 vector registers)
  auto item = [&](int k) {
    int2 w = items[k];
    w.x = __builtin_amdgcn_readfirstlane(w.x);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    return w;
  };
  // next item at or after k (in steps of slots) that is not skipped (hi if none)
  auto next_live = [&](int k) {
    for (; k < hi; k += slots) {
      const int2 w = item(k);
      if (st != nullptr && !st[w.x].active) continue;
      CgCtl* c = lanes[w.x].ctl;
      if (c->done) continue;
      if (iter == 0 && slot_sum<NSLOT>(c->rr[0]) <= c->tol2) {
        if (w.y == 0 && threadIdx.x == 0) c->done = 1;
        continue;
      }
      break;
    }
    return k;
  };
  int k = __builtin_amdgcn_readfirstlane(next_live(lo + slot));
  if (k >= hi) return;
  int2 w = item(k);
  {
    const TileLane<float>& L = lanes[w.x];
    const int n0 = L.m.tile_node_off[w.y], nt = L.m.tile_node_off[w.y + 1] - n0;
    const float* __restrict__ x = L.A.x1;
    for (int j = threadIdx.x; j < nt; j += NT) {
      const int32_t g = L.m.tile_nodes[n0 + j];
      gid[j] = g;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xs[3 * j + c] = x[3 * (int64_t)g + c];
        ys[3 * j + c] = 0.0;
      }
    }
    __syncthreads();
  }
  for (;;) {
    const TileLane<float>& L = lanes[w.x];
    const int t = w.y;
    // lane duties of the tile-0 item: clear the slots the next update kernel
    // accumulates into
    if (t == 0 && threadIdx.x < NSLOT) {
      L.ctl->rz[par ^ 1][threadIdx.x] = 0.0;
      L.ctl->rr[par ^ 1][threadIdx.x] = 0.0;
    }
    const int kn = __builtin_amdgcn_readfirstlane(next_live(k + slots));
    const bool more = kn < hi;
    int2 wn = make_int2(0, 0);
    int32_t pg[NPT];
    float px[NPT][3];
    int ntn = 0;
    if (more) {
      wn = item(kn);
      const TileLane<float>& Ln = lanes[wn.x];
      const int n0 = Ln.m.tile_node_off[wn.y];
      ntn = Ln.m.tile_node_off[wn.y + 1] - n0;
      const float* __restrict__ xn = Ln.A.x1;
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const int j = threadIdx.x + q * NT;
        pg[q] = j < ntn ? Ln.m.tile_nodes[n0 + j] : 0;
      }
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const int64_t g3 = 3 * (int64_t)pg[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) px[q][c] = (threadIdx.x + q * NT < ntn) ? xn[g3 + c] : 0.0f;
      }
    }
    tile_elements<float, NT, false>(L.m, L.emat, L.mats, L.A, t, gid, xs, ys);
    __syncthreads();
    const double energy = tile_scatter<float, NT>(L.m, L.A, t, gid, xs, ys);
    const double e = block_sum_n<NT>(energy, sh);
    if (threadIdx.x == 0) atomic_add(&L.ctl->pAp[t % NSLOT], e);
    __syncthreads();
    if (!more) break;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int j = threadIdx.x + q * NT;
      if (j < ntn) {
        gid[j] = pg[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xs[3 * j + c] = px[q][c];
          ys[3 * j + c] = 0.0;
        }
      }
    }
    __syncthreads();
    k = kn;
    w = wn;
  }
}

// Workgroups of the persistent pass: three per compute unit (the LDS and
// register budget of the FP32 tile pass), a multiple of 8 (one run per XCD),
// at most `cap` when cap > 0 (fewer workgroups, each walking more tiles).
static unsigned pipe_grid(int n_tiles, int cap) {
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess && v > 0)
      n_cu = v;
    else
      n_cu = 256;
  }
  int per_xcd = std::max(1, std::min((n_tiles + 7) / 8, 3 * n_cu / 8));
  if (cap > 0) per_xcd = std::max(1, std::min(per_xcd, cap / 8));
  return (unsigned)(8 * per_xcd);
}

template <typename T>
static size_t tile_lds(int max_tile_nodes) {
  const size_t nmax = max_tile_nodes;
  return 3 * nmax * sizeof(double) + (nmax + (nmax & 1)) * sizeof(int32_t) + 3 * nmax * sizeof(T);
}

constexpr int PIPE_NT = 256, PIPE_NPT = 5;
static_assert(PIPE_NT * PIPE_NPT >= TILE_MAX_NODES, "the pipelined pass must cover a whole tile");

template <typename T>
static void launch_tile(const MeshDev& m, const uint8_t* emat, const MatDev* mats, const TileArgs<T>& a, CgCtl* ctl,
                        int iter, hipStream_t s, int grid_cap = 0) {
  const size_t lds = tile_lds<T>(m.max_tile_nodes);
  if constexpr (sizeof(T) == 4) {
    if (iter >= 0 && a.x2 == nullptr && a.a1 == 1.0f && a.accumulate == 0 && a.vin == nullptr &&
        m.max_tile_nodes <= PIPE_NT * PIPE_NPT && a.n_mat >= 1 && a.n_mat <= PIPE_MATS) {
      if (a.x1h)
        hipLaunchKernelGGL((k_tile_pipe<PIPE_NT, PIPE_NPT, SW_PIPE_PF, true>), dim3(pipe_grid(m.n_tiles, grid_cap)),
                           dim3(PIPE_NT), lds, s, m, emat, mats, a, ctl, iter);
      else
        hipLaunchKernelGGL((k_tile_pipe<PIPE_NT, PIPE_NPT, SW_PIPE_PF>), dim3(pipe_grid(m.n_tiles, grid_cap)),
                           dim3(PIPE_NT), lds, s, m, emat, mats, a, ctl, iter);
      return;
    }
  }
  // 4 waves per workgroup (6 measured slower for FP32)
  constexpr int NT = 256;
  hipLaunchKernelGGL((k_tile<T, NT>), dim3(m.n_tiles), dim3(NT), lds, s, m, emat, mats, a, ctl, iter);
}

static unsigned node_grid(int64_t n_nodes) {
  unsigned g = nblocks(n_nodes);
  return g > 8192 ? 8192 : (g == 0 ? 1 : g);
}

void launch_tile_f64(const MeshDev& m, const uint8_t* emat, const MatDev* mats, const TileArgs<double>& a,
                     CgCtl* ctl, int iter, hipStream_t s) {
  if (!a.eout) {
    launch_tile<double>(m, emat, mats, a, ctl, iter, s);
    return;
  }
  // deterministic: element and face slots, the node pass in slot order, and
  // p.Ap as a fixed-order dot product (a CG pass has x1 = p, a1 = 1)
  constexpr int NT = 256;
  hipLaunchKernelGGL((k_tile<double, NT, true>), dim3(m.n_tiles), dim3(NT), tile_lds<double>(m.max_tile_nodes), s, m,
                     emat, mats, a, ctl, iter);
  const int elems = a.sK != 0.0 || a.sM != 0.0, faces = a.sC != 0.0 || a.vin != nullptr;
  hipLaunchKernelGGL(k_node_gather, dim3(node_grid(m.n_nodes)), dim3(TPB), 0, s, m, a.eout, a.fout, a.y, 3, 0,
                     a.accumulate, elems, faces, ctl, iter);
  if (iter >= 0)
    hipLaunchKernelGGL(k_dot_slots, dim3(NSLOT), dim3(TPB), 0, s, 3 * m.n_nodes, a.x1, a.y, ctl->pAp, ctl);
}
void launch_tile_f32(const MeshDev& m, const uint8_t* emat, const MatDev* mats, const TileArgs<float>& a,
                     CgCtl* ctl, int iter, int grid_cap, hipStream_t s) {
  launch_tile<float>(m, emat, mats, a, ctl, iter, s, grid_cap);
}

void launch_tile_lanes_f64(const TileLane<double>* lanes, const int2* work, int n_work, int max_tile_nodes,
                           const LaneState* st, int iter, hipStream_t s) {
  hipLaunchKernelGGL((k_tile_lanes<double, 256>), dim3(n_work), dim3(256), tile_lds<double>(max_tile_nodes), s, lanes,
                     work, st, iter);
}
void launch_tile_lanes_pipe_f32(const TileLane<float>* lanes, const int2* items, int n_items, int max_tile_nodes,
                                const LaneState* st, int iter, int grid_cap, hipStream_t s) {
  hipLaunchKernelGGL((k_tile_lanes_pipe<PIPE_NT, PIPE_NPT>), dim3(pipe_grid(n_items, grid_cap)), dim3(PIPE_NT),
                     tile_lds<float>(max_tile_nodes), s, lanes, items, n_items, max_tile_nodes, st, iter);
}

// ------------------------------------------------------------ geometry

// Barycentric gradients (rows of the inverse Jacobian, L1..L3) and the volume
// of every element from the FP64 coordinates, in FP64 (geo64[k][e], k < 10)
// and rounded to FP32 (geo32).
__global__ __launch_bounds__(TPB) void k_geom(MeshDev m, float* __restrict__ geo32, double* __restrict__ geo64) {
  __shared__ int32_t gid[TILE_MAX_NODES];
  const int t = blockIdx.x;
  const int n0 = m.tile_node_off[t];
  const int nt = m.tile_node_off[t + 1] - n0;
  for (int j = threadIdx.x; j < nt; j += TPB) gid[j] = m.tile_nodes[n0 + j];
  __syncthreads();
  for (int e = m.tile_elem_off[t] + threadIdx.x; e < m.tile_elem_off[t + 1]; e += TPB) {
    double X[4][3];
    for (int k = 0; k < 4; ++k) {
      const int64_t g = gid[m.conn_loc[k * m.tet_stride + e] / 3];
      for (int d = 0; d < 3; ++d) X[k][d] = m.xyz[3 * g + d];
    }
    Geo<double> G;
    tet_geometry<double>(X, G);
    for (int j = 0; j < 3; ++j) {
      for (int d = 0; d < 3; ++d) {
        geo64[(3 * j + d) * m.tet_stride + e] = G.g[1 + j][d];
        geo32[(3 * j + d) * m.tet_stride + e] = (float)G.g[1 + j][d];
      }
    }
    geo64[9 * m.tet_stride + e] = G.vol;
    geo32[9 * m.tet_stride + e] = (float)G.vol;
  }
}

void launch_geom(const MeshDev& m, float* geo32, double* geo64, hipStream_t s) {
  hipLaunchKernelGGL(k_geom, dim3(m.n_tiles), dim3(TPB), 0, s, m, geo32, geo64);
}

// ------------------------------------------------------------ diagonal

// DET: values 3 half .. 3 half + 2 of each node's block go to the element
// and face slots (eout, fout) instead of the LDS accumulator; a node pass
// sums them in slot order.
template <bool DET>
__global__ __launch_bounds__(TPB) void k_tile_diag(MeshDev m, const uint8_t* __restrict__ emat,
                                                   const MatDev* __restrict__ mats, double cM, double cK, double cC,
                                                   double* __restrict__ diag6, int half, double* __restrict__ eout,
                                                   double* __restrict__ fout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ds = reinterpret_cast<double*>(smem_raw);
  const int t = blockIdx.x;
  const int n0 = m.tile_node_off[t];
  const int nt = m.tile_node_off[t + 1] - n0;
  const int nint = m.tile_nint[t];
  const int64_t ib6 = 6 * (int64_t)m.tile_int_base[t];
  const int32_t* __restrict__ gid = m.tile_nodes + n0;
  for (int k = threadIdx.x; k < 6 * nt; k += TPB) ds[k] = 0.0;
  __syncthreads();
  const int e1 = m.tile_elem_off[t + 1];
  for (int e = m.tile_elem_off[t] + threadIdx.x; e < e1; e += TPB) {
    int ln[10];
    for (int k = 0; k < 10; ++k) ln[k] = m.conn_loc[k * m.tet_stride + e] / 3;
    double X[4][3];
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) X[k][d] = m.xyz[3 * (int64_t)gid[ln[k]] + d];
    Geo<double> G;
    tet_geometry<double>(X, G);
    const MatDev mt = mats[emat[e]];
    double out[10][6];
    diag_blocks<double>(G, mt.lam, mt.mu, mt.rho, cM, cK, out);
    if constexpr (DET) {
      // static register indices (a run-time index would put out[][] in scratch)
#pragma unroll
      for (int k = 0; k < 10; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          eout[30 * (size_t)e + 3 * k + c] = half ? out[k][3 + c] : out[k][c];
    } else {
      for (int k = 0; k < 10; ++k)
        for (int j = 0; j < 6; ++j) atomicAdd(&ds[6 * ln[k] + j], out[k][j]);
    }
  }
  if (cC != 0.0) {
    const int f1 = m.tile_face_off[t + 1];
    for (int f = m.tile_face_off[t] + threadIdx.x; f < f1; f += TPB) {
      double P[3][3];
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) P[k][d] = m.xyz[3 * (int64_t)m.fconn[k * m.face_stride + f] + d];
      const FaceGeo g = face_geometry(P);
      const MatDev mt = mats[emat[m.face_elem[f]]];
      const double dz = mt.zp - mt.zs;
      const double Z[6] = {mt.zs + dz * g.n[0] * g.n[0], mt.zs + dz * g.n[1] * g.n[1], mt.zs + dz * g.n[2] * g.n[2],
                           dz * g.n[1] * g.n[2],         dz * g.n[0] * g.n[2],         dz * g.n[0] * g.n[1]};
      for (int k = 0; k < 6; ++k) {
        const int l = m.fconn_loc[k * m.face_stride + f];
        const double sc = cC * g.area / 180.0 * (k < 3 ? 6.0 : 32.0);
        if constexpr (DET) {
#pragma unroll
          for (int c = 0; c < 3; ++c) fout[18 * (size_t)f + 3 * k + c] = sc * (half ? Z[3 + c] : Z[c]);
        } else {
          for (int j = 0; j < 6; ++j) atomicAdd(&ds[6 * l + j], sc * Z[j]);
        }
      }
    }
  }
  if constexpr (DET) return;
  __syncthreads();
  for (int k = threadIdx.x; k < 6 * nint; k += TPB) diag6[ib6 + k] = ds[k];
  for (int k = 6 * nint + threadIdx.x; k < 6 * nt; k += TPB) {
    const int j = k / 6;
    atomic_add(&diag6[6 * (int64_t)gid[j] + (k - 6 * j)], ds[k]);
  }
}

void launch_tile_diag(const MeshDev& m, const uint8_t* emat, const MatDev* mats, double cM, double cK, double cC,
                      double* diag6, hipStream_t s, double* eout, double* fout) {
  const size_t lds = 6 * (size_t)m.max_tile_nodes * sizeof(double);
  if (!eout) {
    hipLaunchKernelGGL(k_tile_diag<false>, dim3(m.n_tiles), dim3(TPB), lds, s, m, emat, mats, cM, cK, cC, diag6, 0,
                       nullptr, nullptr);
    return;
  }
  for (int half = 0; half < 2; ++half) {
    hipLaunchKernelGGL(k_tile_diag<true>, dim3(m.n_tiles), dim3(TPB), lds, s, m, emat, mats, cM, cK, cC, diag6, half,
                       eout, fout);
    hipLaunchKernelGGL(k_node_gather, dim3(node_grid(m.n_nodes)), dim3(TPB), 0, s, m, eout, fout, diag6, 6, 3 * half,
                       0, 1, cC != 0.0 ? 1 : 0, nullptr, -1);
  }
}

// Inverse of each symmetric 3x3 block [[a xy xz][xy b yz][xz yz c]] by
// cofactors, in FP64; FP32 copy for the mixed-precision inner solve.
__global__ void k_fill_zero_d(double* p) { *p = 0.0; }

__global__ __launch_bounds__(TPB) void k_invert(int64_t n, const double* __restrict__ d6, double* __restrict__ p64,
                                                double* pmax, int* bad) {
  __shared__ double sh[TPB / 64];
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double mx = 0.0;
  if (i < n) {
    const double a = d6[6 * i + 0], b = d6[6 * i + 1], c = d6[6 * i + 2];
    const double yz = d6[6 * i + 3], xz = d6[6 * i + 4], xy = d6[6 * i + 5];
    const double c00 = b * c - yz * yz, c11 = a * c - xz * xz, c22 = a * b - xy * xy;
    const double c12 = -(a * yz - xy * xz), c02 = xy * yz - b * xz, c01 = -(xy * c - yz * xz);
    const double det = a * c00 + xy * c01 + xz * c02;
    if (!(det > 0.0) || !(a > 0.0)) *bad = 1;
    const double id = 1.0 / det;
    const double r[6] = {c00 * id, c11 * id, c22 * id, c12 * id, c02 * id, c01 * id};
    for (int k = 0; k < 6; ++k) p64[6 * i + k] = r[k];
    mx = fmax(fmax(r[0], r[1]), r[2]);
    if (!(mx > 0.0)) mx = 0.0;
  }
  // largest diagonal entry: positive doubles order like their bit patterns
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < TPB / 64; ++w) mx = fmax(mx, sh[w]);
    mx = fmax(mx, sh[0]);
    atomicMax(reinterpret_cast<unsigned long long*>(pmax), (unsigned long long)__double_as_longlong(mx));
  }
}

__global__ __launch_bounds__(TPB) void k_to_half(int64_t n6, const double* __restrict__ p64,
                                                 const double* __restrict__ pmax, __half* __restrict__ p16) {
  const double s = *pmax > 0.0 ? 1.0 / *pmax : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < n6; k += (int64_t)gridDim.x * TPB)
    p16[k] = __float2half((float)(p64[k] * s));
}

void launch_invert_blocks(int64_t n_nodes, const double* diag6, double* pinv64, __half* pinv16, double* pmax,
                          int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero_d, dim3(1), dim3(1), 0, s, pmax);
  hipLaunchKernelGGL(k_invert, dim3(nblocks(n_nodes)), dim3(TPB), 0, s, n_nodes, diag6, pinv64, pmax, bad);
  unsigned g = nblocks(6 * n_nodes);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_to_half, dim3(g), dim3(TPB), 0, s, 6 * n_nodes, pinv64, pmax, pinv16);
}

}  // namespace sw
