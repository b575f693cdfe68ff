// Element-level arithmetic of the matrix-free (element-by-element) operator
// for 10-node tetrahedra and 6-node boundary triangles.
//
// The discretised operator is that of the linear elastodynamic equation of
// Section 2 (Eq. GE:ORG) on second-order tetrahedra (Section 3).  Nothing
// here forms an element matrix: each routine applies one to a vector.
//
// Stiffness.  For an affine quadratic tet the displacement gradient is
// linear, so it is fixed by its values G_k at the four vertices:
//     G_k = 3 u_k (x) g_k + sum_{j != k} (4 u_kj - u_j) (x) g_j,
// g_j = grad L_j.  The stress is linear too (sigma_k at vertex k) and the
// shape-function gradients are linear, so with the P1 mass weights
// int L_i L_k = V (1 + delta_ik) / 20 the element force is
//     S_k  = V/20 (sigma_k + sum_i sigma_i)
//     f_i  = (4 S_i - sum_k S_k) g_i                (vertex node i)
//     f_ij = 4 (S_i g_j + S_j g_i)                  (edge node ij)
// which is the exact K_e u with no quadrature.
//
// Consistent mass.  rho V / 420 times the closed-form P2 table
// {vertex 6, vertex-vertex 1, vertex-incident edge -4, vertex-opposite edge
// -6, edge 32, edges sharing a vertex 16, disjoint edges 8}, applied per
// component through vertex and edge sums.
//
// Face dashpot.  A/180 times the P2 triangle table {vertex 6,
// vertex-vertex -1, vertex-incident edge 0, vertex-opposite edge -4, edge 32,
// edge-edge 16}, times Z = rho Vs I + rho (Vp - Vs) n n^T.
#pragma once

#include <hip/hip_runtime.h>

namespace sw {

#define SW_HD __host__ __device__ __forceinline__

// VTK edge order of the tet: 01, 12, 02, 03, 13, 23
// edge slot (4 + e) for the edge between vertices a < b
SW_HD constexpr int tet_edge(int a, int b) {
  // a < b
  return (a == 0) ? (b == 1 ? 0 : (b == 2 ? 2 : 3)) : (a == 1 ? (b == 2 ? 1 : 4) : 5);
}

template <typename T>
struct Geo {
  T g[4][3];  // barycentric gradients
  T vol;
};

// Geometry from vertex coordinates (always read in FP64, differences taken in
// FP64, then narrowed to T).
template <typename T>
SW_HD bool tet_geometry(const double x[4][3], Geo<T>& G) {
  double c1[3], c2[3], c3[3];
  for (int d = 0; d < 3; ++d) {
    c1[d] = x[1][d] - x[0][d];
    c2[d] = x[2][d] - x[0][d];
    c3[d] = x[3][d] - x[0][d];
  }
  // rows of J^{-1} = (c2 x c3, c3 x c1, c1 x c2) / det
  double r1[3] = {c2[1] * c3[2] - c2[2] * c3[1], c2[2] * c3[0] - c2[0] * c3[2], c2[0] * c3[1] - c2[1] * c3[0]};
  double r2[3] = {c3[1] * c1[2] - c3[2] * c1[1], c3[2] * c1[0] - c3[0] * c1[2], c3[0] * c1[1] - c3[1] * c1[0]};
  double r3[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
  double det = c1[0] * r1[0] + c1[1] * r1[1] + c1[2] * r1[2];
  double inv = 1.0 / det;
  for (int d = 0; d < 3; ++d) {
    double a = r1[d] * inv, b = r2[d] * inv, c = r3[d] * inv;
    G.g[1][d] = (T)a;
    G.g[2][d] = (T)b;
    G.g[3][d] = (T)c;
    G.g[0][d] = (T)(-(a + b + c));
  }
  G.vol = (T)(det / 6.0);
  return det > 0.0;
}

// f = sK K_e w + sMV (table/420) w (sMV = sM rho V): the stiffness through
// the vertex stresses S_k, the mass through per-component vertex and edge
// sums.  Each node's force goes to sink(k, f0, f1, f2) as soon as it is
// complete, so no 30-value force array is held (fewer live registers in the
// tile passes, which scatter each force at once).  STIFF / MASS leave out
// a term whose coefficient the caller knows to be zero; fixed at compile
// time, they leave the per-node code free of branches.  DYN also skips a
// term whose coefficient is zero at run time (per element: branches in the
// per-node code, but a smaller register footprint where that matters more).
template <typename T, bool STIFF, bool MASS, bool DYN, typename Sink>
SW_HD void element_apply(const Geo<T>& G, T lam, T mu, T sK, T sMV, const T w[10][3], Sink&& sink) {
  const bool stiff = STIFF && (!DYN || sK != (T)0), mass = MASS && (!DYN || sMV != (T)0);
  // S'_k = sigma_k + sum_i sigma_i; with gs_j = 4 (V/20) sK g_j the forces
  // are f_i = (S'_i - 5/4 sum_k sigma_k) gs_i and f_ij = S'_i gs_j + S'_j gs_i
  // (the V/20 and the factor 4 folded into the twelve gradient values)
  T S[4][6];
  T s54[6] = {0, 0, 0, 0, 0, 0};
  T gs[4][3];
  if (stiff) {
    T sum[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      T Gm[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int d = 0; d < 3; ++d) Gm[c][d] = (T)3 * w[k][c] * G.g[k][d];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j == k) continue;
        const int e = 4 + (k < j ? tet_edge(k, j) : tet_edge(j, k));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T W = (T)4 * w[e][c] - w[j][c];
#pragma unroll
          for (int d = 0; d < 3; ++d) Gm[c][d] += W * G.g[j][d];
        }
      }
      T tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
      T l = lam * tr;
      S[k][0] = l + (T)2 * mu * Gm[0][0];
      S[k][1] = l + (T)2 * mu * Gm[1][1];
      S[k][2] = l + (T)2 * mu * Gm[2][2];
      S[k][3] = mu * (Gm[1][2] + Gm[2][1]);
      S[k][4] = mu * (Gm[0][2] + Gm[2][0]);
      S[k][5] = mu * (Gm[0][1] + Gm[1][0]);
#pragma unroll
      for (int m = 0; m < 6; ++m) sum[m] += S[k][m];
    }
    const T c4 = sK * G.vol * (T)0.2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int d = 0; d < 3; ++d) gs[j][d] = c4 * G.g[j][d];
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      s54[m] = (T)1.25 * sum[m];
#pragma unroll
      for (int k = 0; k < 4; ++k) S[k][m] += sum[m];
    }
  }
  // mass: per component the vertex sum, edge sum and each vertex's incident-edge sum
  const T s = sMV * (T)(1.0 / 420.0);
  T Uv[3], Ue[3], inc[4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Uv[c] = w[0][c] + w[1][c] + w[2][c] + w[3][c];
    Ue[c] = w[4][c] + w[5][c] + w[6][c] + w[7][c] + w[8][c] + w[9][c];
    inc[0][c] = w[4][c] + w[6][c] + w[7][c];
    inc[1][c] = w[4][c] + w[5][c] + w[8][c];
    inc[2][c] = w[5][c] + w[6][c] + w[9][c];
    inc[3][c] = w[7][c] + w[8][c] + w[9][c];
  }
  auto smv = [](const T sy[6], const T v[3], T o[3]) {
    o[0] = sy[0] * v[0] + sy[5] * v[1] + sy[4] * v[2];
    o[1] = sy[5] * v[0] + sy[1] * v[1] + sy[3] * v[2];
    o[2] = sy[4] * v[0] + sy[3] * v[1] + sy[2] * v[2];
  };
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T f[3] = {(T)0, (T)0, (T)0};
    if (stiff) {
      T sy[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) sy[m] = S[i][m] - s54[m];
      smv(sy, gs[i], f);
    }
    if (mass) {
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] += s * ((T)5 * w[i][c] + (Uv[c] - (T)6 * Ue[c]) + (T)2 * inc[i][c]);
    }
    sink(i, f[0], f[1], f[2]);
  }
  // edges 01,12,02,03,13,23 and their opposite edges 23,03,13,12,02,01
  const int ea[6] = {0, 1, 0, 0, 1, 2};
  const int eb[6] = {1, 2, 2, 3, 3, 3};
  const int eo[6] = {5, 3, 4, 1, 2, 0};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    T f[3] = {(T)0, (T)0, (T)0};
    if (stiff) {
      T f1[3], f2[3];
      smv(S[ea[e]], gs[eb[e]], f1);
      smv(S[eb[e]], gs[ea[e]], f2);
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] = f1[c] + f2[c];
    }
    if (mass) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        f[c] += s * (((T)16 * Ue[c] - (T)6 * Uv[c]) + (T)2 * (w[ea[e]][c] + w[eb[e]][c]) + (T)16 * w[4 + e][c] -
                     (T)8 * w[4 + eo[e]][c]);
    }
    sink(4 + e, f[0], f[1], f[2]);
  }
}

// Diagonal 3x3 blocks (symmetric, 6 values: xx yy zz yz xz xy) of
// cM * M_e + cK * K_e for the ten nodes.
template <typename T>
SW_HD void diag_blocks(const Geo<T>& G, T lam, T mu, T rho, T cM, T cK, T out[10][6]) {
  const T V = G.vol;
  auto outer_add = [](T a, const T u[3], const T v[3], T o[6]) {
    // o += a * sym(u v^T + v u^T) / 2 ... callers pass u == v or use twice
    o[0] += a * u[0] * v[0];
    o[1] += a * u[1] * v[1];
    o[2] += a * u[2] * v[2];
    o[3] += a * (T)0.5 * (u[1] * v[2] + u[2] * v[1]);
    o[4] += a * (T)0.5 * (u[0] * v[2] + u[2] * v[0]);
    o[5] += a * (T)0.5 * (u[0] * v[1] + u[1] * v[0]);
  };
  const int ea[6] = {0, 1, 0, 0, 1, 2};
  const int eb[6] = {1, 2, 2, 3, 3, 3};
  for (int a = 0; a < 10; ++a) {
    T Gm[6] = {0, 0, 0, 0, 0, 0};
    T mdiag;
    if (a < 4) {
      outer_add((T)3 * V / (T)5, G.g[a], G.g[a], Gm);
      mdiag = (T)6;
    } else {
      const T* gi = G.g[ea[a - 4]];
      const T* gj = G.g[eb[a - 4]];
      const T c = (T)4 * V / (T)5;
      outer_add((T)2 * c, gi, gi, Gm);
      outer_add((T)2 * c, gj, gj, Gm);
      outer_add((T)2 * c, gi, gj, Gm);  // g_i g_j^T + g_j g_i^T
      mdiag = (T)32;
    }
    const T tr = Gm[0] + Gm[1] + Gm[2];
    const T m = cM * rho * V * mdiag / (T)420;
    for (int k = 0; k < 6; ++k) out[a][k] = cK * (lam + mu) * Gm[k];
    for (int k = 0; k < 3; ++k) out[a][k] += cK * mu * tr + m;
  }
}

// ---------------------------------------------------------------- faces

struct FaceGeo {
  double n[3];
  double area;
};

SW_HD FaceGeo face_geometry(const double p[3][3]) {
  double a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = p[1][d] - p[0][d];
    b[d] = p[2][d] - p[0][d];
  }
  double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  double l = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  FaceGeo f;
  for (int d = 0; d < 3; ++d) f.n[d] = c[d] / l;
  f.area = 0.5 * l;
  return f;
}

// y += s * C_f w  (w, y: [6][3]); zs = rho Vs, zp = rho Vp
template <typename T>
SW_HD void face_dashpot_apply(const T n[3], T area, T zp, T zs, T s, const T w[6][3], T y[6][3]) {
  T W[6][3];
  const T a = area / (T)180;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T Uv = w[0][c] + w[1][c] + w[2][c];
    T Ue = w[3][c] + w[4][c] + w[5][c];
    // tri edges e0=(0,1) e1=(1,2) e2=(2,0); opposite: v0<->e1, v1<->e2, v2<->e0
    W[0][c] = a * ((T)7 * w[0][c] - Uv - (T)4 * w[4][c]);
    W[1][c] = a * ((T)7 * w[1][c] - Uv - (T)4 * w[5][c]);
    W[2][c] = a * ((T)7 * w[2][c] - Uv - (T)4 * w[3][c]);
    W[3][c] = a * ((T)16 * w[3][c] + (T)16 * Ue - (T)4 * w[2][c]);
    W[4][c] = a * ((T)16 * w[4][c] + (T)16 * Ue - (T)4 * w[0][c]);
    W[5][c] = a * ((T)16 * w[5][c] + (T)16 * Ue - (T)4 * w[1][c]);
  }
  const T dz = zp - zs;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T nw = n[0] * W[k][0] + n[1] * W[k][1] + n[2] * W[k][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) y[k][c] += s * (zs * W[k][c] + dz * nw * n[c]);
  }
}

}  // namespace sw
