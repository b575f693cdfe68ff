// TEST INFRASTRUCTURE ONLY: the oracle's assembled-sparse solver for meshes
// too large for the SciPy oracle.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load it; it shares no code with the HIP
// library.
//
// What it computes (Section 2, Eq. GE:ORG, discretised on second-order
// tetrahedra as in Section 3; absorbing sides and base with the input
// applied as a force at the base, Sections 2-3):
//   * element stiffness by quadrature of the isotropic index form
//       K_ab,ij = int lambda dN_a/dx_i dN_b/dx_j + mu dN_a/dx_j dN_b/dx_i
//                     + mu delta_ij grad N_a . grad N_b  dV,
//     lambda = rho (Vp^2 - 2 Vs^2), mu = rho Vs^2;
//   * element mass  M_ab,ij = rho |J| Mref_ab delta_ij;
//   * boundary faces C_ab,ij = area Sref_ab Z_ij,
//       Z = rho Vp n n^T + rho Vs (I - n n^T)  (material of the owning tet);
//   * base input basis  F_c(a, i) = area Lref_a 2 Z_ic;
//   * global K, M, C_abs as symmetric 3x3 block-sparse matrices (upper
//     triangle stored, FP64), assembled element by element;
//   * the Newmark average-acceleration march (Section 3, Newmark-beta with
//     beta = 1/4, gamma = 1/2):
//       (4/dt^2 M + 2/dt C + K) du = F^{n+1} - K u^n + C v^n + M (a^n + 4/dt v^n),
//       C = alpha M + beta_R K + C_abs,
//     every step solved by 3x3 block-Jacobi preconditioned CG until the true
//     residual ||b - A du||_2 <= rtol ||b||_2.
// The reference-element data (quadrature points' shape-function gradients
// and weights, the reference mass and face tables) come from the Python
// oracle (oracle/fem.py), whose rules are pinned there.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Sys {
  int64_t n = 0;                 // nodes
  // K and M on one upper-triangular block pattern: per block 9 K then 9 M values
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> km;
  // C_abs on its own (boundary) pattern: 9 values per block
  std::vector<int64_t> crp;
  std::vector<int32_t> cci;
  std::vector<double> cv;
  std::vector<double> fb;        // input basis, 3 x 3n
  std::vector<int64_t> chunk;    // row ranges per thread (balanced by blocks)
  int threads = 1;
  std::vector<double> buf;       // per-thread transposed contributions, threads x 3n
};

// Upper-triangular pattern of the node graph of elements with `k` nodes each.
void build_pattern(int64_t n, int64_t ne, int k, const int32_t* conn, std::vector<int64_t>& rp,
                   std::vector<int32_t>& ci) {
  std::vector<int64_t> ip(n + 1, 0);
  for (int64_t e = 0; e < ne * k; ++e) ip[conn[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) ip[i + 1] += ip[i];
  std::vector<int64_t> inc(ip[n]);
  {
    std::vector<int64_t> pos(ip.begin(), ip.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int a = 0; a < k; ++a) inc[pos[conn[e * k + a]]++] = e;
  }
  rp.assign(n + 1, 0);
#pragma omp parallel
  {
    std::vector<int32_t> tmp;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      tmp.clear();
      for (int64_t p = ip[i]; p < ip[i + 1]; ++p)
        for (int a = 0; a < k; ++a) {
          const int32_t j = conn[inc[p] * k + a];
          if (j >= i) tmp.push_back(j);
        }
      std::sort(tmp.begin(), tmp.end());
      rp[i + 1] = std::unique(tmp.begin(), tmp.end()) - tmp.begin();
    }
  }
  for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
  ci.resize(rp[n]);
#pragma omp parallel
  {
    std::vector<int32_t> tmp;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      tmp.clear();
      for (int64_t p = ip[i]; p < ip[i + 1]; ++p)
        for (int a = 0; a < k; ++a) {
          const int32_t j = conn[inc[p] * k + a];
          if (j >= i) tmp.push_back(j);
        }
      std::sort(tmp.begin(), tmp.end());
      std::unique(tmp.begin(), tmp.end());
      std::copy(tmp.begin(), tmp.begin() + (rp[i + 1] - rp[i]), ci.begin() + rp[i]);
    }
  }
}

inline int64_t find_block(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, int32_t i, int32_t j) {
  const int32_t* b = ci.data() + rp[i];
  const int32_t* e = ci.data() + rp[i + 1];
  const int32_t* p = std::lower_bound(b, e, j);
  return rp[i] + (p - b);
}

inline void atomic_add(double* p, double v) {
#pragma omp atomic
  *p += v;
}

// Adds the element matrix E (dim x dim, dim = 3 k, DOF 3 a + i) of an element
// with nodes `nodes` into the upper-triangular pattern; values at stride
// `stride` doubles per block, offset `off`.
void scatter(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, double* vals, int stride, int off,
             int k, const int32_t* nodes, const double* E) {
  const int dim = 3 * k;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      const int32_t na = nodes[a], nb = nodes[b];
      if (na > nb) continue;
      double* blk = vals + find_block(rp, ci, na, nb) * stride + off;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) atomic_add(blk + 3 * i + j, E[(3 * a + i) * dim + 3 * b + j]);
    }
}

inline double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

void inv3(const double J[3][3], double R[3][3]) {
  const double d = det3(J);
  R[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
  R[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
  R[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
  R[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
  R[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
  R[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
  R[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
  R[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
  R[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
}

// y += sum over blocks of (cK K + cM M) x (both triangles) + cC C_abs x.
void spmv(Sys& S, double cK, double cM, double cC, const double* x, double* y) {
  const int64_t n3 = 3 * S.n;
#pragma omp parallel num_threads(S.threads)
  {
    const int t = omp_get_thread_num();
    const int64_t r0 = S.chunk[t], r1 = S.chunk[t + 1];
    double* tb = S.buf.data() + (size_t)t * n3;
    std::fill(tb + 3 * r0, tb + n3, 0.0);
    for (int64_t i = r0; i < r1; ++i) {
      double yi[3] = {0, 0, 0};
      const double* xi = x + 3 * i;
      for (int64_t p = S.rp[i]; p < S.rp[i + 1]; ++p) {
        const int64_t j = S.ci[p];
        const double* kb = S.km.data() + 18 * p;
        double B[9];
        for (int q = 0; q < 9; ++q) B[q] = cK * kb[q] + cM * kb[9 + q];
        const double* xj = x + 3 * j;
        for (int r = 0; r < 3; ++r) yi[r] += B[3 * r] * xj[0] + B[3 * r + 1] * xj[1] + B[3 * r + 2] * xj[2];
        if (j != i) {
          double* yj = tb + 3 * j;
          for (int c = 0; c < 3; ++c) yj[c] += B[c] * xi[0] + B[3 + c] * xi[1] + B[6 + c] * xi[2];
        }
      }
      for (int r = 0; r < 3; ++r) tb[3 * i + r] += yi[r];
    }
#pragma omp barrier
    // reduce the per-thread buffers over this thread's rows
    for (int64_t k = 3 * r0; k < 3 * r1; ++k) {
      double s = 0.0;
      for (int u = 0; u <= t; ++u) s += S.buf[(size_t)u * n3 + k];
      y[k] += s;
    }
  }
  if (cC != 0.0) {  // dashpots: boundary rows only, serial
    for (int64_t i = 0; i < S.n; ++i)
      for (int64_t p = S.crp[i]; p < S.crp[i + 1]; ++p) {
        const int64_t j = S.cci[p];
        const double* B = S.cv.data() + 9 * p;
        for (int r = 0; r < 3; ++r)
          y[3 * i + r] += cC * (B[3 * r] * x[3 * j] + B[3 * r + 1] * x[3 * j + 1] + B[3 * r + 2] * x[3 * j + 2]);
        if (j != i)
          for (int c = 0; c < 3; ++c)
            y[3 * j + c] += cC * (B[c] * x[3 * i] + B[3 + c] * x[3 * i + 1] + B[6 + c] * x[3 * i + 2]);
      }
  }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  const int64_t n = (int64_t)a.size();
#pragma omp parallel for reduction(+ : s)
  for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

}  // namespace

extern "C" {

// Builds K, M, C_abs and the input basis.  Returns a handle (NULL on a bad
// element: non-positive volume).
//   dNref: nq x 10 x 3 reference-coordinate shape gradients at the points
//          of a tetrahedron rule with weights wq (summing to 1/6);
//   Mref:  10 x 10, int N_a N_b over the reference tetrahedron;
//   Sref:  6 x 6, int N_a N_b dA per unit area over a triangle;
//   Lref:  6, int N_a dA per unit area.
void* oracle_bsr_create(int64_t n_nodes, int64_t n_tets, const double* xyz, const int32_t* tet10, int64_t n_faces,
                        const int32_t* tri6, const int32_t* face_tet, const uint8_t* face_role, int32_t n_mat,
                        const double* mat, const uint8_t* tet_mat, int32_t nq, const double* dNref,
                        const double* wq, const double* Mref, const double* Sref, const double* Lref) {
  omp_set_dynamic(0);  // the matvec's row ranges assume a full team
  Sys* S = new Sys;
  S->n = n_nodes;
  S->threads = omp_get_max_threads();
  build_pattern(n_nodes, n_tets, 10, tet10, S->rp, S->ci);
  S->km.assign(S->rp[n_nodes] * 18, 0.0);
  bool bad = false;
#pragma omp parallel
  {
    std::vector<double> Ke(900), Me(900), g(nq * 30);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t e = 0; e < n_tets; ++e) {
      const int32_t* nd = tet10 + 10 * e;
      double J[3][3], R[3][3];
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) J[i][k] = xyz[3 * nd[k + 1] + i] - xyz[3 * nd[0] + i];
      const double detJ = det3(J);
      if (!(detJ > 0.0)) {
        bad = true;
        continue;
      }
      inv3(J, R);  // R[k][c] = d xi_k / d x_c
      const double* m = mat + 3 * tet_mat[e];
      const double rho = m[2], mu = rho * m[1] * m[1], lam = rho * m[0] * m[0] - 2.0 * mu;
      for (int q = 0; q < nq; ++q)
        for (int a = 0; a < 10; ++a)
          for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += R[k][c] * dNref[(q * 10 + a) * 3 + k];
            g[(q * 10 + a) * 3 + c] = s;
          }
      std::fill(Ke.begin(), Ke.end(), 0.0);
      for (int q = 0; q < nq; ++q) {
        const double wv = wq[q] * detJ;
        for (int a = 0; a < 10; ++a)
          for (int b = 0; b < 10; ++b) {
            const double* ga = &g[(q * 10 + a) * 3];
            const double* gb = &g[(q * 10 + b) * 3];
            const double gg = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j)
                Ke[(3 * a + i) * 30 + 3 * b + j] +=
                    wv * (lam * ga[i] * gb[j] + mu * ga[j] * gb[i] + (i == j ? mu * gg : 0.0));
          }
      }
      std::fill(Me.begin(), Me.end(), 0.0);
      for (int a = 0; a < 10; ++a)
        for (int b = 0; b < 10; ++b)
          for (int i = 0; i < 3; ++i) Me[(3 * a + i) * 30 + 3 * b + i] = rho * detJ * Mref[a * 10 + b];
      scatter(S->rp, S->ci, S->km.data(), 18, 0, 10, nd, Ke.data());
      scatter(S->rp, S->ci, S->km.data(), 18, 9, 10, nd, Me.data());
    }
  }
  if (bad) {
    delete S;
    return nullptr;
  }
  // dashpot faces (roles 1, 2) and the input basis (role 2)
  std::vector<int32_t> fconn;
  std::vector<int64_t> fsel;
  for (int64_t f = 0; f < n_faces; ++f)
    if (face_role[f] == 1 || face_role[f] == 2) {
      fsel.push_back(f);
      fconn.insert(fconn.end(), tri6 + 6 * f, tri6 + 6 * f + 6);
    }
  build_pattern(n_nodes, (int64_t)fsel.size(), 6, fconn.data(), S->crp, S->cci);
  S->cv.assign(S->crp[n_nodes] * 9, 0.0);
  S->fb.assign(3 * 3 * (size_t)n_nodes, 0.0);
  std::vector<double> Ce(18 * 18);
  for (size_t s = 0; s < fsel.size(); ++s) {
    const int64_t f = fsel[s];
    const int32_t* nd = tri6 + 6 * f;
    const double* P0 = xyz + 3 * nd[0];
    const double* P1 = xyz + 3 * nd[1];
    const double* P2 = xyz + 3 * nd[2];
    const double e1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    const double e2[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double a2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    const double area = 0.5 * a2;
    const double nv[3] = {cr[0] / a2, cr[1] / a2, cr[2] / a2};
    const double* m = mat + 3 * tet_mat[face_tet[f]];
    const double zp = m[2] * m[0], zs = m[2] * m[1];
    double Z[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Z[i][j] = zp * nv[i] * nv[j] + zs * ((i == j ? 1.0 : 0.0) - nv[i] * nv[j]);
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) Ce[(3 * a + i) * 18 + 3 * b + j] = area * Sref[a * 6 + b] * Z[i][j];
    scatter(S->crp, S->cci, S->cv.data(), 9, 0, 6, nd, Ce.data());
    if (face_role[f] == 2)
      for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 6; ++a)
          for (int i = 0; i < 3; ++i) S->fb[(size_t)c * 3 * n_nodes + 3 * nd[a] + i] += area * Lref[a] * 2.0 * Z[i][c];
  }
  // thread row ranges balanced by stored blocks
  S->chunk.assign(S->threads + 1, n_nodes);
  S->chunk[0] = 0;
  const int64_t nb = S->rp[n_nodes];
  int t = 1;
  for (int64_t i = 0; i < n_nodes && t < S->threads; ++i)
    if (S->rp[i] >= nb * t / S->threads) S->chunk[t++] = i;
  S->buf.assign((size_t)S->threads * 3 * n_nodes, 0.0);
  return S;
}

void oracle_bsr_destroy(void* h) { delete (Sys*)h; }

int32_t oracle_bsr_threads(void* h) { return ((Sys*)h)->threads; }

int64_t oracle_bsr_blocks(void* h) { return ((Sys*)h)->rp.back(); }

// y = (cK K + cM M + cC C_abs) x
void oracle_bsr_apply(void* h, double cK, double cM, double cC, const double* x, double* y) {
  Sys& S = *(Sys*)h;
  std::fill(y, y + 3 * S.n, 0.0);
  spmv(S, cK, cM, cC, x, y);
}

// input basis row c (3n values)
void oracle_bsr_input_basis(void* h, double* out) {
  Sys& S = *(Sys*)h;
  std::copy(S.fb.begin(), S.fb.end(), out);
}

// March n_steps from (u, v, a) (updated in place).  v_in: (n_steps + 1) x 3,
// entry k + 1 drives step k.  guess: 0 = zero, 1 = previous increment.
// Outputs: rec (n_steps x n_rec x 3 velocities), iters (n_steps),
// relres (n_steps, final true relative residual), secs (n_steps, wall time).
// Returns 0, or -1 if a step does not converge within max_iter.
int32_t oracle_bsr_march(void* h, double dt, double alpha, double beta, const double* v_in, int64_t n_steps,
                         int32_t n_rec, const int32_t* rec, double* u, double* v, double* a, double rtol,
                         int32_t max_iter, int32_t guess, double* rec_out, int32_t* iters, double* relres,
                         double* secs) {
  Sys& S = *(Sys*)h;
  const int64_t n3 = 3 * S.n;
  const double cM = 4.0 / (dt * dt) + 2.0 * alpha / dt, cK = 1.0 + 2.0 * beta / dt, cC = 2.0 / dt;
  // 3x3 block-Jacobi inverse of A's diagonal blocks
  std::vector<double> Pinv(9 * S.n);
#pragma omp parallel for
  for (int64_t i = 0; i < S.n; ++i) {
    double D[3][3], R[3][3];
    const double* kb = S.km.data() + 18 * S.rp[i];  // first block of a row is its diagonal
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) D[r][c] = cK * kb[3 * r + c] + cM * kb[9 + 3 * r + c];
    if (S.crp[i + 1] > S.crp[i] && S.cci[S.crp[i]] == i)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) D[r][c] += cC * S.cv[9 * S.crp[i] + 3 * r + c];
    inv3(D, R);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Pinv[9 * i + 3 * r + c] = R[r][c];
  }
  std::vector<double> b(n3), du(n3, 0.0), r(n3), z(n3), p(n3), q(n3), w(n3), t1(n3), t2(n3);
  const double c1 = 4.0 / dt;
  for (int64_t k = 0; k < n_steps; ++k) {
    const auto t0 = std::chrono::steady_clock::now();
    // b = F - K u + C v + M (a + 4/dt v),  C = alpha M + beta K + C_abs
    //   = F + M (a + (4/dt + alpha) v) - K (u - beta v) + C_abs v
#pragma omp parallel for
    for (int64_t j = 0; j < n3; ++j) {
      t1[j] = a[j] + (c1 + alpha) * v[j];
      t2[j] = u[j] - beta * v[j];
      b[j] = v_in[3 * (k + 1)] * S.fb[j] + v_in[3 * (k + 1) + 1] * S.fb[n3 + j] +
             v_in[3 * (k + 1) + 2] * S.fb[2 * n3 + j];
    }
    std::fill(w.begin(), w.end(), 0.0);
    spmv(S, 0.0, 1.0, 0.0, t1.data(), w.data());
    spmv(S, -1.0, 0.0, 0.0, t2.data(), w.data());
    spmv(S, 0.0, 0.0, 1.0, v, w.data());
#pragma omp parallel for
    for (int64_t j = 0; j < n3; ++j) b[j] += w[j];
    const double bn = std::sqrt(dot(b, b));
    if (guess == 0) std::fill(du.begin(), du.end(), 0.0);
    int it = 0;
    double rel = 0.0;
    if (bn == 0.0) {
      std::fill(du.begin(), du.end(), 0.0);
    } else {
      for (;;) {
        // true residual, then CG from the current du
        std::fill(q.begin(), q.end(), 0.0);
        spmv(S, cK, cM, cC, du.data(), q.data());
#pragma omp parallel for
        for (int64_t j = 0; j < n3; ++j) r[j] = b[j] - q[j];
        rel = std::sqrt(dot(r, r)) / bn;
        if (rel <= rtol || it >= max_iter) break;
        double rz = 0.0;
        bool first = true;
        while (it < max_iter) {
#pragma omp parallel for
          for (int64_t i = 0; i < S.n; ++i)
            for (int c = 0; c < 3; ++c)
              z[3 * i + c] = Pinv[9 * i + 3 * c] * r[3 * i] + Pinv[9 * i + 3 * c + 1] * r[3 * i + 1] +
                             Pinv[9 * i + 3 * c + 2] * r[3 * i + 2];
          const double rz_new = dot(r, z);
          if (first) {
            p = z;
            first = false;
          } else {
            const double bet = rz_new / rz;
#pragma omp parallel for
            for (int64_t j = 0; j < n3; ++j) p[j] = z[j] + bet * p[j];
          }
          rz = rz_new;
          std::fill(q.begin(), q.end(), 0.0);
          spmv(S, cK, cM, cC, p.data(), q.data());
          const double al = rz / dot(p, q);
          double rr = 0.0;
#pragma omp parallel for reduction(+ : rr)
          for (int64_t j = 0; j < n3; ++j) {
            du[j] += al * p[j];
            r[j] -= al * q[j];
            rr += r[j] * r[j];
          }
          ++it;
          if (std::sqrt(rr) <= rtol * bn) break;
        }
      }
      if (rel > rtol) return -1;
    }
    // Newmark update
#pragma omp parallel for
    for (int64_t j = 0; j < n3; ++j) {
      const double vn = 2.0 / dt * du[j] - v[j];
      const double an = 4.0 / (dt * dt) * du[j] - c1 * v[j] - a[j];
      u[j] += du[j];
      v[j] = vn;
      a[j] = an;
    }
    for (int32_t s = 0; s < n_rec; ++s)
      for (int c = 0; c < 3; ++c) rec_out[(k * n_rec + s) * 3 + c] = v[3 * (int64_t)rec[s] + c];
    iters[k] = it;
    relres[k] = rel;
    secs[k] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return 0;
}

}  // extern "C"
