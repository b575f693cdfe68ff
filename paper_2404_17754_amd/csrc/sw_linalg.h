// Small dense symmetric solves on the host: the Gram system of the
// projection guess and the normal equations of the input estimation (a few
// dozen unknowns at most).  Header-only, so that a CPU test can build them
// without the device code.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace sw {

// Eigen-decomposition of a symmetric n x n matrix (row-major, destroyed) by
// cyclic Jacobi rotations: A = V diag(w) V^T, V row-major with eigenvectors
// in its columns.
inline void sym_eig(int n, std::vector<double>& A, std::vector<double>& V, std::vector<double>& w) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  auto v = [&](int i, int j) -> double& { return V[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        // rotation in the (p, q) plane that zeroes a(p, q)
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        a(p, p) -= t * apq;
        a(q, q) += t * apq;
        a(p, q) = a(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          if (r != p && r != q) {
            const double arp = a(r, p), arq = a(r, q);
            a(r, p) = a(p, r) = cs * arp - sn * arq;
            a(r, q) = a(q, r) = sn * arp + cs * arq;
          }
          const double vrp = v(r, p), vrq = v(r, q);
          v(r, p) = cs * vrp - sn * vrq;
          v(r, q) = sn * vrp + cs * vrq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a(i, i);
}

// theta = V W^+ V^T h for A = V diag(w) V^T, eigenvalues at or below
// rel_cut times the largest dropped; returns how many were kept.
inline int truncated_solve(int n, const std::vector<double>& V, const std::vector<double>& w, const double* h,
                    double* theta, double rel_cut) {
  double wmax = 0.0;
  for (int i = 0; i < n; ++i) wmax = std::max(wmax, w[i]);
  std::vector<double> y(n, 0.0);
  int kept = 0;
  for (int k = 0; k < n; ++k) {
    if (!(wmax > 0.0 && w[k] > rel_cut * wmax)) continue;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += V[(size_t)i * n + k] * h[i];
    y[k] = acc / w[k];
    ++kept;
  }
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += V[(size_t)i * n + k] * y[k];
    theta[i] = acc;
  }
  return kept;
}

// Solves G theta = h for a symmetric positive semidefinite G (leading
// dimension ldg) in the least-squares sense, on the unit-diagonal scaling
// D G D (D = diag(G)^-1/2) truncated at rel_cut: theta = D (D G D)^+ D h.
inline void psd_solve(int m, const double* G, int ldg, const double* h, double* theta, double rel_cut) {
  std::vector<double> d(m), A((size_t)m * m), V, w, hs(m), ts(m);
  for (int i = 0; i < m; ++i) {
    const double gi = G[i * ldg + i];
    d[i] = gi > 0.0 ? 1.0 / std::sqrt(gi) : 0.0;
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = d[i] * 0.5 * (G[i * ldg + j] + G[j * ldg + i]) * d[j];
  sym_eig(m, A, V, w);
  for (int i = 0; i < m; ++i) hs[i] = d[i] * h[i];
  truncated_solve(m, V, w, hs.data(), ts.data(), rel_cut);
  for (int i = 0; i < m; ++i) theta[i] = d[i] * ts[i];
}

}  // namespace sw
