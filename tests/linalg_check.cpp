// C entry points to the host solvers of csrc/sw_linalg.h for the CPU tests in
// tests/test_linalg.py (built there with g++).
#include <vector>

#include "sw_linalg.h"

extern "C" {

// eigen-decomposition of the symmetric n x n matrix a (row-major): v
// (row-major, eigenvectors in columns) and w
void eig(int n, const double* a, double* v, double* w) {
  std::vector<double> A(a, a + (size_t)n * n), V, W;
  sw::sym_eig(n, A, V, W);
  for (size_t i = 0; i < V.size(); ++i) v[i] = V[i];
  for (int i = 0; i < n; ++i) w[i] = W[i];
}

// theta = A^+ h with eigenvalues at or below cut times the largest dropped;
// returns how many were kept
int tsolve(int n, const double* a, const double* h, double* theta, double cut) {
  std::vector<double> A(a, a + (size_t)n * n), V, W;
  sw::sym_eig(n, A, V, W);
  return sw::truncated_solve(n, V, W, h, theta, cut);
}

void psd(int m, const double* g, const double* h, double* theta, double cut) {
  sw::psd_solve(m, g, m, h, theta, cut);
}
}
