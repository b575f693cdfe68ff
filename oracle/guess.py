"""Initial guesses of the time-step solves, written from their definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A guess changes where each step's CG starts, never the converged result, so
the oracle of the march (march.py) does not use these; they pin the GPU
guesses themselves.

* Lagrange extrapolation of order p from the last p + 1 increments
  (du^{n-1} newest): x0 = sum_j (-1)^j C(p+1, j+1) du^{n-1-j}.
* Galerkin projection onto the span of the last L increments X (columns):
  the combination closest to the step's solution in the energy norm,
      x0 = X theta,  (X^T A X) theta = X^T b,
  taken in the least-squares sense when X^T A X is singular (Fischer,
  projection techniques for successive right-hand sides, Comput. Methods
  Appl. Mech. Engrg. 163 (1998)).  Directions of the span that A cannot
  tell apart from zero above `rel_cut` of the largest (after scaling the
  columns to unit energy) are dropped.
"""
from __future__ import annotations

from math import comb

import numpy as np


def extrapolation(history, order):
    """history: increments, newest last.  Returns the order-p extrapolation."""
    p = min(order, len(history) - 1)
    if p < 0:
        raise ValueError("no history")
    return sum((-1) ** j * comb(p + 1, j + 1) * history[-1 - j] for j in range(p + 1))


def projection(A, X, b, rel_cut=1e-16):
    """Galerkin projection of A^-1 b onto span(X): A symmetric positive
    definite (dense or sparse), X (n, L), b (n,)."""
    X = np.asarray(X, float)
    AX = A @ X
    G = X.T @ AX
    G = 0.5 * (G + G.T)
    h = X.T @ b
    d = np.sqrt(np.clip(np.diag(G), 0.0, None))
    s = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    w, V = np.linalg.eigh(s[:, None] * G * s[None, :])
    keep = w > rel_cut * w.max()
    theta = s * (V[:, keep] @ ((V[:, keep].T @ (s * h)) / w[keep]))
    return X @ theta
