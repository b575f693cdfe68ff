"""Pins of the oracle guesses (oracle/guess.py) against what their
definitions fix: extrapolation is exact on polynomials of its order; the
Galerkin projection reproduces a solution that lies in the span, satisfies
Galerkin orthogonality X^T (b - A x0) = 0, minimises the energy-norm error
over the span (no random combination does better), and ignores a
duplicated column."""
import numpy as np
import scipy.sparse as sp

from oracle import guess


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    B = sp.random(n, n, density=0.05, random_state=seed) + sp.eye(n)
    return (B @ B.T + sp.eye(n) * 0.5).tocsr(), rng


def test_extrapolation_exact_on_polynomials():
    for p in range(4):
        t = np.arange(8, dtype=float)
        hist = [np.array([tt ** p, 1.0 + 2 * tt ** p]) for tt in t[:-1]]
        nxt = np.array([t[-1] ** p, 1.0 + 2 * t[-1] ** p])
        np.testing.assert_allclose(guess.extrapolation(hist, p), nxt, rtol=1e-12)
    # quadratic extrapolation misses a cubic by the third difference
    hist = [np.array([float(k) ** 3]) for k in range(4)]
    assert abs(guess.extrapolation(hist, 2)[0] - 4.0 ** 3) == 6.0


def test_projection_reproduces_solution_in_span():
    A, rng = _spd(200, 1)
    X = rng.standard_normal((200, 5))
    c = rng.standard_normal(5)
    x_true = X @ c
    x0 = guess.projection(A, X, A @ x_true)
    assert np.linalg.norm(x0 - x_true) <= 1e-10 * np.linalg.norm(x_true)


def test_projection_galerkin_orthogonality_and_optimality():
    A, rng = _spd(300, 2)
    X = rng.standard_normal((300, 6))
    b = rng.standard_normal(300)
    x0 = guess.projection(A, X, b)
    r = b - A @ x0
    assert np.abs(X.T @ r).max() <= 1e-10 * np.abs(X.T @ b).max()
    x_star = np.linalg.solve(A.toarray(), b)
    e0 = x_star - x0
    best = e0 @ (A @ e0)
    for k in range(50):
        y = x0 + X @ (0.1 * rng.standard_normal(6))
        e = x_star - y
        assert e @ (A @ e) >= best * (1 - 1e-12)


def test_projection_ignores_dependent_columns():
    A, rng = _spd(150, 3)
    X = rng.standard_normal((150, 3))
    Xd = np.column_stack([X, X[:, 0] * 2.0])   # a repeated direction
    b = rng.standard_normal(150)
    np.testing.assert_allclose(guess.projection(A, Xd, b), guess.projection(A, X, b), rtol=1e-8, atol=1e-12)
