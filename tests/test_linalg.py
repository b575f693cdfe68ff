"""The host solvers of csrc/sw_linalg.h on the CPU (built with g++), against
numpy: the Jacobi eigen-decomposition reproduces the matrix with orthonormal
eigenvectors and numpy's eigenvalues; the truncated solve keeps exactly the
eigenvalues above the cut and equals the truncated pseudo-inverse formed
from a known spectral decomposition; the Gram solve of the projection guess
gives the least-squares projection onto the span of nearly or exactly
dependent vectors."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2404_17754_amd", "csrc")
P = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("linalg") / "liblinalg_check.so"
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, os.path.join(HERE, "linalg_check.cpp"),
                    "-o", str(out)], check=True)
    lib = C.CDLL(str(out))
    lib.tsolve.restype = C.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(P)


def _orthogonal(n, rng):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q


def test_eigen_decomposition(lib):
    rng = np.random.default_rng(3)
    for n in (1, 2, 6, 18):
        a = rng.standard_normal((n, n))
        a = a + a.T
        v = np.zeros((n, n))
        w = np.zeros(n)
        lib.eig(n, _p(np.ascontiguousarray(a)), _p(v), _p(w))
        assert np.allclose(v @ np.diag(w) @ v.T, a, rtol=0, atol=1e-12 * np.abs(a).max())
        assert np.allclose(v.T @ v, np.eye(n), atol=1e-13)
        assert np.allclose(np.sort(w), np.linalg.eigvalsh(a), atol=1e-12 * np.abs(a).max())


def test_truncated_solve_against_known_spectrum(lib):
    rng = np.random.default_rng(5)
    n = 12
    q = _orthogonal(n, rng)
    lam = 10.0 ** -np.arange(n, dtype=float) * 2.0     # 2, 0.2, ..., 2e-11
    a = (q * lam) @ q.T
    h = rng.standard_normal(n)
    for cut in (1e-3, 1e-7, 1e-16):
        theta = np.zeros(n)
        kept = lib.tsolve(n, _p(np.ascontiguousarray(a)), _p(h), _p(theta), C.c_double(cut))
        keep = lam > cut * lam.max()
        assert kept == int(keep.sum())
        want = (q[:, keep] / lam[keep]) @ (q[:, keep].T @ h)
        # rounding of the decomposition: about eps times the condition
        # number of the kept spectrum (measured 0.2 of it)
        kappa = lam.max() / lam[keep].min()
        err = np.linalg.norm(theta - want) / np.linalg.norm(want)
        assert err <= 4 * np.finfo(float).eps * kappa + 1e-15, (cut, err)
    z = np.zeros(n)
    zero = np.zeros((n, n))
    assert lib.tsolve(n, _p(zero), _p(h), _p(z), C.c_double(1e-16)) == 0 and not z.any()


def _ring(noise, dependent, seed=11):
    """Columns of very different scales that differ by small smooth changes
    plus noise (the ring of a smooth march), optionally one repeated."""
    rng = np.random.default_rng(seed)
    n, m = 400, 6
    base = rng.standard_normal((n, 2))
    x = np.stack([base[:, 0] * (1 + 0.01 * k) + base[:, 1] * 1e-3 * k ** 2 + noise * rng.standard_normal(n)
                  for k in range(m)], axis=1) * (10.0 ** np.arange(m))[None, :]
    if dependent:
        x[:, 3] = x[:, 1]
    return x, rng.standard_normal(n)


def _gram_solve(lib, x, b):
    m = x.shape[1]
    theta = np.zeros(m)
    lib.psd(m, _p(np.ascontiguousarray(x.T @ x)), _p(x.T @ b), _p(theta), C.c_double(1e-16))
    assert np.all(np.isfinite(theta))
    return theta


@pytest.mark.parametrize("dependent", [False, True])
def test_gram_solve_projects_onto_the_span(lib, dependent):
    """X theta from the Gram system X^T X theta = X^T b is the least-squares
    projection of b onto span(X) (scaled Gram condition number 6e6, or
    singular with a repeated column)."""
    x, b = _ring(1e-3, dependent)
    want = x @ np.linalg.lstsq(x, b, rcond=None)[0]
    err = np.linalg.norm(x @ _gram_solve(lib, x, b) - want) / np.linalg.norm(want)
    assert err <= 1e-8, err


@pytest.mark.parametrize("dependent", [False, True])
def test_gram_solve_near_optimal_when_ill_conditioned(lib, dependent):
    """With nearly dependent columns (scaled Gram condition number 6e12) the
    coefficients carry the Gram system's rounding, but the residual of the
    projection stays optimal to first order: its norm exceeds the
    least-squares residual by under 1e-7 relative."""
    x, b = _ring(1e-6, dependent)
    r_opt = np.linalg.norm(b - x @ np.linalg.lstsq(x, b, rcond=None)[0])
    r = np.linalg.norm(b - x @ _gram_solve(lib, x, b))
    assert r <= r_opt * (1 + 1e-7), r / r_opt - 1
