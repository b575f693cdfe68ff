"""Pins of the oracle's element and face matrices against closed forms and
invariants of the quadratic-tetrahedron discretisation (second-order
tetrahedral elements, Section 3; linear elastic body, Eq. GE:ORG)."""
import math
from itertools import product

import numpy as np
import pytest

from oracle import fem


def _rand_tets(n, seed=0):
    """Random well-shaped tets: a perturbed unit right tet, randomly
    rotated, scaled and shifted."""
    rng = np.random.default_rng(seed)
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    X = ref[None] + 0.25 * rng.uniform(-1, 1, (n, 4, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    X = np.einsum("nij,nkj->nki", Q, X) * rng.uniform(0.5, 20, (n, 1, 1)) + rng.standard_normal((n, 1, 3))
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], -1)
    bad = np.linalg.det(J) < 0
    X[bad, 1], X[bad, 2] = X[bad, 2].copy(), X[bad, 1].copy()
    return X


# ------------------------------------------------------------ quadrature

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_tet_rule_exact_monomials(n):
    # int_ref x^a y^b z^c = a! b! c! / (a+b+c+3)!
    L, w = fem.tet_rule(n)
    x, y, z = L[:, 1], L[:, 2], L[:, 3]
    for a, b, c in product(range(2 * n), repeat=3):
        if a + b + c > 2 * n - 1:
            continue
        exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        assert abs(np.sum(w * x ** a * y ** b * z ** c) - exact) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tri_rule_exact_monomials(n):
    L, w = fem.tri_rule(n)
    x, y = L[:, 1], L[:, 2]
    for a, b in product(range(2 * n), repeat=2):
        if a + b > 2 * n - 1:
            continue
        exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
        assert abs(np.sum(w * x ** a * y ** b) - exact) < 1e-14


# ------------------------------------------------------------ mass

def _bary_integral(powers, vol, dim=3):
    """int prod L_i^{p_i} over a simplex of measure vol:
    dim! vol prod p_i! / (sum p + dim)!"""
    num = math.factorial(dim) * vol
    for p in powers:
        num *= math.factorial(p)
    return num / math.factorial(sum(powers) + dim)


def _poly_shape(nv, edges):
    """Shape functions as dicts {power tuple: coeff} in barycentric L."""
    out = []
    for i in range(nv):
        p2 = [0] * nv
        p2[i] = 2
        p1 = [0] * nv
        p1[i] = 1
        out.append({tuple(p2): 2.0, tuple(p1): -1.0})
    for a, b in edges:
        p = [0] * nv
        p[a] += 1
        p[b] += 1
        out.append({tuple(p): 4.0})
    return out


def _closed_form_mass(nv, edges, vol):
    N = _poly_shape(nv, edges)
    k = len(N)
    Mm = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            s = 0.0
            for pi, ci in N[i].items():
                for pj, cj in N[j].items():
                    s += ci * cj * _bary_integral([x + y for x, y in zip(pi, pj)], vol, nv - 1)
            Mm[i, j] = s
    return Mm


def test_tet_mass_closed_form():
    X = _rand_tets(5)
    rho = np.array([1.3, 2.0, 1800.0, 0.5, 7.0])
    M = fem.tet_mass(X, rho)
    vol, _ = fem.tet_geometry(X)
    for e in range(5):
        ref = rho[e] * _closed_form_mass(4, fem.TET_EDGES, vol[e])
        np.testing.assert_allclose(M[e][0::3, 0::3], ref, rtol=1e-13, atol=1e-14 * abs(ref).max())
        # the table rho V / 420 x {6, 1, -4, -6, 32, 16, 8}
        t = ref * 420 / (rho[e] * vol[e])
        assert np.allclose(np.diag(t)[:4], 6) and np.allclose(np.diag(t)[4:], 32)
        assert np.isclose(t[0, 1], 1) and np.isclose(t[0, 4], -4) and np.isclose(t[0, 5], -6)
        assert np.isclose(t[4, 5], 16) and np.isclose(t[4, 9], 8)
        rows = ref.sum(1) / (rho[e] * vol[e])
        np.testing.assert_allclose(rows[:4], -1 / 20, rtol=1e-12)
        np.testing.assert_allclose(rows[4:], 1 / 5, rtol=1e-12)
        # components decouple
        assert np.all(M[e][0::3, 1::3] == 0)


def test_face_mass_and_load_closed_form():
    rng = np.random.default_rng(3)
    P = rng.standard_normal((4, 3, 3))
    area, n = fem.face_geometry(P)
    vp, vs, rho = np.full(4, 3.0), np.full(4, 1.0), np.full(4, 2.0)
    C = fem.face_dashpot(P, vp, vs, rho)
    w = fem.face_load_weights(P)
    for f in range(4):
        ref = _closed_form_mass(3, fem.TRI_EDGES, area[f])
        t = ref * 180 / area[f]
        assert np.allclose(np.diag(t)[:3], 6) and np.allclose(np.diag(t)[3:], 32)
        assert np.isclose(t[0, 1], -1) and np.isclose(t[0, 3], 0) and np.isclose(t[0, 4], -4)
        assert np.isclose(t[3, 4], 16)
        Z = rho[f] * vp[f] * np.outer(n[f], n[f]) + rho[f] * vs[f] * (np.eye(3) - np.outer(n[f], n[f]))
        np.testing.assert_allclose(C[f], np.kron(ref, Z), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(w[f], [0, 0, 0, area[f] / 3, area[f] / 3, area[f] / 3], atol=1e-14)


# ------------------------------------------------------------ stiffness

def test_tet_stiffness_invariants():
    X = _rand_tets(6, seed=1)
    lam = np.array([1.0, 2.0, 100.0, 0.0, 3.0, 5e9])
    mu = np.array([1.0, 0.5, 1.0, 2.0, 7.0, 4e8])
    K2 = fem.tet_stiffness(X, lam, mu, nq=2)
    K4 = fem.tet_stiffness(X, lam, mu, nq=4)
    for e in range(6):
        s = np.abs(K2[e]).max()
        np.testing.assert_allclose(K2[e], K4[e], atol=1e-12 * s)
        np.testing.assert_allclose(K2[e], K2[e].T, atol=1e-13 * s)
        ev = np.linalg.eigvalsh(K2[e])
        assert np.all(ev[:6] < 1e-11 * ev[-1]) and np.all(np.abs(ev[:6]) < 1e-11 * ev[-1])
        assert ev[6] > 1e-6 * ev[-1]
        # rigid body modes: translations and rotations w x x at all 10 nodes
        nodes = np.concatenate([X[e], np.array([(X[e][a] + X[e][b]) / 2 for a, b in fem.TET_EDGES])])
        for c in range(3):
            r = np.zeros(30)
            r[c::3] = 1
            assert np.abs(K2[e] @ r).max() < 1e-12 * s
            om = np.eye(3)[c]
            r = np.cross(om[None], nodes).ravel()
            assert np.abs(K2[e] @ r).max() < 1e-12 * s * np.abs(nodes).max()


def test_tet_stiffness_linear_field_energy():
    # For u = G x, the strain energy 1/2 u^T K u equals V (lam/2 tr(e)^2 + mu e:e).
    X = _rand_tets(4, seed=2)
    rng = np.random.default_rng(5)
    lam = np.array([3.0, 0.7, 11.0, 2.0])
    mu = np.array([1.5, 2.5, 0.3, 1.0])
    K = fem.tet_stiffness(X, lam, mu)
    vol, _ = fem.tet_geometry(X)
    for e in range(4):
        G = rng.standard_normal((3, 3))
        eps = 0.5 * (G + G.T)
        nodes = np.concatenate([X[e], np.array([(X[e][a] + X[e][b]) / 2 for a, b in fem.TET_EDGES])])
        u = (nodes @ G.T).ravel()
        W = 0.5 * u @ K[e] @ u
        ref = vol[e] * (0.5 * lam[e] * np.trace(eps) ** 2 + mu[e] * np.sum(eps * eps))
        assert abs(W - ref) < 1e-12 * abs(ref)


def test_tet_stiffness_affine_invariance():
    # K_e depends on geometry only through the map; scaling lengths by s
    # scales K_e by s (3D elasticity: K ~ mu * L).
    X = _rand_tets(2, seed=9)
    lam, mu = np.array([1.0, 2.0]), np.array([3.0, 4.0])
    K = fem.tet_stiffness(X, lam, mu)
    K2 = fem.tet_stiffness(2.5 * X + 7.0, lam, mu)
    np.testing.assert_allclose(K2, 2.5 * K, rtol=1e-12, atol=1e-12 * np.abs(K).max())
