"""Element and boundary-face matrices of the quadratic-tetrahedron
discretisation of the linear elastodynamic equation (Section 2, Eq. GE:ORG;
second-order tetrahedral elements, Section 3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Everything is computed by plain numerical quadrature of the textbook
definitions:
    K_e = int B^T D B dV          (isotropic D from lambda, mu)
    M_e = rho int N^T N dV (x) I3
    C_f = int N^T Z N dA,  Z = rho Vp n n^T + rho Vs (I - n n^T)
    F_f = int N^T dA * 2 Z v_in
with conical-product Gauss-Jacobi rules built from
scipy.special.roots_jacobi.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi, roots_legendre

TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))
TRI_EDGES = ((0, 1), (1, 2), (2, 0))


# ------------------------------------------------------------ quadrature

def _gj01(n, alpha):
    """n-point Gauss-Jacobi rule on [0,1] for weight (1-u)^alpha."""
    if alpha == 0:
        x, w = roots_legendre(n)
    else:
        x, w = roots_jacobi(n, alpha, 0.0)
    return (1.0 + x) / 2.0, w / 2.0 ** (alpha + 1)


def tet_rule(n):
    """Conical-product (Stroud) rule on the reference tetrahedron
    {x, y, z >= 0, x + y + z <= 1} with n points per direction; exact for
    polynomials of degree 2n - 1.  Returns barycentric points (m, 4) and
    weights summing to 1/6."""
    u, wu = _gj01(n, 2)
    v, wv = _gj01(n, 1)
    w, ww = _gj01(n, 0)
    U, V, W = np.meshgrid(u, v, w, indexing="ij")
    WU, WV, WW = np.meshgrid(wu, wv, ww, indexing="ij")
    x = U
    y = V * (1 - U)
    z = W * (1 - U) * (1 - V)
    wt = (WU * WV * WW).ravel()
    L = np.stack([1 - x - y - z, x, y, z], -1).reshape(-1, 4)
    return L, wt


def tri_rule(n):
    """Conical-product rule on the reference triangle {x, y >= 0, x + y <= 1},
    exact for degree 2n - 1.  Barycentric points (m, 3), weights sum 1/2."""
    u, wu = _gj01(n, 1)
    v, wv = _gj01(n, 0)
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    x = U
    y = V * (1 - U)
    L = np.stack([1 - x - y, x, y], -1).reshape(-1, 3)
    return L, (WU * WV).ravel()


# ------------------------------------------------------- shape functions

def tet10_shape(L):
    """Quadratic tetrahedron shape functions at barycentric points L (m,4):
    vertices L_i (2 L_i - 1), edges 4 L_a L_b (edge order 01,12,02,03,13,23)."""
    N = np.empty(L.shape[:-1] + (10,))
    for i in range(4):
        N[..., i] = L[..., i] * (2 * L[..., i] - 1)
    for k, (a, b) in enumerate(TET_EDGES):
        N[..., 4 + k] = 4 * L[..., a] * L[..., b]
    return N


def tet10_dshape(L, gradL):
    """Gradients of the ten shape functions.  L: (m,4) barycentric points;
    gradL: (n,4,3) barycentric gradients per tet.  Returns (n,m,10,3)."""
    n, m = gradL.shape[0], L.shape[0]
    G = np.empty((n, m, 10, 3))
    for i in range(4):
        G[:, :, i] = (4 * L[None, :, i, None] - 1) * gradL[:, None, i]
    for k, (a, b) in enumerate(TET_EDGES):
        G[:, :, 4 + k] = 4 * (L[None, :, a, None] * gradL[:, None, b] + L[None, :, b, None] * gradL[:, None, a])
    return G


def tri6_shape(L):
    N = np.empty(L.shape[:-1] + (6,))
    for i in range(3):
        N[..., i] = L[..., i] * (2 * L[..., i] - 1)
    for k, (a, b) in enumerate(TRI_EDGES):
        N[..., 3 + k] = 4 * L[..., a] * L[..., b]
    return N


# ------------------------------------------------------------- geometry

def tet_geometry(X):
    """X: (n,4,3) vertex coordinates.  Returns volume (n,) and barycentric
    gradients (n,4,3) of the affine map."""
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], -1)  # columns
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)           # rows are grad L1..L3
    g = np.empty((X.shape[0], 4, 3))
    g[:, 1:] = Jinv
    g[:, 0] = -Jinv.sum(1)
    return det / 6.0, g


def lame(mat):
    """(Vp, Vs, rho) rows -> (lambda, mu, rho)."""
    vp, vs, rho = mat[:, 0], mat[:, 1], mat[:, 2]
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2 * mu
    return lam, mu, rho


# ------------------------------------------------------ element matrices

def _bmatrix(dN):
    """Voigt strain-displacement matrix: dN (..., 10, 3) -> B (..., 6, 30)
    with strain order (e11, e22, e33, 2e23, 2e13, 2e12)."""
    sh = dN.shape[:-2]
    B = np.zeros(sh + (6, 30))
    for a in range(10):
        dx, dy, dz = dN[..., a, 0], dN[..., a, 1], dN[..., a, 2]
        c = 3 * a
        B[..., 0, c] = dx
        B[..., 1, c + 1] = dy
        B[..., 2, c + 2] = dz
        B[..., 3, c + 1] = dz
        B[..., 3, c + 2] = dy
        B[..., 4, c] = dz
        B[..., 4, c + 2] = dx
        B[..., 5, c] = dy
        B[..., 5, c + 1] = dx
    return B


def _dmatrix(lam, mu):
    n = lam.shape[0]
    D = np.zeros((n, 6, 6))
    for i in range(3):
        for j in range(3):
            D[:, i, j] = lam
        D[:, i, i] += 2 * mu
        D[:, 3 + i, 3 + i] = mu
    return D


def tet_stiffness(X, lam, mu, nq=2):
    """K_e = sum_q w_q |J| B_q^T D B_q, (n,30,30), DOF order 3*node + comp.
    nq points per direction (nq = 2 is exact for affine quadratic tets)."""
    L, w = tet_rule(nq)
    vol, gL = tet_geometry(X)
    dN = tet10_dshape(L, gL)               # (n,m,10,3)
    B = _bmatrix(dN)                       # (n,m,6,30)
    D = _dmatrix(lam, mu)
    DB = np.einsum("nij,nmjk->nmik", D, B)
    K = np.einsum("m,nmji,nmjk->nik", w, B, DB)
    return K * (6.0 * vol)[:, None, None]


def tet_mass(X, rho, nq=3):
    """M_e = rho int N^T N dV (x) I3, (n,30,30)."""
    L, w = tet_rule(nq)
    vol, _ = tet_geometry(X)
    N = tet10_shape(L)                     # (m,10)
    Ms = np.einsum("m,ma,mb->ab", w, N, N)  # reference, |J| = 1
    Mn = (6.0 * vol * rho)[:, None, None] * Ms[None]
    return _kron3(Mn)


def _kron3(S):
    """Scalar (n,k,k) -> (n,3k,3k) with S (x) I3 in node-major DOF order."""
    n, k, _ = S.shape
    out = np.zeros((n, 3 * k, 3 * k))
    for c in range(3):
        out[:, c::3, c::3] = S
    return out


def face_geometry(P):
    """P: (n,3,3) triangle vertices -> area (n,), unit normal (n,3)."""
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    a2 = np.linalg.norm(cr, axis=1)
    return a2 / 2.0, cr / a2[:, None]


def face_impedance(n, vp, vs, rho):
    """Z = rho Vp n n^T + rho Vs (I - n n^T), (m,3,3)."""
    nn = n[:, :, None] * n[:, None, :]
    I = np.eye(3)[None]
    return (rho * vp)[:, None, None] * nn + (rho * vs)[:, None, None] * (I - nn)


def face_dashpot(P, vp, vs, rho, nq=3):
    """C_f = int N^T Z N dA for a 6-node triangle, (n,18,18)."""
    L, w = tri_rule(nq)
    area, nrm = face_geometry(P)
    N = tri6_shape(L)
    Ms = np.einsum("m,ma,mb->ab", w, N, N) * 2.0   # per unit area
    Z = face_impedance(nrm, vp, vs, rho)
    out = np.zeros((P.shape[0], 18, 18))
    for a in range(6):
        for b in range(6):
            out[:, 3 * a:3 * a + 3, 3 * b:3 * b + 3] = (area * Ms[a, b])[:, None, None] * Z
    return out


def face_load_weights(P, nq=3):
    """int N_a dA per face node, (n,6)."""
    L, w = tri_rule(nq)
    area, _ = face_geometry(P)
    N = tri6_shape(L)
    return area[:, None] * (2.0 * np.einsum("m,ma->a", w, N))[None]
