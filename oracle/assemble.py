"""Global sparse matrices of the semi-discrete system
M u'' + (alpha M + beta K + C_abs) u' + K u = F(t)
on a quadratic-tetrahedron mesh (Section 2, Eq. GE:ORG, with the absorbing
sides and base of Sections 2-3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

DOF numbering: 3 * node + component.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def _dofs(conn):
    return (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(conn.shape[0], -1)


def _coo_add(rows, cols, vals, n):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def element_matrices(mesh, mat, tet_mat, tets=None):
    """K_e, M_e for the selected tets (all by default)."""
    tets = np.arange(mesh.n_tets) if tets is None else np.asarray(tets)
    conn = mesh.tet10[tets]
    X = mesh.xyz[conn[:, :4]]
    lam, mu, rho = fem.lame(mat)
    m = tet_mat[tets]
    return fem.tet_stiffness(X, lam[m], mu[m]), fem.tet_mass(X, rho[m])


def stiffness_and_mass(mesh, mat, tet_mat, chunk=8192):
    """Assembled K and M (CSR, FP64)."""
    n = 3 * mesh.n_nodes
    K = sp.csr_matrix((n, n))
    M = sp.csr_matrix((n, n))
    for s in range(0, mesh.n_tets, chunk):
        t = np.arange(s, min(s + chunk, mesh.n_tets))
        Ke, Me = element_matrices(mesh, mat, tet_mat, t)
        d = _dofs(mesh.tet10[t])
        r = np.repeat(d[:, :, None], 30, 2)
        c = np.repeat(d[:, None, :], 30, 1)
        K = K + _coo_add(r, c, Ke, n)
        M = M + _coo_add(r, c, Me, n)
    return K, M


def face_materials(mesh, mat, tet_mat):
    m = tet_mat[mesh.face_tet]
    return mat[m, 0], mat[m, 1], mat[m, 2]


def dashpots(mesh, mat, tet_mat, roles=(1, 2)):
    """Lysmer dashpot matrix C_abs assembled over faces whose role is in
    ``roles`` (1 = sides, 2 = base); the material is the owning tet's."""
    n = 3 * mesh.n_nodes
    sel = np.isin(mesh.face_role, roles)
    if not np.any(sel):
        return sp.csr_matrix((n, n))
    tri = mesh.tri6[sel]
    vp, vs, rho = (a[sel] for a in face_materials(mesh, mat, tet_mat))
    Cf = fem.face_dashpot(mesh.xyz[tri[:, :3]], vp, vs, rho)
    d = _dofs(tri)
    r = np.repeat(d[:, :, None], 18, 2)
    c = np.repeat(d[:, None, :], 18, 1)
    return _coo_add(r, c, Cf, n)


def input_force_basis(mesh, mat, tet_mat):
    """(3, n_dof) array B such that the base input force at time t is
    F(t) = sum_c v_in,c(t) B[c]: the incident wave enters through the base
    faces as the traction 2 Z v_in, Z = rho Vp n n^T + rho Vs (I - n n^T)."""
    n = 3 * mesh.n_nodes
    out = np.zeros((3, n))
    sel = mesh.face_role == 2
    tri = mesh.tri6[sel]
    if tri.shape[0] == 0:
        return out
    vp, vs, rho = (a[sel] for a in face_materials(mesh, mat, tet_mat))
    P = mesh.xyz[tri[:, :3]]
    w = fem.face_load_weights(P)            # (f,6)
    _, nrm = fem.face_geometry(P)
    Z = fem.face_impedance(nrm, vp, vs, rho)  # (f,3,3)
    for c in range(3):
        t = 2.0 * Z[:, :, c]                # traction per unit v_in,c  (f,3)
        vals = w[:, :, None] * t[:, None, :]  # (f,6,3)
        np.add.at(out[c], (3 * tri[:, :, None] + np.arange(3)).ravel(), vals.ravel())
    return out


def node_dofs(nodes):
    nodes = np.asarray(nodes)
    return (3 * nodes[:, None] + np.arange(3)[None]).ravel()
