"""Pins of the oracle's assembled system and Newmark time march against
invariants and exact solutions: rigid-body null space and the patch test of
the discretised Eq. GE:ORG, the exact energy identity of the Newmark
average-acceleration scheme (Section 3), exact modal solutions, linearity,
and the closed forms of the inputs (Ricker wavelet, Rayleigh damping)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import casegen as cg
from oracle import assemble, march


def _rigid_modes(xyz):
    n = xyz.shape[0]
    R = []
    for c in range(3):
        r = np.zeros((n, 3))
        r[:, c] = 1
        R.append(r.ravel())
        om = np.eye(3)[c]
        R.append(np.cross(om[None], xyz).ravel())
    return R


def _graded_mesh():
    return cg.box_mesh(40.0, 30.0, 30.0, 10.0, jitter=0.15, seed=9, z_levels=cg.graded_levels(30.0, 2.5, 1.6))


def _delaunay_mesh():
    # unstructured: Delaunay tetrahedra refined towards a 15 m deep interface
    return cg.delaunay_mesh(40.0, 30.0, 30.0, 15.0, 2.5, 10.0, seed=4)


def _mesh(which, small_mesh, jitter_mesh):
    if which == "small":
        return small_mesh
    if which == "jitter":
        return jitter_mesh
    return _graded_mesh() if which == "graded" else _delaunay_mesh()


@pytest.mark.parametrize("which", ["small", "jitter", "graded", "delaunay"])
def test_global_stiffness_rigid_modes(which, small_mesh, small_case, jitter_mesh):
    mesh = _mesh(which, small_mesh, jitter_mesh)
    tet_mat = small_case.tet_mat if which == "small" else (np.arange(mesh.n_tets) % 2).astype(np.uint8)
    K, M = assemble.stiffness_and_mass(mesh, cg.material_table(), tet_mat)
    kn = abs(K).sum(1).max()
    for r in _rigid_modes(mesh.xyz):
        assert np.linalg.norm(K @ r) / (kn * np.linalg.norm(r)) < 1e-13
    # M: total mass of each translation = rho V summed
    mat = cg.material_table()
    X = mesh.xyz[mesh.tet10[:, :4]]
    V = np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], -1)) / 6
    t = np.zeros(3 * mesh.n_nodes)
    t[0::3] = 1
    assert abs(t @ M @ t - np.sum(V * mat[tet_mat, 2])) < 1e-12 * np.sum(V * mat[tet_mat, 2])


@pytest.mark.parametrize("which", ["jitter", "graded", "delaunay"])
def test_patch_test_linear_field(which, jitter_mesh):
    # one material: a linear displacement then has uniform stress, so the
    # interior nodal forces vanish and the interior solution is exact
    mesh = _mesh(which, None, jitter_mesh)
    tet_mat = np.zeros(mesh.n_tets, np.uint8)
    K, _ = assemble.stiffness_and_mass(mesh, cg.material_table(), tet_mat)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((3, 3)) * 1e-3
    c = rng.standard_normal(3)
    ulin = (mesh.xyz @ G.T + c).ravel()
    x = mesh.xyz
    Lx, Ly, Lz = mesh.box
    tol = 1e-9
    bnd = (np.abs(x[:, 0]) < tol) | (np.abs(x[:, 0] - Lx) < tol) | (np.abs(x[:, 1]) < tol) | \
          (np.abs(x[:, 1] - Ly) < tol) | (np.abs(x[:, 2] + Lz) < tol) | (np.abs(x[:, 2]) < tol)
    assert (~bnd).sum() > 10
    bd = assemble.node_dofs(np.nonzero(bnd)[0])
    idd = assemble.node_dofs(np.nonzero(~bnd)[0])
    Ku = K @ ulin
    assert np.abs(Ku[idd]).max() < 1e-12 * abs(K).max() * np.abs(ulin).max()
    import scipy.sparse.linalg as spla
    ui = spla.spsolve(K[idd][:, idd].tocsc(), -K[idd][:, bd] @ ulin[bd])
    assert np.abs(ui - ulin[idd]).max() < 1e-12 * np.abs(ulin).max()


@pytest.fixture(scope="module")
def tiny():
    mesh = cg.box_mesh(40.0, 30.0, 20.0, 10.0)
    cfg = cg.CONFIGS["small"]
    case = cg.make_case(mesh, cfg, n_steps=200, n_rec=1)
    return mesh, case


def _energy(sys, u, v):
    return 0.5 * v @ (sys.M @ v) + 0.5 * u @ (sys.K @ u)


def test_energy_conserved_without_damping(tiny):
    mesh, case = tiny
    sys = march.build_system(mesh, case, damping=False, dashpot_roles=(), input_force=False)
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(sys.K.shape[0]) * 1e-3
    v0 = rng.standard_normal(sys.K.shape[0]) * 1e-2
    a0 = march.consistent_acceleration(sys, u0, v0, np.zeros_like(u0))
    r = march.run(sys, case.dt, np.zeros((201, 3)), 200, case.rec_node, u0, v0, a0, keep_states=True)
    E = np.array([_energy(sys, u, v) for u, v, _ in r.states])
    assert np.abs(E - E[0]).max() < 1e-12 * E[0]


def test_energy_identity_with_damping_dashpots_and_input(tiny):
    # E^{n+1} - E^n = 1/2 (u^{n+1}-u^n)^T (F^{n+1}+F^n) - dt/4 vb^T C vb,
    # vb = v^{n+1} + v^n, E = 1/2 v^T M v + 1/2 u^T K u.
    mesh, case = tiny
    sys = march.build_system(mesh, case)
    n = 120
    F0 = case.v_in[0] @ sys.Fb
    a0 = march.consistent_acceleration(sys, np.zeros(sys.K.shape[0]), np.zeros(sys.K.shape[0]), F0)
    r = march.run(sys, case.dt, case.v_in, n, case.rec_node, a0=a0, keep_states=True)
    C = sys.C
    scale = max(_energy(sys, u, v) for u, v, _ in r.states)
    for k in range(n):
        u0, v0, _ = r.states[k]
        u1, v1, _ = r.states[k + 1]
        F0 = case.v_in[k] @ sys.Fb
        F1 = case.v_in[k + 1] @ sys.Fb
        vb = v1 + v0
        lhs = _energy(sys, u1, v1) - _energy(sys, u0, v0)
        rhs = 0.5 * (u1 - u0) @ (F1 + F0) - case.dt / 4 * vb @ (C @ vb)
        assert abs(lhs - rhs) < 1e-11 * scale
    assert scale > 0


def _modes(sys, k):
    w2, phi = sla.eigh(sys.K.toarray(), sys.M.toarray())
    return w2[k], phi[:, k]


def test_modal_exactness_undamped(tiny):
    # u^n = phi cos(n Om), tan(Om/2) = w dt / 2 (trapezoidal rule)
    mesh, case = tiny
    sys = march.build_system(mesh, case, damping=False, dashpot_roles=(), input_force=False)
    w2, phi = _modes(sys, 20)
    w = math.sqrt(w2)
    dt = case.dt
    r = march.run(sys, dt, np.zeros((101, 3)), 100, case.rec_node, phi, 0 * phi, -w2 * phi, keep_states=True)
    Om = 2 * math.atan(w * dt / 2)
    for n_, (u, v, _) in enumerate(r.states):
        assert np.abs(u - phi * math.cos(n_ * Om)).max() < 1e-10 * np.abs(phi).max()
        assert np.abs(v + w * phi * math.sin(n_ * Om)).max() < 1e-10 * w * np.abs(phi).max()


def test_modal_exactness_rayleigh_damped(tiny):
    # Mode phi with modal damping 2 xi w = alpha + beta w^2; trapezoidal
    # amplification lambda_k = (1 + dt mu_k / 2) / (1 - dt mu_k / 2),
    # mu_k the roots of mu^2 + (alpha + beta w^2) mu + w^2 = 0.
    mesh, case = tiny
    sys = march.build_system(mesh, case, damping=True, dashpot_roles=(), input_force=False)
    w2, phi = _modes(sys, 30)
    c = case.ray_alpha + case.ray_beta * w2
    mu = np.roots([1.0, c, w2]).astype(complex)
    lam = (1 + case.dt * mu / 2) / (1 - case.dt * mu / 2)
    c1 = mu[1] / (mu[1] - mu[0])
    c2 = -mu[0] / (mu[1] - mu[0])
    a0 = march.consistent_acceleration(sys, phi, 0 * phi, 0 * phi)
    r = march.run(sys, case.dt, np.zeros((81, 3)), 80, case.rec_node, phi, 0 * phi, a0, keep_states=True)
    for n_, (u, _, _) in enumerate(r.states):
        q = (c1 * lam[0] ** n_ + c2 * lam[1] ** n_).real
        assert np.abs(u - q * phi).max() < 1e-10 * np.abs(phi).max()


def test_linearity(tiny):
    mesh, case = tiny
    sys = march.build_system(mesh, case)
    rng = np.random.default_rng(4)
    f1 = rng.standard_normal((41, 3))
    f2 = rng.standard_normal((41, 3))
    r1 = march.run(sys, case.dt, f1, 40, case.rec_node)
    r2 = march.run(sys, case.dt, f2, 40, case.rec_node)
    r3 = march.run(sys, case.dt, 2.0 * f1 - 0.5 * f2, 40, case.rec_node)
    ref = 2.0 * r1.rec_v - 0.5 * r2.rec_v
    assert np.abs(r3.rec_v - ref).max() < 1e-12 * np.abs(ref).max()


def test_cg_solver_matches_lu(small_mesh, small_case):
    r1 = march.run_case(small_mesh, small_case, n_steps=10, solver="lu")
    r2 = march.run_case(small_mesh, small_case, n_steps=10, solver="cg", rtol=1e-12)
    assert np.linalg.norm(r2.rec_v - r1.rec_v) < 1e-9 * np.linalg.norm(r1.rec_v)


# ------------------------------------------------------------ inputs

def test_ricker_closed_form():
    fp, t0 = 2.0, 0.5
    assert cg.ricker(t0, fp, t0) == 1.0
    z = 1 / (math.pi * fp * math.sqrt(2))
    assert abs(cg.ricker(t0 + z, fp, t0)) < 1e-15 and abs(cg.ricker(t0 - z, fp, t0)) < 1e-15
    # minimum at tau^2 = 3 / (2 pi^2 f^2) with value -2 exp(-3/2)
    tm = t0 + math.sqrt(1.5) / (math.pi * fp)
    assert abs(cg.ricker(tm, fp, t0) + 2 * math.exp(-1.5)) < 1e-15


def test_rayleigh_closed_form():
    a, b = cg.rayleigh_coefficients(0.02, 1.0, 5.0)
    assert abs(a - math.pi / 15) < 1e-15 and abs(b - 1 / (300 * math.pi)) < 1e-18
    for f in (1.0, 5.0):
        w = 2 * math.pi * f
        assert abs(a / (2 * w) + b * w / 2 - 0.02) < 1e-15


def test_mesh_counts_match_config_sizes():
    # nodes = (2nx+1)(2ny+1)(2nz+1), tets = 6 nx ny nz, boundary faces 2 per cell face
    m = cg.config_mesh(cg.CONFIGS["small"])
    assert (m.n_nodes, m.n_tets, m.n_faces) == (4851, 3000, 600)
    assert np.bincount(m.face_role).tolist() == [0, 400, 200]


def test_delaunay_mesh_is_a_conforming_partition():
    """The unstructured generator's output: positive volumes summing to the
    box, edge nodes at midpoints, every interior face shared by exactly two
    elements and every other face on the sides, base (with faces listed) or
    top; element sizes vary several fold."""
    m = _delaunay_mesh()
    Lx, Ly, Lz = m.box
    X = m.xyz[m.tet10[:, :4]]
    V = np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])) / 6
    assert V.min() > 0 and abs(V.sum() - Lx * Ly * Lz) < 1e-9 * Lx * Ly * Lz
    for k, (a, b) in enumerate(cg.TET_EDGES):
        assert np.abs(m.xyz[m.tet10[:, 4 + k]] - 0.5 * (X[:, a] + X[:, b])).max() < 1e-12
    faces = np.sort(np.concatenate([m.tet10[:, list(v)] for v in ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))]), 1)
    u, cnt = np.unique(faces, axis=0, return_counts=True)
    assert cnt.max() == 2
    P = m.xyz[u[cnt == 1]]
    top = np.all(np.abs(P[..., 2]) < 1e-9, 1)
    assert (cnt == 1).sum() - top.sum() == m.n_faces
    assert set(np.unique(m.face_role)) == {1, 2}
    h = np.cbrt(6 * V)
    assert h.max() / h.min() > 4
