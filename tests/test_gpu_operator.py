"""GPU parity of the matrix-free operator, the right-hand side, the
block-Jacobi diagonal and the misfit against the CPU oracle (through the
C-ABI).  Meshes: the small two-layer box (3000 tets: 11 full workgroups of
256 tets plus a ragged tail), a jittered mesh (no lattice left in the
geometry), a jittered mesh graded towards the surface (element sizes varying
fourfold) and an unstructured Delaunay mesh refined towards a layer
interface (no lattice in the connectivity either)."""
import numpy as np
import pytest

import casegen as cg
from oracle import assemble, march, misfit as omisfit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


def _meshes():
    out = {"small": cg.config_mesh(cg.CONFIGS["small"]),
           "jitter": cg.box_mesh(80.0, 60.0, 40.0, 10.0, jitter=0.22, seed=3),
           # layers from 2.5 m at the surface to ~11 m at the base, jittered
           "graded": cg.box_mesh(80.0, 60.0, 40.0, 10.0, jitter=0.15, seed=4,
                                 z_levels=cg.graded_levels(40.0, 2.5, 1.5)),
           # unstructured Delaunay tetrahedra refined towards a 20 m deep interface
           "delaunay": cg.delaunay_mesh(80.0, 60.0, 40.0, 20.0, 2.5, 10.0, seed=6)}
    return out


MESHES = _meshes()


def _case_for(name, mesh):
    if name == "small":
        return cg.make_case(mesh, cg.CONFIGS["small"])
    c = cg.make_case(mesh, cg.CONFIGS["small"], n_rec=2)
    rng = np.random.default_rng(5)
    c.tet_mat = rng.integers(0, 2, mesh.n_tets).astype(np.uint8)
    return c


@pytest.fixture(scope="module", params=list(MESHES))
def setup(request, sw, ctx):
    name = request.param
    mesh = MESHES[name]
    case = _case_for(name, mesh)
    sys_ = march.build_system(mesh, case)
    gm = sw.Mesh(ctx, mesh)
    gc = sw.Case(ctx, gm, case)
    return name, mesh, case, sys_, gc


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_operator_terms_fp64(setup):
    import torch
    name, mesh, case, S, gc = setup
    x = cg.random_vector(3 * mesh.n_nodes, 1)
    xt = torch.from_numpy(x)
    dt = case.dt
    cM = 4 / dt ** 2 + 2 * case.ray_alpha / dt
    cK = 1 + 2 * case.ray_beta / dt
    refs = {"M": S.M @ x, "K": S.K @ x, "Cabs": S.Cabs @ x,
            "A": (cM * S.M + cK * S.K + (2 / dt) * S.Cabs) @ x,
            "M+K": S.M @ x + S.K @ x}
    for op, ref in refs.items():
        y = gc.apply(op, xt).cpu().numpy()
        assert _rel(y, ref) < 1e-12, (name, op, _rel(y, ref))


def test_operator_fp32(setup):
    import torch
    name, mesh, case, S, gc = setup
    x = cg.random_vector(3 * mesh.n_nodes, 2)
    dt = case.dt
    cM = 4 / dt ** 2 + 2 * case.ray_alpha / dt
    cK = 1 + 2 * case.ray_beta / dt
    ref = (cM * S.M + cK * S.K + (2 / dt) * S.Cabs) @ x
    y = gc.apply_f32("A", torch.from_numpy(x).float()).double().cpu().numpy()
    assert _rel(y, ref) < 2e-5, _rel(y, ref)


def test_rigid_modes_gpu(setup):
    import torch
    name, mesh, case, S, gc = setup
    kn = abs(S.K).sum(1).max()
    for c in range(3):
        r = np.zeros((mesh.n_nodes, 3))
        r[:, c] = 1
        for v in (r.ravel(), np.cross(np.eye(3)[c][None], mesh.xyz).ravel()):
            y = gc.apply("K", torch.from_numpy(v)).cpu().numpy()
            assert np.linalg.norm(y) / (kn * np.linalg.norm(v)) < 1e-13


def test_patch_matvec_gpu(sw, ctx):
    # one material, linear field: K u vanishes at interior nodes
    import torch
    mesh = MESHES["jitter"]
    case = _case_for("jitter", mesh)
    case.tet_mat = np.zeros(mesh.n_tets, np.uint8)
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case)
    G = np.random.default_rng(3).standard_normal((3, 3)) * 1e-3
    u = (mesh.xyz @ G.T).ravel()
    y = gc.apply("K", torch.from_numpy(u)).cpu().numpy().reshape(-1, 3)
    Lx, Ly, Lz = mesh.box
    x = mesh.xyz
    tol = 1e-9
    bnd = (np.abs(x[:, 0]) < tol) | (np.abs(x[:, 0] - Lx) < tol) | (np.abs(x[:, 1]) < tol) | \
          (np.abs(x[:, 1] - Ly) < tol) | (np.abs(x[:, 2] + Lz) < tol) | (np.abs(x[:, 2]) < tol)
    K, _ = assemble.stiffness_and_mass(mesh, case.mat, case.tet_mat)
    scale = abs(K).max() * np.abs(u).max()
    assert np.abs(y[~bnd]).max() < 1e-12 * scale


def test_diag_blocks(setup):
    name, mesh, case, S, gc = setup
    dt = case.dt
    A = ((4 / dt ** 2 + 2 * case.ray_alpha / dt) * S.M + (1 + 2 * case.ray_beta / dt) * S.K
         + (2 / dt) * S.Cabs).tocsr()
    n = mesh.n_nodes
    ref = np.zeros((n, 6))
    idx = 3 * np.arange(n)
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    for k, (i, j) in enumerate(pairs):
        ref[:, k] = np.asarray(A[idx + i, idx + j]).ravel()
    d = gc.diag_blocks().cpu().numpy()
    assert _rel(d, ref) < 1e-12


def test_rhs_from_state(setup):
    name, mesh, case, S, gc = setup
    rng = np.random.default_rng(9)
    n = 3 * mesh.n_nodes
    u, v, a = rng.standard_normal(n) * 1e-3, rng.standard_normal(n) * 1e-2, rng.standard_normal(n)
    step = 7
    gc.set_state(u, v, a, step)
    b = gc.rhs().cpu().numpy()
    dt = case.dt
    F = case.v_in[step + 1] @ S.Fb
    ref = F - S.K @ u + S.C @ v + S.M @ (a + 4 / dt * v)
    assert _rel(b, ref) < 1e-12, _rel(b, ref)
    gc.set_state(np.zeros(n), np.zeros(n), np.zeros(n), 0)


def test_misfit_gpu_vs_oracle(sw, ctx):
    import torch
    rng = np.random.default_rng(0)
    obs = rng.standard_normal((300, 40, 3))
    obs[:, 3, 1] = 0.0   # a silent pair is skipped
    U = obs + 0.05 * rng.standard_normal(obs.shape)
    e_ref, n_ref = omisfit.err(U, obs)
    e, n = sw.misfit(ctx, torch.from_numpy(U), torch.from_numpy(obs))
    assert n == n_ref == 119
    assert abs(e - e_ref) < 1e-13 * e_ref
    assert sw.misfit(ctx, torch.from_numpy(obs), torch.from_numpy(obs))[0] == 0.0
    assert abs(sw.misfit(ctx, torch.zeros_like(torch.from_numpy(obs)), torch.from_numpy(obs))[0] - 1.0) < 1e-15
