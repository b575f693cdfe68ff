"""Pins of the native assembled-sparse oracle (oracle/bsr.py,
C++/OpenMP symmetric 3x3 block-sparse FP64) against the SciPy oracle,
whose element integrals and march are pinned by the closed-form tests:
the assembled products with K, M and C_abs and the input basis on a
regular, a jittered and a surface-graded mesh; the symmetry its upper-
triangle storage implies; and marched receiver records (Newmark step,
Section 3) from rest and from a non-zero state."""
import numpy as np
import pytest

import casegen as cg
from oracle import bsr, march


def _meshes():
    return {
        "small": cg.config_mesh(cg.CONFIGS["small"]),
        "jitter": cg.box_mesh(40.0, 30.0, 20.0, 10.0, jitter=0.2, seed=7),
        "graded": cg.box_mesh(30.0, 20.0, 40.0, 10.0, jitter=0.15, seed=3,
                              z_levels=cg.graded_levels(40.0, 2.5, 1.6)),
    }


@pytest.fixture(scope="module")
def meshes():
    return _meshes()


@pytest.mark.parametrize("name", ["small", "jitter", "graded"])
def test_bsr_operators_match_scipy_oracle(meshes, name):
    mesh = meshes[name]
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=2, n_rec=1)
    # a third material, so that every (Vp, Vs, rho) enters
    mat = np.vstack([case.mat, [900.0, 300.0, 1900.0]])
    tm = case.tet_mat.copy()
    tm[::7] = 2
    case.mat, case.tet_mat = mat, tm
    ref = march.build_system(mesh, case)
    S = bsr.System(mesh, mat, tm)
    x = np.random.default_rng(3).standard_normal(3 * mesh.n_nodes)
    for kw, R in ((dict(cK=1.0), ref.K), (dict(cM=1.0), ref.M), (dict(cC=1.0), ref.Cabs)):
        y, yr = S.apply(x, **kw), R @ x
        assert np.linalg.norm(y - yr) <= 1e-13 * np.linalg.norm(yr), kw
    # fused form, as the solver applies it
    cK, cM, cC = 1.2, 1.6e5, 400.0
    y = S.apply(x, cK=cK, cM=cM, cC=cC)
    yr = cK * (ref.K @ x) + cM * (ref.M @ x) + cC * (ref.Cabs @ x)
    assert np.linalg.norm(y - yr) <= 1e-13 * np.linalg.norm(yr)
    F = S.input_basis()
    assert np.abs(F - ref.Fb).max() <= 1e-13 * np.abs(ref.Fb).max()


def test_bsr_symmetric_storage(meshes):
    mesh = meshes["jitter"]
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=2, n_rec=1)
    S = bsr.System(mesh, case.mat, case.tet_mat)
    rng = np.random.default_rng(9)
    x, y = rng.standard_normal((2, 3 * mesh.n_nodes))
    Ax = S.apply(x, cK=1.0, cM=3e4, cC=200.0)
    Ay = S.apply(y, cK=1.0, cM=3e4, cC=200.0)
    assert abs(x @ Ay - y @ Ax) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)
    # rigid translations and rotations are in the null space of K
    xyz = mesh.xyz - mesh.xyz.mean(0)
    for m in range(6):
        r = np.zeros((mesh.n_nodes, 3))
        if m < 3:
            r[:, m] = 1.0
        else:
            w = np.eye(3)[m - 3]
            r = np.cross(w, xyz)
        Kr = S.apply(r.ravel(), cK=1.0)
        Kx = S.apply(x, cK=1.0)
        assert np.linalg.norm(Kr) <= 1e-12 * np.linalg.norm(Kx) * np.linalg.norm(r) / np.linalg.norm(x)


def test_bsr_march_matches_lu_oracle(meshes):
    mesh = meshes["small"]
    case = cg.make_case(mesh, cg.CONFIGS["small"])
    S = bsr.System(mesh, case.mat, case.tet_mat)
    out = S.march(case.dt, case.ray_alpha, case.ray_beta, case.v_in, case.n_steps, case.rec_node, rtol=1e-12)
    ref = march.run_case(mesh, case, solver="lu")
    assert np.all(out["relres"] <= 1e-12)
    assert np.linalg.norm(out["rec_v"] - ref.rec_v) <= 1e-9 * np.linalg.norm(ref.rec_v)
    for k in ("u", "v", "a"):
        r = getattr(ref, k)
        assert np.linalg.norm(out[k] - r) <= 1e-9 * np.linalg.norm(r), k


def test_bsr_march_from_state_with_offset_input(meshes):
    """Non-zero (u, v, a) and an input window starting at step 5: the state
    and the input enter as the SciPy oracle's do."""
    mesh = meshes["jitter"]
    cfg = cg.CONFIGS["small"]
    case = cg.make_case(mesh, cfg, n_steps=25, n_rec=1)
    case.rec_node = np.array([0, 17, mesh.n_nodes - 1], np.int32)
    n3 = 3 * mesh.n_nodes
    rng = np.random.default_rng(4)
    u0 = 1e-4 * rng.standard_normal(n3)
    v0 = cg.smooth_field(mesh, 5, corr=15.0, amp=1e-3)
    a0 = 1e-2 * rng.standard_normal(n3)
    S = bsr.System(mesh, case.mat, case.tet_mat)
    out = S.march(case.dt, case.ray_alpha, case.ray_beta, case.v_in[5:], 20, case.rec_node, u0=u0, v0=v0, a0=a0,
                  rtol=1e-12, guess="zero")
    sysm = march.build_system(mesh, case)
    ref = march.run(sysm, case.dt, case.v_in[5:], 20, case.rec_node, u0=u0, v0=v0, a0=a0, solver="lu")
    assert np.linalg.norm(out["rec_v"] - ref.rec_v) <= 1e-9 * np.linalg.norm(ref.rec_v)
    assert np.linalg.norm(out["u"] - ref.u) <= 1e-9 * np.linalg.norm(ref.u)


def test_smooth_field_is_seeded_and_scaled(meshes):
    mesh = meshes["small"]
    a = cg.smooth_field(mesh, 1, corr=40.0, amp=2e-3)
    assert a.shape == (3 * mesh.n_nodes,)
    assert abs(np.abs(a).max() - 2e-3) < 1e-15
    assert np.array_equal(a, cg.smooth_field(mesh, 1, corr=40.0, amp=2e-3))
    assert not np.array_equal(a, cg.smooth_field(mesh, 2, corr=40.0, amp=2e-3))
