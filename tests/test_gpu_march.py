"""GPU parity of the whole time march against the oracle (sparse LU, exact
per-step solves): receiver waveforms of the small two-layer case (50 steps)
for FP64 PCG, mixed FP32/FP64 refinement and the polynomial guess, and over
400 steps in the benchmark's configuration; the FP64 true residual of every
step; exact energy conservation and modal solutions of the Newmark scheme
on the GPU; checkpoint/resume."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import casegen as cg
from oracle import march

pytestmark = pytest.mark.gpu

TOL_WAVE = 1e-6   # relative L2 waveform error against the oracle


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


@pytest.fixture(scope="module")
def small():
    cfg = cg.CONFIGS["small"]
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg)
    ref = march.run_case(mesh, case, solver="lu")
    return mesh, case, ref


@pytest.fixture(scope="module")
def gmesh(sw, ctx, small):
    return sw.Mesh(ctx, small[0])


def _relL2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision,guess", [("fp64", "zero"), ("fp64", "poly"), ("mixed", "zero"),
                                             ("mixed", "poly")])
def test_small_case_waveforms(sw, ctx, small, gmesh, precision, guess):
    mesh, case, ref = small
    gc = sw.Case(ctx, gmesh, case, rtol=1e-8, precision=precision, guess=guess)
    gc.step(case.n_steps)
    w = gc.waveforms()
    err = _relL2(w, ref.rec_v)
    print(f"{precision}/{guess}: waveform rel L2 {err:.3e}, stats {gc.stats()}", flush=True)
    assert err < TOL_WAVE
    it, rel = gc.step_log()
    assert np.all(rel <= 1e-8) and np.all(it > 0)
    st = gc.stats()
    assert st["flags"] == 0 and st["steps"] == case.n_steps


def test_guess_reduces_iterations(sw, ctx, small, gmesh):
    mesh, case, _ = small
    its = {}
    for g in ("zero", "poly"):
        gc = sw.Case(ctx, gmesh, case, guess=g)
        gc.step(case.n_steps)
        its[g] = gc.stats()["cg_iters"]
    assert its["poly"] < its["zero"]


def test_jittered_mesh_march(sw, ctx):
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.2, seed=1)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=20, n_rec=2)
    case.tet_mat = np.random.default_rng(2).integers(0, 2, mesh.n_tets).astype(np.uint8)
    ref = march.run_case(mesh, case, solver="lu")
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="mixed", guess="poly")
    gc.step(case.n_steps)
    assert _relL2(gc.waveforms(), ref.rec_v) < TOL_WAVE


def _no_face_mesh(mesh):
    m = cg.Mesh(mesh.xyz, mesh.tet10, np.zeros((0, 6), np.int32), np.zeros(0, np.int32),
                np.zeros(0, np.uint8), mesh.box, mesh.cell, mesh.ncell)
    return m


def test_energy_conservation_gpu(sw, ctx):
    # no damping, no dashpots, no input: E = 1/2 v'Mv + 1/2 u'Ku is constant
    mesh = _no_face_mesh(cg.box_mesh(40.0, 30.0, 20.0, 10.0))
    case = cg.make_case(cg.box_mesh(40.0, 30.0, 20.0, 10.0), cg.CONFIGS["small"], n_steps=60, n_rec=1)
    case.ray_alpha = case.ray_beta = 0.0
    case.v_in = np.zeros_like(case.v_in)
    S = march.build_system(mesh, case, damping=False, dashpot_roles=(), input_force=False)
    rng = np.random.default_rng(0)
    n = 3 * mesh.n_nodes
    u0, v0 = rng.standard_normal(n) * 1e-3, rng.standard_normal(n) * 1e-2
    a0 = march.consistent_acceleration(S, u0, v0, np.zeros(n))
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, rtol=1e-12)
    gc.set_state(u0, v0, a0, 0)
    E0 = 0.5 * v0 @ (S.M @ v0) + 0.5 * u0 @ (S.K @ u0)
    for _ in range(6):
        gc.step(10)
        u, v, _, _ = gc.get_state()
        E = 0.5 * v @ (S.M @ v) + 0.5 * u @ (S.K @ u)
        assert abs(E - E0) < 1e-8 * E0


def test_modal_solution_gpu(sw, ctx):
    mesh = _no_face_mesh(cg.box_mesh(40.0, 30.0, 20.0, 10.0))
    case = cg.make_case(cg.box_mesh(40.0, 30.0, 20.0, 10.0), cg.CONFIGS["small"], n_steps=40, n_rec=1)
    case.ray_alpha = case.ray_beta = 0.0
    case.v_in = np.zeros_like(case.v_in)
    S = march.build_system(mesh, case, damping=False, dashpot_roles=(), input_force=False)
    w2, phi = sla.eigh(S.K.toarray(), S.M.toarray())
    k = 25
    w, phi = math.sqrt(w2[k]), phi[:, k]
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, rtol=1e-12)
    gc.set_state(phi, 0 * phi, -w2[k] * phi, 0)
    Om = 2 * math.atan(w * case.dt / 2)
    for n_ in range(1, 41):
        gc.step(1)
        if n_ % 10 == 0:
            u, _, _, _ = gc.get_state()
            assert np.abs(u - phi * math.cos(n_ * Om)).max() < 1e-7 * np.abs(phi).max()


def test_checkpoint_resume(sw, ctx, small, gmesh):
    mesh, case, _ = small
    a = sw.Case(ctx, gmesh, case, guess="zero")
    a.step(20)
    b = sw.Case(ctx, gmesh, case, guess="zero")
    b.step(10)
    u, v, acc, st = b.get_state()
    c = sw.Case(ctx, gmesh, case, guess="zero")
    c.set_state(u, v, acc, st)
    c.step(10)
    wa = a.waveforms(10, 10)
    wc = c.waveforms(10, 10)
    assert _relL2(wc, wa) < 1e-7


def test_case_misfit_against_oracle_reference(sw, ctx, small, gmesh):
    import torch
    from oracle import misfit as om
    mesh, case, ref = small
    # reference model: a different interface seed, same mesh and input
    case2 = cg.make_case(mesh, cg.CONFIGS["small"], seed=5)
    obs = march.run_case(mesh, case2, solver="lu").rec_v
    gc = sw.Case(ctx, gmesh, case)
    gc.step(case.n_steps)
    e, n = gc.misfit(torch.from_numpy(obs))
    e_ref, n_ref = om.err(ref.rec_v, obs)
    assert n == n_ref
    assert abs(e - e_ref) < 1e-5 * e_ref


def test_graded_mesh_march(sw, ctx):
    """A mesh refined towards the surface (layers 2.5 m at the top to ~11 m
    at the base, jittered): mixed precision with the projection guess
    against the oracle's exact solves."""
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.15, seed=5, z_levels=cg.graded_levels(40.0, 2.5, 1.5))
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=20, n_rec=2)
    ref = march.run_case(mesh, case, solver="lu")
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="mixed", guess="proj")
    gc.step(case.n_steps)
    assert _relL2(gc.waveforms(), ref.rec_v) < TOL_WAVE
    assert gc.stats()["max_true_rel_res"] <= 1e-8 and gc.stats()["flags"] == 0


def test_unstructured_mesh_march(sw, ctx):
    """An unstructured Delaunay mesh refined towards a 15 m deep layer
    interface (element sizes 2.5-10 m), the benchmark's solver (mixed
    precision, projected guess), as a single case and as a batch lane,
    against the oracle's exact solves."""
    mesh = cg.delaunay_mesh(40.0, 30.0, 30.0, 15.0, 2.5, 10.0, seed=8)
    cfg = cg.CONFIGS["small"]
    case = cg.make_case(mesh, cfg, n_steps=30, n_rec=3)
    ref = march.run_case(mesh, case, solver="lu").rec_v
    gm = sw.Mesh(ctx, mesh)
    alone = sw.Case(ctx, gm, case, precision="mixed", guess="proj")
    alone.step(case.n_steps)
    lanes = [sw.Case(ctx, gm, case, precision="mixed", guess="proj") for _ in range(2)]
    sw.Batch(ctx, lanes).step(case.n_steps)
    for gc in [alone] + lanes:
        err = np.linalg.norm(gc.waveforms() - ref) / np.linalg.norm(ref)
        st = gc.stats()
        assert err < TOL_WAVE and st["max_true_rel_res"] <= 1e-8 and not st["flags"] & 3, (err, st)


def test_long_march_as_benchmarked(sw, ctx):
    """400 steps of the small model (4 s: the wave crosses the box, reflects
    at the free surface and leaves through the dashpots) in the benchmark's
    configuration (FP32 inner CG in FP64 refinement, projection guess over
    6 increments): receiver waveforms within 1e-6 of the oracle's exact
    solves over the whole record, and the true residual of every step
    within 1e-8, so neither the projection nor the refinement drifts."""
    cfg = cg.CONFIGS["small"]
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg, n_steps=400)
    ref = march.run_case(mesh, case, solver="lu")
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="mixed", guess="proj", proj_dim=6)
    gc.step(400)
    it, rel = gc.step_log()
    err = _relL2(gc.waveforms(), ref.rec_v)
    late = _relL2(gc.waveforms()[300:], ref.rec_v[300:])
    print(f"400 steps: waveform rel L2 {err:.2e} (steps 300-400: {late:.2e}); "
          f"CG iterations/step {it.mean():.1f}", flush=True)
    assert err < TOL_WAVE and late < TOL_WAVE
    assert np.all(rel <= 1e-8) and gc.stats()["flags"] == 0
