"""GPU projection guess (Galerkin projection onto the span of past
increments): the march stays within 1e-6 of the oracle's exact solves with
every step's true residual at 1e-8; the guess itself matches the oracle's
projection (oracle/guess.py) built from the same increments with the
assembled operator; it cuts CG iterations against extrapolation; batched
lanes use it like single cases; a state reset empties its history."""
import numpy as np
import pytest

import casegen as cg
from oracle import guess as og
from oracle import march

pytestmark = pytest.mark.gpu

TOL_WAVE = 1e-6


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


def _relL2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_projection_march_matches_oracle(sw, ctx, small, precision):
    mesh, case, ref = small
    gm = sw.Mesh(ctx, mesh)
    gc = sw.Case(ctx, gm, case, precision=precision, guess="proj", proj_dim=8)
    gc.step(case.n_steps)
    err = _relL2(gc.waveforms(), ref.rec_v)
    it, rel = gc.step_log()
    pc = sw.Case(ctx, gm, case, precision=precision, guess="poly")
    pc.step(case.n_steps)
    itp, _ = pc.step_log()
    print(f"{precision}: rel L2 {err:.2e}; CG iterations/step proj {it[10:].mean():.1f} vs poly "
          f"{itp[10:].mean():.1f}; flags {gc.stats()['flags']}", flush=True)
    assert err < TOL_WAVE
    assert np.all(rel <= 1e-8) and gc.stats()["flags"] == 0
    assert it[10:].sum() < 0.85 * itp[10:].sum()


def test_projected_guess_matches_oracle_projection(sw, ctx, small):
    mesh, case, _ = small
    L = 6
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="mixed", guess="proj", proj_dim=L)
    U = [gc.get_state()[0]]
    for _ in range(14):
        gc.step(1)
        U.append(gc.get_state()[0])
    u, v, a, step = gc.get_state()
    x_gpu = gc.guess().cpu().numpy()
    S = march.build_system(mesh, case)
    A = march.step_matrix(S, case.dt).tocsr()
    b = case.v_in[step + 1] @ S.Fb - S.K @ u + S.C @ v + S.M @ (a + (4.0 / case.dt) * v)
    X = np.diff(np.array(U), axis=0)[-L:].T
    x_or = og.projection(A, X, b)
    nb = np.linalg.norm(b)
    r_gpu = np.linalg.norm(b - A @ x_gpu) / nb
    r_or = np.linalg.norm(b - A @ x_or) / nb
    r_p2 = np.linalg.norm(b - A @ og.extrapolation(list(X.T), 2)) / nb
    e = x_gpu - x_or
    e_rel = np.sqrt(e @ (A @ e)) / np.sqrt(x_or @ (A @ x_or))
    print(f"initial residual: gpu {r_gpu:.3e} oracle {r_or:.3e} quadratic {r_p2:.3e}; energy diff {e_rel:.2e}",
          flush=True)
    assert r_gpu <= 1.05 * r_or + 1e-12
    assert e_rel <= 1e-6
    assert r_or < 0.5 * r_p2


def test_batched_projection_lanes_match_single(sw, ctx):
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.1, seed=7)
    gm = sw.Mesh(ctx, mesh)
    base = cg.CONFIGS["small"]
    cfg = cg.BoxConfig("pb", (60.0, 40.0, 40.0), 10.0, 20.0, (4.0, 10.0), (30.0, 60.0), base.freqs, base.t0,
                       base.dt, 30, 2, 60)
    cases = [cg.make_case(mesh, cfg, seed=60 + k, n_rec=2) for k in range(3)]
    lanes = [sw.Case(ctx, gm, c, precision="mixed", guess=g, proj_dim=6)
             for c, g in zip(cases, ["proj", "proj", "poly"])]
    sw.Batch(ctx, lanes).step(30)
    for c, g, lane in zip(cases, ["proj", "proj", "poly"], lanes):
        alone = sw.Case(ctx, gm, c, precision="mixed", guess=g, proj_dim=6)
        alone.step(30)
        assert _relL2(lane.waveforms(), alone.waveforms()) < TOL_WAVE
        it, rel = lane.step_log()
        it1, _ = alone.step_log()
        assert np.all(rel <= 1e-8) and lane.stats()["flags"] == 0
        assert abs(int(it.sum()) - int(it1.sum())) <= 0.05 * it1.sum() + 30


def test_state_reset_empties_projection_history(sw, ctx, small):
    mesh, case, ref = small
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="mixed", guess="proj")
    gc.step(20)
    u, v, a, _ = gc.get_state()
    gc.set_state(np.zeros_like(u), np.zeros_like(v), np.zeros_like(a), 0)
    gc.step(case.n_steps)
    assert _relL2(gc.waveforms(0, case.n_steps), ref.rec_v) < TOL_WAVE
    assert gc.stats()["max_true_rel_res"] <= 1e-8


def test_bad_proj_dim_rejected(sw, ctx, small):
    mesh, case, _ = small
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, sw.Mesh(ctx, mesh), case, guess="proj", proj_dim=17)
