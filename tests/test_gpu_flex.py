"""The flexible outer CG (SW_MIXED_FP32_FLEX: FP64 flexible CG whose
variable preconditioner is the FP32 inner CG; Section 3 names CG with
variable preconditioning) against the oracle's exact solves: receiver
waveforms of the small case and of a jittered unstructured mesh with every
guess, the true residual on every step, and the rejection of flexible cases
by batches."""
import numpy as np
import pytest

import casegen as cg
from oracle import march

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


@pytest.fixture(scope="module")
def small(sw, ctx):
    mesh = cg.config_mesh(cg.CONFIGS["small"])
    case = cg.make_case(mesh, cg.CONFIGS["small"])
    ref = march.run_case(mesh, case, solver="lu").rec_v
    return mesh, case, ref, sw.Mesh(ctx, mesh)


@pytest.mark.parametrize("guess", ["zero", "poly", "proj"])
def test_flex_march_matches_oracle(sw, ctx, small, guess):
    mesh, case, ref, gm = small
    gc = sw.Case(ctx, gm, case, precision="flex", guess=guess)
    gc.step(case.n_steps)
    w = gc.waveforms()
    st = gc.stats()
    _, rel = gc.step_log()
    err = np.linalg.norm(w - ref) / np.linalg.norm(ref)
    ir = sw.Case(ctx, gm, case, precision="mixed", guess=guess)
    ir.step(case.n_steps)
    print(f"flex/{guess}: rel L2 {err:.2e}, CG iterations {st['cg_iters']} (refinement: {ir.stats()['cg_iters']}), "
          f"FP64 passes {st['ir_outer']} (refinement: {ir.stats()['ir_outer']})", flush=True)
    assert err < 1e-6
    assert np.all(rel <= 1e-8) and st["flags"] & 3 == 0


def test_flex_on_jittered_mesh_matches_oracle(sw, ctx):
    mesh = cg.box_mesh(60.0, 40.0, 30.0, 10.0, jitter=0.2, seed=11)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=30, n_rec=2)
    case.tet_mat = np.random.default_rng(3).integers(0, 2, mesh.n_tets).astype(np.uint8)
    ref = march.run_case(mesh, case, solver="lu").rec_v
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="flex", guess="proj")
    gc.step(case.n_steps)
    err = np.linalg.norm(gc.waveforms() - ref) / np.linalg.norm(ref)
    assert err < 1e-6 and gc.stats()["max_true_rel_res"] <= 1e-8


def test_batch_rejects_flex_cases(sw, ctx, small):
    mesh, case, _, gm = small
    lanes = [sw.Case(ctx, gm, case, precision="flex", guess="proj")]
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Batch(ctx, lanes)
