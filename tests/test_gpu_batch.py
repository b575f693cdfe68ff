"""GPU parity of batched marching: many candidate models of uneven mesh
sizes stepped together (one launch per phase for all lanes) give the same
waveforms as the oracle's exact per-step solves and as each case stepped
alone; every lane meets the true-residual tolerance on every step; lanes
keep their own guesses, convergence and fallbacks; degenerate lanes (zero
input) and bad batches are handled."""
import dataclasses

import numpy as np
import pytest

import casegen as cg
from oracle import march
from oracle import mlp as om

pytestmark = pytest.mark.gpu

TOL_WAVE = 1e-6   # relative L2 waveform error against the oracle


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


def _relL2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def uneven():
    """Two meshes of different sizes (one jittered), three candidate models
    on each with their own interface fields."""
    base = cg.CONFIGS["small"]
    cfg = cg.BoxConfig("uneven", (60.0, 40.0, 40.0), 10.0, 20.0, (4.0, 10.0), (30.0, 60.0), base.freqs, base.t0,
                       base.dt, 24, 2, 40)
    meshes = [cg.box_mesh(60.0, 40.0, 40.0, 10.0), cg.box_mesh(80.0, 60.0, 40.0, 10.0, jitter=0.15, seed=3)]
    cases = []
    for mi, m in enumerate(meshes):
        for k in range(3):
            cases.append((mi, cg.make_case(m, cfg, seed=40 + 3 * mi + k, n_rec=2)))
    return meshes, cases


def test_uneven_batch_matches_oracle_and_single(sw, ctx, uneven):
    meshes, cases = uneven
    gms = [sw.Mesh(ctx, m) for m in meshes]
    guesses = ["poly", "zero", "poly", "poly", "zero", "poly"]
    lanes = [sw.Case(ctx, gms[mi], c, precision="mixed", guess=g) for (mi, c), g in zip(cases, guesses)]
    b = sw.Batch(ctx, lanes)
    n = cases[0][1].n_steps
    b.step(n // 2)
    b.step(n - n // 2)
    for (mi, c), g, lane in zip(cases, guesses, lanes):
        ref = march.run_case(meshes[mi], c, solver="lu")
        w = lane.waveforms()
        err = _relL2(w, ref.rec_v)
        it, rel = lane.step_log()
        st = lane.stats()
        print(f"mesh {mi} guess {g}: rel L2 {err:.2e}, its/step {it.mean():.1f}, flags {st['flags']}", flush=True)
        assert err < TOL_WAVE
        assert np.all(rel <= 1e-8) and st["flags"] == 0 and st["steps"] == n
        # the same case stepped alone
        alone = sw.Case(ctx, gms[mi], c, precision="mixed", guess=g)
        alone.step(n)
        assert _relL2(w, alone.waveforms()) < TOL_WAVE
        it1, _ = alone.step_log()
        assert abs(it.sum() - it1.sum()) <= 0.05 * it1.sum() + n


def test_batch_multi_tile_mesh_matches_single(sw, ctx):
    """A mesh of many tiles (interior and shared nodes, XCD-ordered work
    items) with five lanes: each lane equals its case stepped alone."""
    cfg = cg.CONFIGS["batch200"]
    mesh = cg.box_mesh(100.0, 100.0, 50.0, 5.0)
    gm = sw.Mesh(ctx, mesh)
    cases = [cg.make_case(mesh, cfg, seed=1100 + k, n_steps=30, n_rec=4) for k in range(5)]
    lanes = [sw.Case(ctx, gm, c, precision="mixed", guess="poly") for c in cases]
    sw.Batch(ctx, lanes).step(30)
    for c, lane in zip(cases, lanes):
        alone = sw.Case(ctx, gm, c, precision="mixed", guess="poly")
        alone.step(30)
        w, w1 = lane.waveforms(), alone.waveforms()
        assert _relL2(w, w1) < TOL_WAVE
        _, rel = lane.step_log()
        assert np.all(rel <= 1e-8)
        u, v, a, step = lane.get_state()
        u1, v1, a1, _ = alone.get_state()
        assert step == 30 and _relL2(u, u1) < TOL_WAVE


def test_zero_input_lane_and_fallback_lane(sw, ctx):
    """A lane with no input (b = 0 every step: zero increments, no
    iterations) and a lane whose network is NaN (guess rejected, flag 4,
    still correct) beside an ordinary lane."""
    mesh = cg.box_mesh(40.0, 30.0, 30.0, 10.0)
    gm = sw.Mesh(ctx, mesh)
    base = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=12, n_rec=1)
    quiet = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=12, n_rec=1)
    quiet.v_in = np.zeros_like(quiet.v_in)
    ref = march.run_case(mesh, base, solver="lu")
    l0 = sw.Case(ctx, gm, base, precision="mixed", guess="poly")
    l1 = sw.Case(ctx, gm, quiet, precision="mixed", guess="poly")
    l2 = sw.Case(ctx, gm, base, precision="mixed", guess="mlp")
    l2.attach_mlp(sw.Mlp(ctx, np.full(om.N_PARAM, np.nan)))
    sw.Batch(ctx, [l0, l1, l2]).step(12)
    assert _relL2(l0.waveforms(), ref.rec_v) < TOL_WAVE
    assert np.all(l1.waveforms() == 0.0)
    it1, rel1 = l1.step_log()
    assert np.all(it1 == 0) and np.all(rel1 == 0.0) and l1.stats()["flags"] == 0
    st2 = l2.stats()
    assert st2["flags"] & 4 and not st2["flags"] & 3
    assert _relL2(l2.waveforms(), ref.rec_v) < TOL_WAVE


def test_batch_rejects_bad_sets(sw, ctx):
    mesh = cg.box_mesh(30.0, 20.0, 20.0, 10.0)
    gm = sw.Mesh(ctx, mesh)
    c = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=3, n_rec=1)
    a = sw.Case(ctx, gm, c, precision="mixed")
    f = sw.Case(ctx, gm, c, precision="fp64")
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Batch(ctx, [a, f])
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Batch(ctx, [a, a])
    b = sw.Batch(ctx, [a])
    b.step(3)
    with pytest.raises(sw.SwError, match="SW_ESTATE"):
        b.step(1)
    m = sw.Case(ctx, gm, c, precision="mixed", guess="mlp")
    with pytest.raises(sw.SwError, match="SW_ESTATE"):
        sw.Batch(ctx, [m]).step(1)


def test_many_materials(sw, ctx):
    """A case with more materials than the pipelined FP32 pass keeps in LDS
    (32) marches on the other FP32 pass, alone and in a batch (the lane
    pass reads the table from global memory); its extra table rows repeat
    the bedrock, so its waveforms are those of the two-material case, each
    within the solver tolerance of the oracle."""
    cfg = cg.CONFIGS["small"]
    mesh = cg.config_mesh(cfg)
    c = cg.make_case(mesh, cfg, n_steps=20)
    many = dataclasses.replace(c, mat=np.concatenate([c.mat, np.repeat(c.mat[-1:], 31, axis=0)]))
    gm = sw.Mesh(ctx, mesh)
    two = sw.Case(ctx, gm, c, precision="mixed", guess="proj")
    wide = sw.Case(ctx, gm, many, precision="mixed", guess="proj")
    lane = sw.Case(ctx, gm, many, precision="mixed", guess="proj")
    two.step(20)
    wide.step(20)
    sw.Batch(ctx, [lane]).step(20)
    ref = march.run_case(mesh, c, solver="lu")
    for x in (wide, lane):
        assert x.stats()["max_true_rel_res"] <= 1e-8
        assert _relL2(x.waveforms(), ref.rec_v) < TOL_WAVE
        assert _relL2(x.waveforms(), two.waveforms()) < TOL_WAVE
