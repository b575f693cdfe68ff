"""Deterministic FP64 mode (sw_case_desc.deterministic): every element's and
face's results go to slot buffers and each node sums its own slots in
element order; every reduction adds in a fixed order.  Checked: the operator
terms, right-hand side and block-Jacobi diagonal against the oracle's
assembled matrices (and equal bits on repetition); repeated marches with the
zero, polynomial and projection guesses give identical bits (waveforms,
states and iteration logs), with and without CG graphs; 50 steps straight
against 25 steps, a checkpoint into a new case and 25 more, bit for bit; the
march against the oracle's exact solves; and the rejected requests."""
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
def jittered(sw, ctx):
    """A jittered two-material mesh of several tiles (tile cap 256 nodes)."""
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.15, seed=4)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=50, n_rec=2)
    case.tet_mat = np.random.default_rng(5).integers(0, 2, mesh.n_tets).astype(np.uint8)
    gm = sw.Mesh(ctx, mesh, tile_nodes=256, deterministic=True)
    assert gm.info()[0] >= 4
    return mesh, case, gm


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_operator_rhs_diag_against_oracle(sw, ctx, jittered):
    import torch
    mesh, case, gm = jittered
    S = march.build_system(mesh, case)
    dt = case.dt
    cM = 4 / dt ** 2 + 2 * case.ray_alpha / dt
    cK = 1 + 2 * case.ray_beta / dt
    A = (cM * S.M + cK * S.K + (2 / dt) * S.Cabs).tocsr()
    gc = sw.Case(ctx, gm, case, deterministic=True)
    x = cg.random_vector(3 * mesh.n_nodes, 1)
    xt = torch.from_numpy(x)
    for op, ref in (("M", S.M @ x), ("K", S.K @ x), ("Cabs", S.Cabs @ x), ("A", A @ x)):
        y = gc.apply(op, xt).cpu().numpy()
        assert _rel(y, ref) < 1e-12, (op, _rel(y, ref))
        assert np.array_equal(gc.apply(op, xt).cpu().numpy(), y), op
    n = mesh.n_nodes
    idx = 3 * np.arange(n)
    ref = np.stack([np.asarray(A[idx + i, idx + j]).ravel()
                    for i, j in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]], 1)
    d = gc.diag_blocks().cpu().numpy()
    assert _rel(d, ref) < 1e-12
    d2 = sw.Case(ctx, gm, case, deterministic=True).diag_blocks().cpu().numpy()
    assert np.array_equal(d, d2)
    rng = np.random.default_rng(9)
    u, v, a = rng.standard_normal(3 * n) * 1e-3, rng.standard_normal(3 * n) * 1e-2, rng.standard_normal(3 * n)
    gc.set_state(u, v, a, 7)
    b = gc.rhs().cpu().numpy()
    bref = case.v_in[8] @ S.Fb - S.K @ u + S.C @ v + S.M @ (a + 4 / dt * v)
    assert _rel(b, bref) < 1e-12
    assert np.array_equal(gc.rhs().cpu().numpy(), b)


def _march(sw, ctx, gm, case, guess, n, graphs=True):
    ctx.set_graphs(graphs)
    gc = sw.Case(ctx, gm, case, precision="fp64", guess=guess, deterministic=True, proj_dim=6)
    gc.step(n)
    ctx.set_graphs(True)
    u, v, a, step = gc.get_state()
    return gc, gc.waveforms(), (u, v, a), gc.step_log()[0]


@pytest.mark.parametrize("guess", ["zero", "poly", "proj"])
def test_repeated_marches_identical_bits(sw, ctx, jittered, guess):
    mesh, case, gm = jittered
    ref = march.run_case(mesh, case, solver="lu").rec_v
    g1, w1, s1, it1 = _march(sw, ctx, gm, case, guess, 50)
    _, w2, s2, it2 = _march(sw, ctx, gm, case, guess, 50)
    _, w3, s3, it3 = _march(sw, ctx, gm, case, guess, 50, graphs=False)
    for w, s, it in ((w2, s2, it2), (w3, s3, it3)):
        assert np.array_equal(w, w1) and np.array_equal(it, it1)
        assert all(np.array_equal(p, q) for p, q in zip(s, s1))
    _, rel = g1.step_log()
    assert np.all(rel <= 1e-8) and not g1.stats()["flags"] & 3
    assert np.linalg.norm(w1 - ref) <= 1e-6 * np.linalg.norm(ref)


def test_checkpoint_resume_identical_bits(sw, ctx, jittered):
    """50 steps straight against 25 steps, the state into a new case and 25
    more (the zero guess: a step depends on the state alone)."""
    mesh, case, gm = jittered
    _, w_all, s_all, _ = _march(sw, ctx, gm, case, "zero", 50)
    a = sw.Case(ctx, gm, case, precision="fp64", guess="zero", deterministic=True)
    a.step(25)
    u, v, acc, st = a.get_state()
    b = sw.Case(ctx, gm, case, precision="fp64", guess="zero", deterministic=True)
    b.set_state(u, v, acc, st)
    b.step(25)
    assert all(np.array_equal(p, q) for p, q in zip(b.get_state()[:3], s_all))
    assert np.array_equal(np.concatenate([a.waveforms(0, 25), b.waveforms(25, 25)]), w_all)


def test_deterministic_requests_rejected(sw, ctx, jittered):
    mesh, case, gm = jittered
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, case, precision="mixed", guess="zero", deterministic=True)
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, case, precision="fp64", guess="mlp", deterministic=True)
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="fp64", deterministic=True)
