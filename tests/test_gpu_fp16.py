"""The 16-bit precision mode (SW_MIXED_FP16: the FP32 inner CG with its
direction vector stored in bfloat16, gathered by the operator pass and used
by the x and p updates, inside the FP64 refinement) against the oracle's
exact solves: receiver waveforms within 1e-6 relative L2 and the true
relative residual within 1e-8 on every step, for every guess, on the small
case, a jittered two-material mesh, and a mesh of small tiles walked by a
capped persistent grid (every workgroup hands several tiles over); with and
without HIP graph replays; batches reject it."""
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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _check(gc, ref, n):
    st = gc.stats()
    _, rel = gc.step_log()
    err = _rel(gc.waveforms(), ref)
    assert st["steps"] == n and err < 1e-6 and np.all(rel <= 1e-8) and not st["flags"] & 3, (err, st)
    return err, st


@pytest.mark.parametrize("guess", ["zero", "poly", "proj"])
def test_fp16_march_matches_oracle(sw, ctx, small, guess):
    mesh, case, ref, gm = small
    gc = sw.Case(ctx, gm, case, precision="fp16", guess=guess)
    gc.step(case.n_steps)
    err, st = _check(gc, ref, case.n_steps)
    g32 = sw.Case(ctx, gm, case, precision="mixed", guess=guess)
    g32.step(case.n_steps)
    print(f"fp16/{guess}: rel L2 {err:.2e}, CG iterations {st['cg_iters']} (FP32 direction: "
          f"{g32.stats()['cg_iters']}), FP64 passes {st['ir_outer']} (FP32: {g32.stats()['ir_outer']})", flush=True)


def test_fp16_on_jittered_two_material_mesh(sw, ctx):
    mesh = cg.box_mesh(60.0, 40.0, 30.0, 10.0, jitter=0.2, seed=11)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=30, n_rec=2)
    case.tet_mat = np.random.default_rng(3).integers(0, 2, mesh.n_tets).astype(np.uint8)
    ref = march.run_case(mesh, case, solver="lu").rec_v
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, precision="fp16", guess="proj")
    gc.step(case.n_steps)
    _check(gc, ref, case.n_steps)


def test_fp16_with_small_tiles_and_a_capped_grid(sw, small):
    mesh, case, ref, _ = small
    c = sw.Context(0)
    c.set_grid_cap(8)
    gm = sw.Mesh(c, mesh, tile_nodes=64)
    assert gm.info()[0] >= 32
    gc = sw.Case(c, gm, case, precision="fp16", guess="proj")
    gc.step(case.n_steps)
    _check(gc, ref, case.n_steps)


def test_fp16_graph_replays_match_direct_launches(sw, ctx, small):
    mesh, case, ref, gm = small
    out = {}
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        gc = sw.Case(ctx, gm, case, precision="fp16", guess="proj")
        gc.step(case.n_steps)
        it, _ = gc.step_log()
        out[graphs] = (gc.waveforms(), it)
        _check(gc, ref, case.n_steps)
    ctx.set_graphs(True)
    (w0, it0), (w1, it1) = out[False], out[True]
    # the atomic sums add in a different order on every run; rounding p to
    # bfloat16 can turn such a last-bit difference into a different rounded
    # direction, and a solve near its threshold into one more refinement
    # round (measured: one step 53 against 49, totals 5 apart in 2785),
    # where FP32 directions differ by one iteration at most.  A step may so
    # differ by up to one inner solve, and the two marches by up to what
    # the 1e-8 residual leaves in the waveforms; both meet the oracle bound
    assert np.abs(it0 - it1).max() <= 40 and abs(int(it0.sum()) - int(it1.sum())) <= 0.02 * it0.sum(), (it0, it1)
    assert _rel(w1, w0) < 5e-7


def test_batch_rejects_fp16_cases(sw, ctx, small):
    mesh, case, _, gm = small
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Batch(ctx, [sw.Case(ctx, gm, case, precision="fp16", guess="proj")])


def test_fp16_with_learned_guess_autotune_and_checkpoint(sw, ctx, small):
    """The 16-bit mode with the learned guess (the network's initial
    parameters: extrapolation through the network's kernels), after the
    set-up autotuner, and resumed from a checkpoint taken mid-march: the
    resumed waveforms match the oracle's over the same steps."""
    mesh, case, ref, gm = small
    net = sw.Mlp(ctx, seed=1)
    gc = sw.Case(ctx, gm, case, precision="fp16", guess="mlp")
    gc.attach_mlp(net)
    gc.autotune(reps=2)
    half = case.n_steps // 2
    gc.step(half)
    u, v, a, st = gc.get_state()
    gr = sw.Case(ctx, gm, case, precision="fp16", guess="mlp")
    gr.attach_mlp(net)
    gr.set_state(u, v, a, st)
    gr.step(case.n_steps - half)
    w = gr.waveforms(half, case.n_steps - half)
    assert _rel(w, ref[half:]) < 1e-6
    _, rel = gr.step_log(half, case.n_steps - half)
    assert np.all(rel <= 1e-8) and not gr.stats()["flags"] & 3
