"""CG iterations replayed from captured HIP graphs (the default) against the
same solves with every kernel launched directly: a graph of two iterations
is replayed many times per solve, with the step's own eager kernels (right-
hand side, true residuals, refinement updates, Newmark update) and host
synchronisations between the replays.  Every step's CG iteration count must
be the same (up to one, from the rounding order of atomic sums), the
receiver waveforms agree to rounding, and both match the oracle's exact
solves; for FP64 PCG, mixed precision, the flexible outer CG
and a batch."""
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
def setup(sw):
    mesh = cg.config_mesh(cg.CONFIGS["small"])
    case = cg.make_case(mesh, cg.CONFIGS["small"])
    ref = march.run_case(mesh, case, solver="lu").rec_v
    ctx = sw.Context(0)
    return mesh, case, ref, ctx, sw.Mesh(ctx, mesh)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision,guess", [("fp64", "zero"), ("mixed", "proj"), ("mixed", "poly"),
                                             ("flex", "proj")])
def test_graph_replays_match_direct_launches(sw, setup, precision, guess):
    mesh, case, ref, ctx, gm = setup
    out = {}
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        gc = sw.Case(ctx, gm, case, precision=precision, guess=guess)
        gc.step(case.n_steps)
        it, rel = gc.step_log()
        out[graphs] = (gc.waveforms(), it, rel, gc.stats())
    ctx.set_graphs(True)
    (w0, it0, _, st0), (w1, it1, rel1, st1) = out[False], out[True]
    # the same arithmetic up to the order of the atomic sums, which varies
    # from run to run: iteration counts equal up to one (a step may cross
    # its threshold), waveforms equal to well within the solve tolerance
    # (measured 1e-9 relative and below)
    assert np.abs(it0 - it1).max() <= 1 and abs(int(it0.sum()) - int(it1.sum())) <= 2, (it0, it1)
    assert _rel(w1, w0) < 1e-7
    assert _rel(w1, ref) < 1e-6 and np.all(rel1 <= 1e-8) and not st1["flags"] & 3


def test_batch_graph_replays_match_direct_launches(sw, setup):
    mesh, case, ref, ctx, gm = setup
    res = {}
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        lanes = [sw.Case(ctx, gm, case, precision="mixed", guess=g) for g in ("proj", "poly", "zero")]
        sw.Batch(ctx, lanes).step(case.n_steps)
        res[graphs] = [(l.waveforms(), l.step_log()[0]) for l in lanes]
    ctx.set_graphs(True)
    for (w0, it0), (w1, it1) in zip(res[False], res[True]):
        assert np.abs(it0 - it1).max() <= 1
        assert _rel(w1, w0) < 1e-7 and _rel(w1, ref) < 1e-6
