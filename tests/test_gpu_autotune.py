"""Set-up-time schedule tuning of the persistent FP32 passes
(sw_batch_autotune: work-item order x workgroups per compute unit;
sw_case_autotune: workgroups per compute unit): every candidate is timed,
the fastest is kept, and the march that follows gives the oracle's
waveforms and, to well within the solve tolerance, those of an untuned
batch (another schedule adds the element results in another order, so the
iterates differ by rounding: measured 1e-9 relative)."""
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
    ctx = sw.Context(0)
    small = cg.config_mesh(cg.CONFIGS["small"])
    other = cg.box_mesh(60.0, 40.0, 40.0, 5.0, jitter=0.2, seed=5)
    return ctx, small, other


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_batch_autotune_then_march(sw, setup):
    ctx, small, other = setup
    case = cg.make_case(small, cg.CONFIGS["small"], n_steps=30)
    ref = march.run_case(small, case, solver="lu").rec_v
    c2 = cg.make_case(other, cg.CONFIGS["small"], n_steps=30, n_rec=2)
    gs, go = sw.Mesh(ctx, small), sw.Mesh(ctx, other)
    runs = {}
    for tuned in (False, True):
        lanes = [sw.Case(ctx, gs, case, precision="mixed", guess="proj"),
                 sw.Case(ctx, go, c2, precision="mixed", guess="proj"),
                 sw.Case(ctx, gs, case, precision="mixed", guess="poly")]
        b = sw.Batch(ctx, lanes)
        if tuned:
            choice, ms = b.autotune(reps=3)
            print(f"batch schedule {choice}, candidate pass times (ms) {np.round(ms, 4).tolist()}", flush=True)
            assert 0 <= choice < 4 and np.all(np.isfinite(ms)) and np.all(ms > 0)
            assert ms[choice] == ms.min()
        b.step(case.n_steps)
        runs[tuned] = [(l.waveforms(), l.step_log()[0], l.stats()) for l in lanes]
    for (w0, it0, _), (w1, it1, st1) in zip(runs[False], runs[True]):
        assert _rel(w1, w0) < 1e-7 and np.abs(it0 - it1).max() <= 2
        assert st1["max_true_rel_res"] <= 1e-8 and not st1["flags"] & 3
    for k in (0, 2):
        assert _rel(runs[True][k][0], ref) < 1e-6


def test_case_autotune_then_march(sw, setup):
    ctx, small, _ = setup
    case = cg.make_case(small, cg.CONFIGS["small"], n_steps=30)
    ref = march.run_case(small, case, solver="lu").rec_v
    gc = sw.Case(ctx, sw.Mesh(ctx, small), case, precision="mixed", guess="proj")
    choice, ms = gc.autotune(reps=3)
    assert 0 <= choice < 3 and np.all(ms > 0) and ms[choice] == ms.min()
    gc.step(case.n_steps)
    assert _rel(gc.waveforms(), ref) < 1e-6 and gc.stats()["max_true_rel_res"] <= 1e-8


def test_autotune_rejects_bad_requests(sw, setup):
    ctx, small, _ = setup
    case = cg.make_case(small, cg.CONFIGS["small"], n_steps=2)
    gm = sw.Mesh(ctx, small)
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, case, precision="fp64").autotune()
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, case, precision="mixed").autotune(reps=0)
