"""Receiver waveforms of the benchmarked path (FP32 inner CG inside FP64
refinement, projection guess over 6 increments; batches of lanes where the
workload is batched) against the oracle's records at the workloads' full
sizes (tests/golden/*.npz, written by tests/golden/make_golden.py with the
assembled FP64 oracle, oracle/bsr.py, every step solved to a true relative
residual of 1e-12):

* the batched uneven workload: one model on each of the 200, 300 and
  400 m meshes (0.81 / 1.80 / 3.19 M DOF), 240 steps from rest, and two
  held-out models of the learned-guess workload (300 m mesh) marched with
  the learned guess, all five as one batch;
* the large single case (39.07 M DOF) over a window of 6 steps;
* three sampled models of the full sweep (19.8 M DOF each) as one batch over
  a window of 6 steps.

The windows start from a seeded smooth velocity field (every element in
motion) with the input near its peak.  Each case runs twice: at the
benchmark's relative residual 1e-8 and at 1e-11.  The difference from the
oracle is the solve tolerance carried into the waveforms, so it must fall
with the tolerance (by at least 30x from 1e-8 to 1e-11) and be within 1e-6
relative L2 at 1e-11 (the discretisation and the arithmetic are the
oracle's).  At 1e-8 the bound is stated per workload (TOL_BENCH): from rest
the waveforms meet 1e-6; from the rough initial fields of the windows the
error at 1e-8 is a few 1e-5 (measured 3.6e-5 on the large case, 8e-5 on a
sweep model), the relative residual amplified by the conditioning of the
step operator on the field's slow components."""
import os
import sys

import numpy as np
import pytest

import casegen as cg

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from recipes import RECIPES, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-6          # relative L2 against the oracle at rtol 1e-11
# relative L2 against the oracle at the benchmark's rtol 1e-8, per workload
TOL_BENCH = {"c2": 1e-6, "c3": 1e-6, "c1": 1e-4, "c4": 3e-4}


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle record {name}.npz not generated")
    return np.load(path)


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    import torch
    torch.cuda.empty_cache()
    return sw.Context(0)


def _lane(sw, ctx, gm, name, mesh, guess="proj", net=None, rtol=1e-8):
    _, case, u0, v0, a0, step0 = inputs(name, mesh)
    c = sw.Case(ctx, gm, case, rtol=rtol, precision="mixed", guess=guess, proj_dim=6)
    if net is not None:
        c.attach_mlp(net)
    c.set_state(u=u0, v=v0, a=a0, step=step0)
    return c


def _check_pair(name, bench, tight):
    """bench: the lane marched at rtol 1e-8, tight: at 1e-11."""
    e8 = _check(name, bench, TOL_BENCH[name[:2]], 1e-8)
    e11 = _check(name, tight, TOL, 1e-11)
    assert e11 <= e8 / 30.0, (name, e8, e11)


def _check(name, lane, tol, rtol):
    g = _golden(name)
    n = RECIPES[name]["steps"]
    step0 = RECIPES[name].get("step0", 0)
    keep = g["receivers"]
    w = lane.waveforms(step0, n)[:, keep]
    ref = g["rec_v"]
    err = np.linalg.norm(w - ref) / np.linalg.norm(ref)
    worst = np.linalg.norm(w - ref, axis=0).max() / np.linalg.norm(ref, axis=0).max()
    st = lane.stats()
    _, rel = lane.step_log(step0, n)
    print(f"{name} at rtol {rtol:g}: waveform rel L2 vs oracle {err:.2e} (worst receiver {worst:.2e}), "
          f"CG iterations {st['cg_iters'] / max(st['steps'], 1):.1f}/step, worst true residual {rel.max():.2e}",
          flush=True)
    assert err <= tol, (name, rtol, err)
    assert st["steps"] == n and np.all(rel <= rtol) and not st["flags"] & 3, (name, st)
    return err


def test_batched_workload_against_oracle(sw, ctx):
    """The five 100 m deep models (three mesh sizes) as one batch, 240 steps
    from rest; the two held-out models use the learned guess (the
    network's initial parameters: its zero output layer makes the guess the
    extrapolation, through the network's kernels)."""
    names = ["c2_200m_seed1000", "c2_300m_seed1001", "c2_400m_seed1002", "c3_300m_seed2000",
             "c3_300m_seed2001"]
    for n in names:
        _golden(n)
    meshes, gms, lanes = {}, {}, []
    net = sw.Mlp(ctx, seed=1)
    for n in names:
        cfg_name = RECIPES[n]["config"]
        if cfg_name not in meshes:
            meshes[cfg_name] = cg.config_mesh(cg.CONFIGS[cfg_name])
            gms[cfg_name] = sw.Mesh(ctx, meshes[cfg_name])
        guess, nn = ("mlp", net) if n.startswith("c3") else ("proj", None)
        for rtol in (1e-8, 1e-11):
            lanes.append(_lane(sw, ctx, gms[cfg_name], n, meshes[cfg_name], guess, nn, rtol))
    b = sw.Batch(ctx, lanes)
    b.step(RECIPES[names[0]]["steps"])
    for k, n in enumerate(names):
        _check_pair(n, lanes[2 * k], lanes[2 * k + 1])
    st = b.stats()
    assert [s["steps"] for s in st] == [lane.stats()["steps"] for lane in lanes]


def test_large_case_window_against_oracle(sw, ctx):
    name = "c1_window"
    _golden(name)
    mesh = cg.config_mesh(cg.CONFIGS["large"])
    gm = sw.Mesh(ctx, mesh)
    lanes = [_lane(sw, ctx, gm, name, mesh, rtol=rtol) for rtol in (1e-8, 1e-11)]
    for lane in lanes:
        lane.step(RECIPES[name]["steps"])
    _check_pair(name, *lanes)


def test_sweep_models_window_against_oracle(sw, ctx):
    names = ["c4_seed3000_window", "c4_seed3500_window", "c4_seed3999_window"]
    for n in names:
        _golden(n)
    mesh = cg.config_mesh(cg.CONFIGS["sweep"])
    gm = sw.Mesh(ctx, mesh)
    lanes = [_lane(sw, ctx, gm, n, mesh, rtol=rtol) for n in names for rtol in (1e-8, 1e-11)]
    sw.Batch(ctx, lanes).step(RECIPES[names[0]]["steps"])
    for k, n in enumerate(names):
        _check_pair(n, lanes[2 * k], lanes[2 * k + 1])
