"""GPU input estimation and misfit (Section 2) against the oracle
(oracle/inversion.py): coefficients, rank and ERR on seeded records,
exact recovery when the records lie in the model's span, the whole method
on a small model (Green's records from GPU runs vs the oracle's own exact
march), selection of the true model among candidates, and bad arguments."""
import numpy as np
import pytest

import casegen as cg
from oracle import inversion as inv
from oracle import march

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def test_fit_matches_oracle_on_seeded_records(sw, ctx):
    rng = np.random.default_rng(1)
    G = rng.standard_normal((3, 200, 5, 3))
    obs = rng.standard_normal((200, 5, 3))
    obs[:, 4, 1] = 0.0                          # a silent pair
    c, e, used, rank = sw.fit_input(ctx, [_dev(g) for g in G], _dev(obs), 10, 15)
    c_or, _, e_or, used_or, rank_or = inv.fit(G, obs, 10, 15)
    assert used == used_or == 14 and rank == rank_or == 45
    assert np.abs(c - c_or).max() <= 1e-9 * np.abs(c_or).max()
    assert abs(e - e_or) <= 1e-10


def test_fit_events_matches_oracle_on_seeded_records(sw, ctx):
    """Per-event fits and the worst event through sw_fit_events against the
    oracle's fit of each event: one event in the model's span (ERR 0), two
    not, one with a silent pair."""
    rng = np.random.default_rng(6)
    G = rng.standard_normal((3, 160, 4, 3))
    ev = [(inv.design(G, 8, 12) @ rng.standard_normal(36)).reshape(160, 4, 3),
          rng.standard_normal((160, 4, 3)), rng.standard_normal((160, 4, 3))]
    ev[2][:, 1, 2] = 0.0
    fits, emax, worst = sw.fit_events(ctx, [_dev(g) for g in G], [_dev(o) for o in ev], 8, 12)
    fits_or, emax_or, worst_or = inv.fit_events(G, ev, 8, 12)
    assert worst == worst_or and worst != 0
    assert abs(emax - emax_or) <= 1e-10 and emax == max(f[1] for f in fits)
    assert fits[0][1] <= 1e-12
    for (c, e, used, rank), (c_or, _, e_or, used_or, rank_or) in zip(fits, fits_or):
        assert used == used_or and rank == rank_or
        assert np.abs(c - c_or).max() <= 1e-9 * np.abs(c_or).max()
        assert abs(e - e_or) <= 1e-10


def test_fit_recovers_coefficients_in_span(sw, ctx):
    rng = np.random.default_rng(2)
    G = rng.standard_normal((3, 120, 4, 3))
    c_true = rng.standard_normal((3, 8))
    obs = (inv.design(G, 12, 8) @ c_true.reshape(-1)).reshape(120, 4, 3)
    c, e, _, rank, U = sw.fit_input(ctx, [_dev(g) for g in G], _dev(obs), 12, 8, return_response=True)
    assert rank == 24
    assert np.abs(c - c_true).max() <= 1e-9 * np.abs(c_true).max()
    assert e <= 1e-12
    assert np.abs(U.cpu().numpy() - obs).max() <= 1e-10 * np.abs(obs).max()


def _green_runs(sw, ctx, gm, case, n, stride):
    """Green's records of one model: three lanes driven by the impulse along
    x1, x2, x3, marched together."""
    lanes = []
    for v_in in cg.impulse_inputs(n, stride):
        c = cg.Case(mat=case.mat, tet_mat=case.tet_mat, rec_node=case.rec_node, v_in=v_in, dt=case.dt,
                    n_steps=n, ray_alpha=case.ray_alpha, ray_beta=case.ray_beta, meta={})
        lanes.append(sw.Case(ctx, gm, c, precision="mixed", guess="proj"))
    sw.Batch(ctx, lanes).step(n)
    return lanes


def test_method_on_a_model_matches_oracle(sw, ctx):
    mesh = cg.box_mesh(40.0, 30.0, 30.0, 10.0)
    n, stride, L = 40, 4, 8
    base = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=n, n_rec=1)
    c_true = np.random.default_rng(3).standard_normal((3, L))
    f = inv.input_waveform(c_true, cg.hann_impulse(n, stride), stride, n)
    gm = sw.Mesh(ctx, mesh)
    lanes = _green_runs(sw, ctx, gm, base, n, stride)
    src = cg.Case(mat=base.mat, tet_mat=base.tet_mat, rec_node=base.rec_node, v_in=f, dt=base.dt, n_steps=n,
                  ray_alpha=base.ray_alpha, ray_beta=base.ray_beta, meta={})
    rec = sw.Case(ctx, gm, src, precision="mixed", guess="proj")
    rec.step(n)
    import torch
    obs = torch.from_numpy(rec.waveforms()).cuda()
    c, e, used, rank = sw.fit_input(ctx, [torch.from_numpy(l.waveforms()).cuda() for l in lanes], obs, stride, L)
    # the oracle's own march: Green's records and observation
    S = march.build_system(mesh, base)
    G_or = np.array([march.run(S, base.dt, v, n, base.rec_node, solver="lu").rec_v
                     for v in cg.impulse_inputs(n, stride)])
    obs_or = march.run(S, base.dt, f, n, base.rec_node, solver="lu").rec_v
    c_or, _, e_or, _, rank_or = inv.fit(G_or, obs_or, stride, L)
    print(f"fit: ERR gpu {e:.2e} oracle {e_or:.2e}; |c - c_true| gpu {np.abs(c - c_true).max():.2e} "
          f"oracle {np.abs(c_or - c_true).max():.2e}; rank {rank}/{rank_or}", flush=True)
    assert rank == rank_or == 3 * L
    assert np.abs(c_or - c_true).max() <= 1e-6 * np.abs(c_true).max()
    assert np.abs(c - c_or).max() <= 1e-4 * np.abs(c_true).max()
    assert e <= 1e-5 and e_or <= 1e-8


def test_true_model_has_the_smallest_misfit(sw, ctx):
    """Records of a model driven by a Ricker input; the input is estimated
    for that model and for two other candidates (other interface fields):
    the true model reproduces the records best (the selection principle of
    Section 2)."""
    import torch
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0)
    base = cg.CONFIGS["small"]
    cfg = cg.BoxConfig("sel", (60.0, 40.0, 40.0), 10.0, 20.0, (6.0, 12.0), (30.0, 60.0), base.freqs, base.t0,
                       base.dt, 60, 2, 70)
    n, stride, L = 60, 4, 15
    cands = [cg.make_case(mesh, cfg, seed=70 + k, n_rec=2) for k in range(3)]
    gm = sw.Mesh(ctx, mesh)
    rec = sw.Case(ctx, gm, cands[0], precision="mixed", guess="proj")
    rec.step(n)
    obs = torch.from_numpy(rec.waveforms()).cuda()
    errs = []
    for cand in cands:
        lanes = _green_runs(sw, ctx, gm, cand, n, stride)
        _, e, _, _ = sw.fit_input(ctx, [torch.from_numpy(l.waveforms()).cuda() for l in lanes], obs, stride, L)
        errs.append(e)
    print("ERR of the candidates (true first):", errs, flush=True)
    # (a Ricker is only approximately a sum of 15 Hann pulses, and ERR weighs
    # every component by its own norm, so the true model's ERR is not zero)
    assert errs[0] < 0.5 * min(errs[1:])


def test_fit_rejects_bad_arguments(sw, ctx):
    G = [_dev(np.zeros((30, 2, 3))) for _ in range(3)]
    obs = _dev(np.ones((30, 2, 3)))
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.fit_input(ctx, G, obs, 7, 2)        # 30 steps not a multiple of 7
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.fit_input(ctx, G, obs, 5, 7)        # more shifts than blocks


def test_events_reuse_green_records(sw, ctx):
    """Several events recorded on the true model (different inputs): the
    Green's records of each candidate are computed once and every event is
    fitted against them; the true model has the smallest worst-event ERR,
    and each event's fit matches a direct sw_fit_input call."""
    import torch
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0)
    base = cg.CONFIGS["small"]
    cfg = cg.BoxConfig("ev", (60.0, 40.0, 40.0), 10.0, 20.0, (6.0, 12.0), (30.0, 60.0), base.freqs, base.t0,
                       base.dt, 60, 2, 80)
    n, stride, L = 60, 2, 30          # a finer impulse basis: the events go up to 3 Hz
    cands = [cg.make_case(mesh, cfg, seed=80 + k, n_rec=2) for k in range(3)]
    gm = sw.Mesh(ctx, mesh)
    events = []
    for k, (freqs, d) in enumerate((((2.0,), 0), ((1.5,), 1), ((3.0,), 2))):
        c = cands[0]
        v = cg.incident_velocity(n, c.dt, freqs, 0.45, direction=d)
        ev = cg.Case(mat=c.mat, tet_mat=c.tet_mat, rec_node=c.rec_node, v_in=v, dt=c.dt, n_steps=n,
                     ray_alpha=c.ray_alpha, ray_beta=c.ray_beta, meta={})
        r = sw.Case(ctx, gm, ev, precision="mixed", guess="proj")
        r.step(n)
        events.append(torch.from_numpy(r.waveforms()).cuda())
    worst = []
    for cand in cands:
        green = [torch.from_numpy(l.waveforms()).cuda() for l in _green_runs(sw, ctx, gm, cand, n, stride)]
        fits, w, _ = sw.fit_events(ctx, green, events, stride, L)
        single = sw.fit_input(ctx, green, events[1], stride, L)
        assert abs(fits[1][1] - single[1]) <= 1e-14 and np.array_equal(fits[1][0], single[0])
        worst.append(w)
    print("worst-event ERR of the candidates (true first):", worst, flush=True)
    assert worst[0] < 0.5 * min(worst[1:])
