"""Pins of the input-estimation oracle (oracle/inversion.py, Section 2):
the shifted design matrix by brute force; exact recovery of coefficients
when the records lie in the model's span (ERR = 0); stationarity and
minimality of the quadratic objective with noisy records; silent pairs;
a rank-deficient set of Green's functions; and the physical basis of the
method: the oracle march driven by sum_l c_jl p(t - l dT) gives exactly the
superposition of the delayed Green's records (linear, time-invariant,
started from rest)."""
import numpy as np

import casegen as cg
from oracle import inversion as inv
from oracle import march


def _random_G(seed, n=40, n_rec=2):
    return np.random.default_rng(seed).standard_normal((3, n, n_rec, 3))


def test_design_matches_brute_force():
    G = _random_G(1, n=12, n_rec=1)
    H = inv.design(G, 3, 4)
    for t in range(12):
        for i in range(3):
            for j in range(3):
                for l in range(4):
                    want = G[j, t - 3 * l, 0, i] if t >= 3 * l else 0.0
                    assert H[(t * 1 + 0) * 3 + i, j * 4 + l] == want


def test_fit_recovers_coefficients_in_span():
    G = _random_G(2)
    c_true = np.random.default_rng(3).standard_normal((3, 6))
    obs = (inv.design(G, 5, 6) @ c_true.reshape(-1)).reshape(40, 2, 3)
    c, U, e, used, rank = inv.fit(G, obs, 5, 6)
    assert rank == 18 and used == 6
    assert np.abs(c - c_true).max() <= 1e-10 * np.abs(c_true).max()
    assert e <= 1e-12


def test_fit_is_the_stationary_minimum():
    G = _random_G(4)
    rng = np.random.default_rng(5)
    obs = rng.standard_normal((40, 2, 3))
    c, _, e, _, _ = inv.fit(G, obs, 5, 6)
    J0 = inv.objective(G, obs, 5, c)
    h = 1e-6
    for _ in range(10):
        d = rng.standard_normal(c.shape)
        g = (inv.objective(G, obs, 5, c + h * d) - inv.objective(G, obs, 5, c - h * d)) / (2 * h)
        assert abs(g) <= 1e-6 * max(1.0, J0)
        assert inv.objective(G, obs, 5, c + 0.01 * d) >= J0
    assert 0.0 < e < 1.0


def test_silent_pairs_carry_no_weight():
    G = _random_G(6)
    obs = np.random.default_rng(7).standard_normal((40, 2, 3))
    obs[:, 1, 2] = 0.0
    w = inv.pair_weights(obs)
    assert w[1, 2] == 0.0 and np.all(w[0] > 0)
    c, _, e, used, _ = inv.fit(G, obs, 5, 6)
    assert used == 5 and np.isfinite(e)


def test_rank_deficient_green_functions():
    G = _random_G(8)
    G[1] = G[0]                         # two directions indistinguishable
    obs = np.random.default_rng(9).standard_normal((40, 2, 3))
    c, _, _, _, rank = inv.fit(G, obs, 5, 6)
    assert rank == 12
    # same objective as the dense least-squares solution on the same span
    H = inv.design(G, 5, 6)
    w = np.sqrt(np.broadcast_to(inv.pair_weights(obs)[None], obs.shape).reshape(-1))
    cl = np.linalg.lstsq(w[:, None] * H, w * obs.reshape(-1), rcond=None)[0]
    assert abs(inv.objective(G, obs, 5, c) - inv.objective(G, obs, 5, cl.reshape(3, 6))) <= 1e-9


def test_march_is_superposition_of_delayed_green_records():
    mesh = cg.box_mesh(40.0, 30.0, 30.0, 10.0)
    base = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=24, n_rec=1)
    S = march.build_system(mesh, base)
    stride, n = 4, 24
    G = []
    for v_in in cg.impulse_inputs(n, stride):
        r = march.run(S, base.dt, v_in, n, base.rec_node, solver="lu")
        G.append(r.rec_v)
    c = np.random.default_rng(10).standard_normal((3, 5))
    f = inv.input_waveform(c, cg.hann_impulse(n, stride), stride, n)
    direct = march.run(S, base.dt, f, n, base.rec_node, solver="lu").rec_v
    sup = (inv.design(np.array(G), stride, 5) @ c.reshape(-1)).reshape(direct.shape)
    assert np.abs(direct - sup).max() <= 1e-10 * np.abs(direct).max()
    # and the fit of those records recovers c with ERR ~ 0
    c2, _, e, _, _ = inv.fit(np.array(G), direct, stride, 5)
    assert e <= 1e-8
    assert np.abs(c2 - c).max() <= 1e-6 * np.abs(c).max()


def test_fit_events_takes_the_worst_event():
    """The model's misfit over events is its worst event's (Section 3):
    an event in the span of the model (ERR 0) never decides it, and each
    event's fit is the single-event fit."""
    rng = np.random.default_rng(12)
    G = rng.standard_normal((3, 60, 3, 3))
    in_span = (inv.design(G, 6, 10) @ rng.standard_normal(30)).reshape(60, 3, 3)
    noisy = in_span + 0.3 * rng.standard_normal(in_span.shape)
    other = rng.standard_normal((60, 3, 3))
    fits, emax, worst = inv.fit_events(G, [in_span, noisy, other], 6, 10)
    assert fits[0][2] < 1e-12
    assert worst == 2 and emax == fits[2][2] > fits[1][2] > 0
    single = inv.fit(G, noisy, 6, 10)
    assert np.array_equal(fits[1][0], single[0]) and fits[1][2] == single[2]
