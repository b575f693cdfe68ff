"""GPU parity of the learned initial guess against the FP64 oracle
(oracle/mlp.py): matrix-core FP16 inference, FP32 back-propagation, Adam,
the features of the guess (last increments, element-neighbour means, node
material) and the guess itself; the fallback on a bad network; and what a
network trained on the solver's own histories gains over quadratic
extrapolation on held-out cases."""
import numpy as np
import pytest

import casegen as cg
from oracle import mlp as om

pytestmark = pytest.mark.gpu

# FP16 weights and activations (11-bit significands) through two layers of
# 64 terms: the output error is a few 1e-3 of the output scale.
TOL_FP16 = 1e-2


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    th = om.init(seed)
    p = om.unpack(th)
    p["w3"] = rng.standard_normal(om.N_H) * scale
    p["b1"] = rng.standard_normal(om.N_H) * 0.1
    p["b2"] = rng.standard_normal(om.N_H) * 0.1
    p["b3"] = np.array([0.05])
    return om.pack(p)


def test_forward_matches_oracle(sw, ctx):
    import torch
    th = _theta(1)
    net = sw.Mlp(ctx, th)
    X = np.random.default_rng(2).uniform(-1, 1, (1000, 10))  # the guess's inputs are within [-1, 1]
    y = net.forward(torch.from_numpy(X).float()).cpu().numpy()
    ref = om.forward(th.astype(np.float32).astype(np.float64), X)
    assert np.abs(y - ref).max() <= TOL_FP16 * np.abs(ref).max()
    # ragged count (not a multiple of the 16-row passes) and a single row
    y7 = net.forward(torch.from_numpy(X[:7]).float()).cpu().numpy()
    np.testing.assert_allclose(y7, y[:7], rtol=0, atol=1e-6)
    assert net.forward(torch.from_numpy(X[:1]).float()).shape == (1,)


def test_gradient_matches_oracle(sw, ctx):
    import torch
    rng = np.random.default_rng(3)
    n = 1000
    S = np.zeros((n, 12))
    S[:, :10] = rng.uniform(-1, 1, (n, 10))
    S[:, 10] = rng.standard_normal(n) * 0.3
    S[:, 11] = rng.uniform(0.01, 2.0, n)
    th = _theta(4)
    th32 = th.astype(np.float32).astype(np.float64)
    S32 = S.astype(np.float32).astype(np.float64)
    net = sw.Mlp(ctx, th)
    g, loss = net.gradient(torch.from_numpy(S).float())
    gr = om.gradient(th32, S32[:, :10], S32[:, 10], S32[:, 11])
    lr = om.loss(th32, S32[:, :10], S32[:, 10], S32[:, 11])
    assert np.linalg.norm(g - gr) <= 1e-5 * np.linalg.norm(gr)
    assert abs(loss - lr) <= 1e-5 * lr
    # every parameter block carries gradient
    for name, sl in (("W1", slice(0, 640)), ("W2", slice(704, 4800)), ("w3", slice(4864, 4928))):
        assert np.abs(g[sl]).max() > 0, name


def test_adam_step_matches_oracle(sw, ctx):
    import torch
    # identical rows: every minibatch has the same gradient as the single row
    row = np.zeros((1, 12))
    row[0, :10] = np.linspace(-0.9, 0.8, 10)
    row[0, 10], row[0, 11] = 0.7, 1.3
    S = np.repeat(row, 64, 0)
    th = _theta(5)
    th32 = th.astype(np.float32).astype(np.float64)
    net = sw.Mlp(ctx, th)
    losses = net.train(torch.from_numpy(S).float(), steps=3, batch=32, lr=1e-3, seed=9)
    t, m, v = th32.copy(), np.zeros_like(th32), np.zeros_like(th32)
    for k in range(1, 4):
        g = om.gradient(t, row[:, :10], row[:, 10], row[:, 11])
        t, m, v = om.adam_step(t, m, v, g, k, 1e-3)
    p = net.params()
    assert np.abs(p - t).max() <= 1e-6 + 1e-5 * np.abs(t).max()
    assert losses[0] > 0


def _march_states(sw, ctx, mesh, case, n, guess, net=None, **kw):
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, guess=guess, **kw)
    if net is not None:
        gc.attach_mlp(net)
    states = [gc.get_state()[0]]
    for _ in range(n):
        gc.step(1)
        states.append(gc.get_state()[0])
    return gc, np.array(states)


def test_guess_features_and_network_match_oracle(sw, ctx):
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.15, seed=4)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=12, n_rec=2)
    th = _theta(6, scale=0.05)
    net = sw.Mlp(ctx, th)
    gc, U = _march_states(sw, ctx, mesh, case, 7, "mlp", net)
    x = gc.guess().cpu().numpy()
    du = np.diff(U, axis=0)                       # du^0 .. du^6
    n = mesh.n_nodes
    own = np.stack([du[-1 - k] for k in range(4)], 1)               # (n_dof, 4)
    nbr = np.stack([om.neighbour_mean(mesh.tet10, n, du[-1 - k].reshape(n, 3)).ravel() for k in range(4)], 1)
    vs, rho = om.node_material(mesh.tet10, n, case.mat, case.tet_mat)
    ref = om.guess(th.astype(np.float32).astype(np.float64), own, nbr, np.repeat(vs, 3), np.repeat(rho, 3))
    X, s = om.features(own, nbr, np.repeat(vs, 3), np.repeat(rho, 3))
    err = np.abs(x - ref)
    assert np.all(err <= TOL_FP16 * s + 1e-14 * np.abs(ref).max())
    # the untrained network gives exactly the quadratic extrapolation
    gz, U2 = _march_states(sw, ctx, mesh, case, 7, "mlp", sw.Mlp(ctx, om.init(3)))
    du2 = np.diff(U2, axis=0)
    p2 = 3 * du2[-1] - 3 * du2[-2] + du2[-3]
    assert np.abs(gz.guess().cpu().numpy() - p2).max() <= 1e-12 * np.abs(p2).max()


def test_bad_network_falls_back_and_stays_correct(sw, ctx):
    from oracle import march
    mesh = cg.box_mesh(40.0, 30.0, 30.0, 10.0)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=15, n_rec=1)
    ref = march.run_case(mesh, case, solver="lu")
    th = np.full(om.N_PARAM, np.nan)
    for prec in ("fp64", "mixed"):
        gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, guess="mlp", precision=prec)
        gc.attach_mlp(sw.Mlp(ctx, th))
        gc.step(15)
        st = gc.stats()
        assert st["flags"] & 4 and not st["flags"] & 3, st
        w = gc.waveforms()
        assert np.linalg.norm(w - ref.rec_v) <= 1e-6 * np.linalg.norm(ref.rec_v)


def test_mlp_guess_requires_network(sw, ctx):
    mesh = cg.box_mesh(30.0, 20.0, 20.0, 10.0)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=3, n_rec=1)
    gc = sw.Case(ctx, sw.Mesh(ctx, mesh), case, guess="mlp")
    with pytest.raises(sw.SwError, match="SW_ESTATE"):
        gc.step(1)


def _train_and_compare(sw, ctx, n_train=3, n_test=2, steps=60, size=(100.0, 100.0, 50.0), cell=5.0,
                       train_steps=1500):
    """Collect rows from training cases marched with quadratic extrapolation,
    train the network, then march held-out cases with each guess."""
    import torch
    base = cg.CONFIGS["batch300"]
    cfg = cg.BoxConfig("learn", size, cell, 25.0, base.amp, base.corr, (4.0,), 0.3, 0.005, steps, 4, 1000)
    mesh = cg.config_mesh(cfg)
    gm = sw.Mesh(ctx, mesh)
    rows = []
    for k in range(n_train):
        case = cg.make_case(mesh, cfg, seed=1000 + k)
        gc = sw.Case(ctx, gm, case, guess="poly", precision="mixed")
        gc.set_sampler(capacity=steps * 4096, per_step=4096, seed=11 + k)
        gc.step(steps)
        rows.append(gc.samples().clone())
    S = torch.cat(rows)
    net = sw.Mlp(ctx, om.init(1))
    losses = net.train(S, steps=train_steps, batch=4096, lr=2e-3, seed=5)
    res = {}
    for guess in ("poly", "mlp"):
        its = []
        for k in range(n_test):
            case = cg.make_case(mesh, cfg, seed=2000 + k)
            gc = sw.Case(ctx, gm, case, guess=guess, precision="mixed")
            if guess == "mlp":
                gc.attach_mlp(net)
            gc.step(steps)
            it, rel = gc.step_log()
            assert np.all(rel <= 1e-8) and gc.stats()["flags"] & 3 == 0
            its.append(it[8:])
        res[guess] = float(np.mean(np.concatenate(its)))
    return res, losses


def test_trained_network_gain_over_extrapolation(sw, ctx):
    """What the trained network gains over the method without it: on
    held-out models with a 4 Hz input (a regime where extrapolation from
    the last increments leaves a sizeable error), the learned guess needs
    fewer CG iterations per step than quadratic extrapolation (measured
    about 6 % fewer; asserted at least 2 %).  At 2 Hz on the batched
    workload's meshes extrapolation is already close and the network does
    not gain; the benchmark's guess study reports that case."""
    res, losses = _train_and_compare(sw, ctx)
    print(f"learned guess: CG iterations/step poly {res['poly']:.2f} -> mlp {res['mlp']:.2f}; "
          f"training loss {losses[:20].mean():.3e} -> {losses[-20:].mean():.3e}", flush=True)
    assert losses[-20:].mean() < 0.5 * losses[:20].mean()
    assert res["mlp"] <= res["poly"] * 0.98


def _constant_net(value):
    """A network whose output is the constant `value` (every weight zero but
    the output bias): its correction is w = value * s per DOF, a nonlinear
    function of the history (s = the largest magnitude of the DOF's last
    increments and their neighbour means) and so outside their span, known
    to FP64 rounding on both sides."""
    p = om.unpack(np.zeros(om.N_PARAM))
    p["b3"] = np.array([value])
    return om.pack(p)


def test_projection_with_network_direction_matches_oracle(sw, ctx):
    """SW_GUESS_PROJ_MLP: the Galerkin projection over the last L increments
    and the network's correction w.  The GPU guess equals the oracle's
    projection (oracle/guess.py) over the same increments and the oracle
    network's correction (energy norm, 1e-6), and it is no worse in the
    energy norm than the projection over the increments alone (a larger
    Galerkin space)."""
    from scipy.sparse.linalg import spsolve

    from oracle import guess as og
    from oracle import march
    mesh = cg.box_mesh(60.0, 40.0, 40.0, 10.0, jitter=0.15, seed=4)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=16, n_rec=2)
    th = _constant_net(0.3)
    L = 4
    gc, U = _march_states(sw, ctx, mesh, case, 9, "proj_mlp", sw.Mlp(ctx, th), precision="mixed", proj_dim=L)
    x = gc.guess().cpu().numpy()
    u, v, a, step = gc.get_state()
    S = march.build_system(mesh, case)
    A = march.step_matrix(S, case.dt).tocsr()
    b = case.v_in[step + 1] @ S.Fb - S.K @ u + S.C @ v + S.M @ (a + (4.0 / case.dt) * v)
    du = np.diff(U, axis=0)
    n = mesh.n_nodes
    own = np.stack([du[-1 - k] for k in range(4)], 1)
    nbr = np.stack([om.neighbour_mean(mesh.tet10, n, du[-1 - k].reshape(n, 3)).ravel() for k in range(4)], 1)
    vs, rho = om.node_material(mesh.tet10, n, case.mat, case.tet_mat)
    p2 = 3 * own[:, 0] - 3 * own[:, 1] + own[:, 2]
    w = om.guess(th.astype(np.float32).astype(np.float64), own, nbr, np.repeat(vs, 3), np.repeat(rho, 3)) - p2
    X = du[-L:].T
    xs = spsolve(A.tocsc(), b)

    def energy(e):
        return float(np.sqrt(e @ (A @ e)))

    x_proj = og.projection(A, X, b)
    x_or = og.projection(A, np.column_stack([X, w]), b)
    e_gpu, e_proj, e_or = energy(x - xs), energy(x_proj - xs), energy(x_or - xs)
    print(f"energy error: projection {e_proj:.3e}, with the network's direction {e_or:.3e} (oracle), "
          f"{e_gpu:.3e} (GPU); GPU vs oracle guess {energy(x - x_or) / energy(x_or):.2e}", flush=True)
    assert energy(x - x_or) <= 1e-6 * energy(x_or)
    assert e_gpu <= e_proj * (1 + 1e-9)
    assert e_or < e_proj  # the direction is outside the increments' span


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_projection_with_network_march_matches_oracle(sw, ctx, precision):
    from oracle import march
    cfg = cg.CONFIGS["small"]
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg)
    ref = march.run_case(mesh, case, solver="lu").rec_v
    gm = sw.Mesh(ctx, mesh)
    net = sw.Mlp(ctx, _theta(6, scale=0.05))
    gc = sw.Case(ctx, gm, case, precision=precision, guess="proj_mlp", proj_dim=6)
    gc.attach_mlp(net)
    gc.step(case.n_steps)
    it, rel = gc.step_log()
    err = np.linalg.norm(gc.waveforms() - ref) / np.linalg.norm(ref)
    assert err < 1e-6 and np.all(rel <= 1e-8) and not gc.stats()["flags"] & 3
    # batched lanes take the same guesses as the case alone
    lanes = [sw.Case(ctx, gm, case, precision="mixed", guess=g, proj_dim=6) for g in ("proj_mlp", "proj")]
    lanes[0].attach_mlp(net)
    sw.Batch(ctx, lanes).step(case.n_steps)
    if precision == "mixed":
        assert np.abs(lanes[0].step_log()[0] - it).max() <= 1
        assert np.linalg.norm(lanes[0].waveforms() - gc.waveforms()) <= 1e-7 * np.linalg.norm(ref)
    assert np.linalg.norm(lanes[0].waveforms() - ref) <= 1e-6 * np.linalg.norm(ref)


def test_projection_with_network_requires_network_and_valid_dim(sw, ctx):
    mesh = cg.box_mesh(30.0, 20.0, 20.0, 10.0)
    case = cg.make_case(mesh, cg.CONFIGS["small"], n_steps=3, n_rec=1)
    gm = sw.Mesh(ctx, mesh)
    gc = sw.Case(ctx, gm, case, guess="proj_mlp")
    with pytest.raises(sw.SwError, match="SW_ESTATE"):
        gc.step(1)
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, case, guess="proj_mlp", proj_dim=16)


def test_learned_guess_on_heldout_c3_models(sw, ctx):
    """The learned-guess workload's shape: a network trained on histories of
    16 models of the batched workload's 200 m mesh (2 Hz input, seeds 500
    on), then two held-out models of the 300 m mesh (seeds 2000, 2001)
    marched 100 steps from rest with extrapolation, the network's guess, the
    projection, and the projection with the network's direction.  Measured
    (64 models): the network alone needs under 1 % fewer CG iterations than
    extrapolation, although from step 60 on its guesses have a 2-3x
    smaller residual;
    projection with the network's direction 36 % fewer (the projection's
    own gain: the network's direction adds nothing measurable to it).
    Asserted: the learned guess needs at least 5 % fewer iterations than
    extrapolation, the network alone is not worse than extrapolation (to
    0.5 %), and
    the network's direction never costs the projection more than rounding."""
    import torch
    base = cg.CONFIGS["batch200"]
    tcfg = cg.BoxConfig("train", base.box, base.cell, base.h0, base.amp, base.corr, base.freqs, base.t0, base.dt,
                        150, 4, 500)
    tmesh = cg.config_mesh(tcfg)
    gtm = sw.Mesh(ctx, tmesh)
    lanes = []
    for k in range(16):
        c = sw.Case(ctx, gtm, cg.make_case(tmesh, tcfg, seed=500 + k), precision="mixed", guess="poly")
        c.set_sampler(capacity=150 * 4096, per_step=4096, seed=k)
        lanes.append(c)
    sw.Batch(ctx, lanes).step(150)
    S = torch.cat([c.samples() for c in lanes])
    del lanes
    net = sw.Mlp(ctx, seed=1)
    losses = net.train(S, steps=3000, batch=8192, lr=2e-3, seed=5)
    del S
    torch.cuda.empty_cache()
    cfg = cg.CONFIGS["batch300"]
    mesh = cg.config_mesh(cfg)
    gm = sw.Mesh(ctx, mesh)
    models = [cg.make_case(mesh, cfg, seed=2000 + k, n_steps=100) for k in range(2)]
    its = {}
    for g in ("poly", "mlp", "proj", "proj_mlp"):
        lanes = [sw.Case(ctx, gm, m, precision="mixed", guess=g, proj_dim=6) for m in models]
        if g in ("mlp", "proj_mlp"):
            for lane in lanes:
                lane.attach_mlp(net)
        sw.Batch(ctx, lanes).step(100)
        for lane in lanes:
            _, rel = lane.step_log()
            assert np.all(rel <= 1e-8) and not lane.stats()["flags"] & 3
        its[g] = float(np.mean([lane.step_log()[0].mean() for lane in lanes]))
    print("held-out 300 m models, CG iterations/step: " + ", ".join(f"{k} {v:.2f}" for k, v in its.items()) +
          f"; training loss {losses[:20].mean():.2e} -> {losses[-20:].mean():.2e}", flush=True)
    assert losses[-20:].mean() < 0.2 * losses[:20].mean()
    assert its["proj_mlp"] <= 0.95 * its["poly"]
    assert its["mlp"] <= 1.005 * its["poly"]
    assert its["proj_mlp"] <= 1.01 * its["proj"]
