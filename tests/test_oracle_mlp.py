"""Pins of the initial-guess network oracle: back-propagation against
central finite differences, the untrained network reproducing quadratic
extrapolation, hand-set weights realising a known function, hidden-unit
permutation invariance (catches transposed weight blocks), and Adam against
its closed form on a scalar."""
import numpy as np
import pytest

from oracle import mlp


def _data(n=64, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    t = rng.standard_normal(n)
    w = rng.uniform(0.1, 2.0, n)
    return X, t, w


def _theta(seed=1):
    rng = np.random.default_rng(seed)
    th = mlp.init(seed)
    p = mlp.unpack(th)
    p["w3"] = rng.standard_normal(mlp.N_H) * 0.3
    p["b1"] = rng.standard_normal(mlp.N_H) * 0.1
    p["b2"] = rng.standard_normal(mlp.N_H) * 0.1
    p["b3"] = np.array([0.2])
    return mlp.pack(p)


def test_param_count():
    assert mlp.N_PARAM == 4929


def test_gradient_matches_central_differences():
    X, t, w = _data()
    th = _theta()
    g = mlp.gradient(th, X, t, w)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(mlp.N_PARAM, 200, replace=False), [mlp.N_PARAM - 1, 0, 700, 4800]])
    h = 1e-6
    for j in idx:
        e = np.zeros(mlp.N_PARAM)
        e[j] = h
        fd = (mlp.loss(th + e, X, t, w) - mlp.loss(th - e, X, t, w)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-8, (j, fd, g[j])


def test_untrained_network_is_quadratic_extrapolation():
    rng = np.random.default_rng(5)
    own, nbr = rng.standard_normal((50, 4)), rng.standard_normal((50, 4))
    vs, rho = rng.uniform(150, 500, 50), rng.uniform(1800, 2000, 50)
    g = mlp.guess(mlp.init(7), own, nbr, vs, rho)
    np.testing.assert_allclose(g, 3 * own[:, 0] - 3 * own[:, 1] + own[:, 2], rtol=1e-15, atol=1e-15)
    # zero history gives zero guess
    assert np.all(mlp.guess(mlp.init(7), 0 * own, 0 * nbr, vs, rho) == 0)


def test_hand_set_network_realises_identity_of_first_input():
    # y = relu(x0) - relu(-x0) = x0 through two ReLU layers
    p = mlp.unpack(np.zeros(mlp.N_PARAM))
    p["W1"][0, 0], p["W1"][1, 0] = 1.0, -1.0
    p["W2"][0, 0], p["W2"][1, 1] = 1.0, 1.0
    p["w3"][0], p["w3"][1] = 1.0, -1.0
    th = mlp.pack(p)
    X = np.random.default_rng(0).standard_normal((20, mlp.N_IN))
    np.testing.assert_allclose(mlp.forward(th, X), X[:, 0], atol=1e-15)
    own = np.random.default_rng(1).standard_normal((20, 4))
    nbr = np.zeros((20, 4))
    g = mlp.guess(th, own, nbr, np.full(20, 150.0), np.full(20, 1800.0))
    np.testing.assert_allclose(g, 3 * own[:, 0] - 3 * own[:, 1] + own[:, 2] + own[:, 0], atol=1e-13)


def test_hidden_unit_permutation_invariance():
    th = _theta(4)
    p = mlp.unpack(th)
    rng = np.random.default_rng(9)
    P1, P2 = rng.permutation(mlp.N_H), rng.permutation(mlp.N_H)
    q = {"W1": p["W1"][P1], "b1": p["b1"][P1], "W2": p["W2"][P2][:, P1], "b2": p["b2"][P2], "w3": p["w3"][P2],
         "b3": p["b3"]}
    X, _, _ = _data(30, 2)
    np.testing.assert_allclose(mlp.forward(mlp.pack(q), X), mlp.forward(th, X), rtol=1e-12, atol=1e-12)


def test_adam_closed_form_first_steps():
    # first step moves every parameter by lr * sign(g) (bias correction)
    th = np.zeros(3)
    g = np.array([2.0, -0.5, 1e-3])
    th1, m, v = mlp.adam_step(th, np.zeros(3), np.zeros(3), g, 1, 0.01)
    np.testing.assert_allclose(th1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # constant gradient: the normalised step stays lr * sign(g)
    th2, m, v = mlp.adam_step(th1, m, v, g, 2, 0.01)
    np.testing.assert_allclose(th2 - th1, -0.01 * np.sign(g), rtol=1e-5)


def test_neighbour_mean_preserves_constants_and_linears_on_uniform_grid():
    import casegen as cg
    m = cg.box_mesh(30.0, 20.0, 20.0, 10.0)
    n = m.n_nodes
    c = np.full((n, 3), 2.5)
    np.testing.assert_allclose(mlp.neighbour_mean(m.tet10, n, c), c, rtol=1e-15)
    # a single element: every node gets the element mean
    one = np.arange(10)
    v = np.random.default_rng(0).standard_normal((10, 1))
    np.testing.assert_allclose(mlp.neighbour_mean(one[None], 10, v), np.full((10, 1), v.mean()), rtol=1e-14)
    vs, rho = mlp.node_material(m.tet10, n, cg.material_table(), np.zeros(m.n_tets, np.uint8))
    assert np.allclose(vs, 150.0) and np.allclose(rho, 1800.0)


@pytest.mark.parametrize("s_zero", [True, False])
def test_features_normalisation(s_zero):
    own = np.zeros((3, 4)) if s_zero else np.array([[1.0, -4.0, 2.0, 0.5]] * 3)
    nbr = np.zeros((3, 4)) if s_zero else np.array([[0.0, 1.0, -8.0, 0.0]] * 3)
    X, s = mlp.features(own, nbr, np.full(3, 500.0), np.full(3, 2000.0))
    if s_zero:
        assert np.all(s == 0) and np.all(X[:, :8] == 0)
    else:
        # backward differences of orders 0..3, by hand, over s = 8
        assert np.all(s == 8.0)
        own_d = [1.0, 1.0 + 4.0, 1.0 + 8.0 + 2.0, 1.0 + 12.0 + 6.0 - 0.5]
        nbr_d = [0.0, -1.0, 0.0 - 2.0 - 8.0, 0.0 - 3.0 - 24.0]
        assert np.array_equal(X[0, :8], np.array(own_d + nbr_d) / 8.0)
    assert np.all(X[:, 8] == 1.0) and np.all(X[:, 9] == 1.0)
