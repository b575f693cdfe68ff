"""FP64 reference of the per-DOF initial-guess network.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper has no network; the target adds a learned initial guess for each
step's CG solve.  The reading implemented on both sides:

* features of DOF (node n, component c) before the step that computes
  du^m: the last four increments d_k = du^{m-1-k}(n, c), k = 0..3, their
  element-neighbour means nb_k (mean over the elements containing node n of
  the element mean of the same component), and the node's Vs/500 and
  rho/2000 (means over the elements containing it);
* scale s = max_k(|d_k|, |nb_k|); network input
  x = (D(d), D(nb)) / s, Vs/500, rho/2000, where D(a) = (a_0, a_0 - a_1,
  a_0 - 2 a_1 + a_2, a_0 - 3 a_1 + 3 a_2 - a_3) are the differences of
  increasing order (the same information as the increments, but the small
  higher differences, which carry the extrapolation error, keep their
  relative precision when the network rounds its inputs to FP16);
* network: x (10) -> ReLU(64) -> ReLU(64) -> y (linear), parameters packed
  as W1[64][10], b1[64], W2[64][64], b2[64], w3[64], b3 (4929 values);
* guess: du0 = p2 + s y with p2 = 3 d_0 - 3 d_1 + d_2 (quadratic
  extrapolation); s = 0 gives du0 = 0;
* training target t = (du^m - p2) / s with weight s^2, loss
  L = sum_i s_i^2 (y_i - t_i)^2 / sum_i s_i^2 (the squared error of the
  unnormalised guess, normalised), Adam (beta 0.9, 0.999, eps 1e-8).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 10, 64
SIZES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", (1,)))
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SIZES])


def init(seed):
    """Glorot-uniform hidden layers, zero output layer (the untrained
    network reproduces the quadratic extrapolation exactly)."""
    rng = np.random.default_rng(seed)
    a1 = np.sqrt(6.0 / (N_IN + N_H))
    a2 = np.sqrt(6.0 / (N_H + N_H))
    return pack({"W1": rng.uniform(-a1, a1, (N_H, N_IN)), "b1": np.zeros(N_H),
                 "W2": rng.uniform(-a2, a2, (N_H, N_H)), "b2": np.zeros(N_H),
                 "w3": np.zeros(N_H), "b3": np.zeros(1)})


def relu(z):
    return np.maximum(z, 0.0)


def forward(theta, X):
    """X: (n, 10) -> y (n,)."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = relu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = relu(z2)
    return h2 @ p["w3"] + p["b3"][0]


def loss(theta, X, t, w):
    y = forward(theta, X)
    return float(np.sum(w * (y - t) ** 2) / np.sum(w))


def gradient(theta, X, t, w):
    """dL/dtheta by back-propagation through the three layers."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = relu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = relu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    dy = 2.0 * w * (y - t) / np.sum(w)            # (n,)
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)        # (n, 64)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return pack(g)


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def neighbour_mean(tet10, n_nodes, v):
    """Element-neighbour mean of a node field v (n_nodes, k): for each node,
    the mean over the elements containing it of the element mean of v over
    the element's ten nodes."""
    v = np.asarray(v, np.float64).reshape(n_nodes, -1)
    elem_mean = v[tet10].mean(1)                        # (n_tets, k)
    acc = np.zeros_like(v)
    cnt = np.zeros(n_nodes)
    for a in range(tet10.shape[1]):
        np.add.at(acc, tet10[:, a], elem_mean)
        np.add.at(cnt, tet10[:, a], 1.0)
    return acc / cnt[:, None]


def node_material(tet10, n_nodes, mat, tet_mat):
    """Per-node Vs and rho: means over the elements containing the node."""
    vals = mat[tet_mat][:, [1, 2]]
    acc = np.zeros((n_nodes, 2))
    cnt = np.zeros(n_nodes)
    for a in range(tet10.shape[1]):
        np.add.at(acc, tet10[:, a], vals)
        np.add.at(cnt, tet10[:, a], 1.0)
    acc /= cnt[:, None]
    return acc[:, 0], acc[:, 1]


def differences(a):
    """(n, 4) newest first -> (a_0, a_0 - a_1, a_0 - 2 a_1 + a_2,
    a_0 - 3 a_1 + 3 a_2 - a_3): backward differences of orders 0..3."""
    return np.stack([a[:, 0], a[:, 0] - a[:, 1], a[:, 0] - 2 * a[:, 1] + a[:, 2],
                     a[:, 0] - 3 * a[:, 1] + 3 * a[:, 2] - a[:, 3]], 1)


def features(own, nbr, vs, rho):
    """own, nbr: (n, 4) newest first; vs, rho: (n,).  Returns X (n, 10), s (n,)."""
    own = np.asarray(own, np.float64)
    nbr = np.asarray(nbr, np.float64)
    s = np.maximum(np.abs(own).max(1), np.abs(nbr).max(1))
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    X = np.concatenate([differences(own) * inv[:, None], differences(nbr) * inv[:, None],
                        (vs / 500.0)[:, None], (rho / 2000.0)[:, None]], 1)
    return X, s


def guess(theta, own, nbr, vs, rho):
    X, s = features(own, nbr, vs, rho)
    p2 = 3 * own[:, 0] - 3 * own[:, 1] + own[:, 2]
    return np.where(s > 0, p2 + s * forward(theta, X), 0.0)
