"""Input estimation and the misfit of Section 2, written from its definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The input velocity along direction j is parametrised by shifted copies of a
unit impulse p (Section 2):  f_j(t) = sum_l c_{jl} p(t - l dT).  With
G_ij^k the velocity along i at observation point k caused by p input along
j at the base, a linear time-invariant model started from rest responds to
f with  U_i^k(t) = sum_j sum_l G_ij^k(t - l dT) c_{jl}.  The coefficients
minimise the misfit to the observed records; the paper writes the
stationarity condition as a small linear system A c = b solved with a
pseudo-inverse that discards negligible singular values, and reports ERR
(Eq. eqerr) at that c.

Readings (ERR itself is a sum of square roots, not a quadratic):
* the quadratic objective is J(c) = sum_{k,i} |U_i^k - obs_i^k|^2 / |obs_i^k|^2
  (the squares of ERR's terms; integrals as sums over the record);
* (k, i) pairs whose observed record is silent (norm <= 1e-12 of the
  largest) carry no weight, as in ERR;
* dT is a whole number `stride` of time steps and the record length is a
  multiple of it; the responses are recorded at steps 1..n_steps, so the
  response to the impulse shifted by l strides is the Green's record
  delayed by l * stride samples (zero before);
* singular values of A below rel_cut times the largest are discarded.
"""
from __future__ import annotations

import numpy as np

from . import misfit


def design(G, stride, n_shift):
    """G: (3, n_steps, n_rec, 3) Green's records, G[j][t, k, i].  Returns H
    with rows (t, k, i) and columns (j, l): H[(t,k,i), (j,l)] =
    G[j][t - l stride, k, i] (zero when t < l stride)."""
    G = np.asarray(G, float)
    _, n, n_rec, _ = G.shape
    H = np.zeros((n, n_rec, 3, 3, n_shift))
    for j in range(3):
        for l in range(n_shift):
            s = l * stride
            if s < n:
                H[s:, :, :, j, l] = G[j, : n - s]
    return H.reshape(n * n_rec * 3, 3 * n_shift)


def pair_weights(obs, skip_rel=1e-12):
    """1 / |obs_i^k|^2 per (k, i), zero for silent pairs."""
    nrm = np.sqrt((np.asarray(obs, float) ** 2).sum(0))   # (n_rec, 3)
    thr = skip_rel * nrm.max() if nrm.size else 0.0
    return np.where(nrm > thr, 1.0 / np.where(nrm > thr, nrm, 1.0) ** 2, 0.0)


def fit(G, obs, stride, n_shift, rel_cut=1e-6):
    """Least-squares input coefficients and the misfit.

    Returns c (3, n_shift), U (n_steps, n_rec, 3), ERR, pairs used, rank."""
    obs = np.asarray(obs, float)
    n, n_rec, _ = obs.shape
    if n % stride:
        raise ValueError("record length must be a multiple of the stride")
    H = design(G, stride, n_shift)
    w = np.broadcast_to(pair_weights(obs)[None], (n, n_rec, 3)).reshape(-1)
    A = H.T @ (w[:, None] * H)
    b = H.T @ (w * obs.reshape(-1))
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    keep = lam > rel_cut * lam.max() if lam.max() > 0 else np.zeros_like(lam, bool)
    c = V[:, keep] @ ((V[:, keep].T @ b) / lam[keep])
    U = (H @ c).reshape(n, n_rec, 3)
    e, used = misfit.err(U, obs)
    return c.reshape(3, n_shift), U, e, used, int(keep.sum())


def fit_events(G, events, stride, n_shift, rel_cut=1e-6):
    """Several observed events of one model (Section 3, the events recorded
    at one site): the Green's records G are the model's, each event's input
    is fitted on its own (fit), and the model's misfit is its worst event's
    ERR.  Returns (list of fit results per event, largest ERR, its event)."""
    fits = [fit(G, obs, stride, n_shift, rel_cut) for obs in events]
    errs = [f[2] for f in fits]
    worst = int(np.argmax(errs))
    return fits, errs[worst], worst


def objective(G, obs, stride, c):
    """J(c) = sum_{k,i} |U - obs|^2 / |obs|^2 over the non-silent pairs."""
    c = np.asarray(c, float)
    H = design(G, stride, c.shape[1])
    U = (H @ c.reshape(-1)).reshape(np.shape(obs))
    w = pair_weights(obs)
    return float((w[None] * (U - obs) ** 2).sum())


def input_waveform(c, p, stride, n_steps):
    """f_j(t) = sum_l c_jl p(t - l stride) at steps 0..n_steps, (n_steps+1, 3)."""
    c = np.asarray(c, float)
    f = np.zeros((n_steps + 1, 3))
    for j in range(3):
        for l in range(c.shape[1]):
            s = l * stride
            if s <= n_steps:
                f[s:, j] += c[j, l] * p[: n_steps + 1 - s]
    return f
