"""Waveform misfit ERR of Eq. (eqerr), Section 2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

ERR = 1/(3 n_obs) sum_k sum_i sqrt(int (U_i^k - obs_i^k)^2 dt) / sqrt(int (obs_i^k)^2 dt)

The time integrals are sums over the recorded samples (the common factor dt
cancels in the ratio).  A (receiver, component) pair whose observed record
has norm <= 1e-12 times the largest observed norm has no defined ratio; such
pairs are skipped and the mean is taken over the pairs that remain.
"""
from __future__ import annotations

import numpy as np


def err(U, obs, skip_rel=1e-12):
    """U, obs: (n_steps, n_rec, 3).  Returns (ERR, number of pairs used)."""
    U = np.asarray(U, float)
    obs = np.asarray(obs, float)
    n_rec = U.shape[1]
    total, used = 0.0, 0
    norms = np.zeros((n_rec, 3))
    for k in range(n_rec):
        for i in range(3):
            norms[k, i] = np.sqrt(np.sum(obs[:, k, i] ** 2))
    thresh = skip_rel * norms.max() if norms.size else 0.0
    for k in range(n_rec):
        for i in range(3):
            if norms[k, i] <= thresh:
                continue
            total += np.sqrt(np.sum((U[:, k, i] - obs[:, k, i]) ** 2)) / norms[k, i]
            used += 1
    return (total / used if used else float("nan")), used
