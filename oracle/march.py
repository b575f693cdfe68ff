"""Newmark-beta time march (Section 3: implicit Newmark-beta integration of
the discretised Eq. GE:ORG), average-acceleration variant beta = 1/4,
gamma = 1/2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With C = alpha M + beta_R K + C_abs and the Newmark relations
    u^{n+1} = u^n + dt v^n + dt^2/4 (a^n + a^{n+1})
    v^{n+1} = v^n + dt/2 (a^n + a^{n+1})
the equation of motion at t^{n+1} becomes, for du = u^{n+1} - u^n,
    (4/dt^2 M + 2/dt C + K) du = F^{n+1} - K u^n + C v^n + M (a^n + 4/dt v^n)
after which
    u^{n+1} = u^n + du,  v^{n+1} = 2/dt du - v^n,
    a^{n+1} = 4/dt^2 du - 4/dt v^n - a^n.
Each step's system is solved by sparse LU (exact up to rounding) or by
conjugate gradients to a relative residual tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assemble


@dataclass
class System:
    K: sp.csr_matrix
    M: sp.csr_matrix
    Cabs: sp.csr_matrix
    Fb: np.ndarray          # (3, n_dof) input-force basis
    alpha: float
    beta: float

    @property
    def C(self):
        return self.alpha * self.M + self.beta * self.K + self.Cabs


def build_system(mesh, case, damping=True, dashpot_roles=(1, 2), input_force=True):
    K, M = assemble.stiffness_and_mass(mesh, case.mat, case.tet_mat)
    Cabs = assemble.dashpots(mesh, case.mat, case.tet_mat, dashpot_roles)
    Fb = assemble.input_force_basis(mesh, case.mat, case.tet_mat)
    if not input_force:
        Fb = np.zeros_like(Fb)
    a, b = (case.ray_alpha, case.ray_beta) if damping else (0.0, 0.0)
    return System(K, M, Cabs, Fb, a, b)


def step_matrix(sys: System, dt):
    return (4.0 / dt ** 2) * sys.M + (2.0 / dt) * sys.C + sys.K


@dataclass
class Result:
    rec_v: np.ndarray       # (n_steps, n_rec, 3) velocity at receivers, steps 1..n
    u: np.ndarray           # final state
    v: np.ndarray
    a: np.ndarray
    states: list            # optional [(u, v, a)] for n = 0..n_steps
    iters: list             # CG iterations per step (empty for LU)


def consistent_acceleration(sys: System, u0, v0, f0, free=None):
    """a0 = M^{-1} (F0 - C v0 - K u0) on the free DOFs."""
    rhs = f0 - sys.C @ v0 - sys.K @ u0
    a0 = np.zeros_like(u0)
    if free is None:
        a0[:] = spla.spsolve(sys.M.tocsc(), rhs)
    else:
        a0[free] = spla.spsolve(sys.M[free][:, free].tocsc(), rhs[free])
    return a0


def run(sys: System, dt, v_in, n_steps, rec_node, u0=None, v0=None, a0=None,
        solver="lu", rtol=1e-12, fixed_dofs=None, keep_states=False):
    """March n_steps steps from (u0, v0, a0) (zero by default).

    v_in: (n_steps + 1, 3) incident velocity at t = n dt.
    fixed_dofs: DOFs held at zero displacement (test constraints only).
    """
    n = sys.K.shape[0]
    u = np.zeros(n) if u0 is None else np.array(u0, float)
    v = np.zeros(n) if v0 is None else np.array(v0, float)
    a = np.zeros(n) if a0 is None else np.array(a0, float)
    free = np.ones(n, bool)
    if fixed_dofs is not None:
        free[np.asarray(fixed_dofs)] = False
    fi = np.nonzero(free)[0]
    A = step_matrix(sys, dt)[fi][:, fi].tocsc()
    if solver == "lu":
        lu = spla.splu(A)
        solve = lambda b: (lu.solve(b), 0)  # noqa: E731
    else:
        Ad = A.tocsr()
        dinv = 1.0 / Ad.diagonal()
        P = spla.LinearOperator(A.shape, matvec=lambda x: dinv * x)

        def solve(b):
            cnt = [0]

            def cb(_):
                cnt[0] += 1
            if not np.any(b):
                return np.zeros_like(b), 0
            x, info = spla.cg(Ad, b, rtol=rtol, atol=0.0, M=P, maxiter=100000, callback=cb)
            if info != 0:
                raise RuntimeError(f"oracle CG did not converge (info={info})")
            return x, cnt[0]

    C = sys.C
    rec_dofs = assemble.node_dofs(rec_node)
    rec_v = np.zeros((n_steps, len(rec_node), 3))
    states = [(u.copy(), v.copy(), a.copy())] if keep_states else []
    iters = []
    c1 = 4.0 / dt
    for k in range(n_steps):
        F = v_in[k + 1] @ sys.Fb
        b = F - sys.K @ u + C @ v + sys.M @ (a + c1 * v)
        du = np.zeros(n)
        x, it = solve(b[fi])
        du[fi] = x
        iters.append(it)
        v_new = (2.0 / dt) * du - v
        a_new = (4.0 / dt ** 2) * du - c1 * v - a
        u = u + du
        v, a = v_new, a_new
        rec_v[k] = v[rec_dofs].reshape(-1, 3)
        if keep_states:
            states.append((u.copy(), v.copy(), a.copy()))
    return Result(rec_v, u, v, a, states, iters)


def run_case(mesh, case, n_steps=None, solver="lu", rtol=1e-12, **kw):
    """Full analysis of one case with zero initial state: velocity at the
    case's receivers for steps 1..n_steps."""
    n_steps = case.n_steps if n_steps is None else n_steps
    sys = build_system(mesh, case)
    return run(sys, case.dt, case.v_in, n_steps, case.rec_node, solver=solver, rtol=rtol, **kw)
