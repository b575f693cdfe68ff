"""Rows of the step operator A = c_M M + c_K K + c_C C_abs at a few nodes of
a mesh too large for the assembled oracle, formed by the oracle from the
element and face matrices around each node (one row at a time), for the
full-size parity tests."""
import numpy as np

from oracle import assemble, fem


def coefficients(case):
    """(c_M, c_K, c_C) of A = 4/dt^2 M + 2/dt (alpha M + beta K + C_abs) + K."""
    dt = case.dt
    return 4.0 / dt ** 2 + 2.0 * case.ray_alpha / dt, 1.0 + 2.0 * case.ray_beta / dt, 2.0 / dt


def sample_nodes(mesh, n_random=16, seed=7):
    """Seeded random nodes plus a vertex and an edge node of two faces of
    each absorbing role (sides, base)."""
    rng = np.random.default_rng(seed)
    nodes = list(rng.choice(mesh.n_nodes, n_random, replace=False))
    for role in (1, 2):
        f = np.nonzero(mesh.face_role == role)[0]
        tri = mesh.tri6[rng.choice(f, 2, replace=False)]
        nodes += [int(tri[0, 0]), int(tri[1, 4])]
    return np.unique(np.asarray(nodes, dtype=np.int64))


def oracle_rows(mesh, case, nodes, x):
    """Rows of A x at `nodes` (len(nodes) x 3) and the same rows of |A| |x|,
    the scale of the rounding."""
    cM, cK, cC = coefficients(case)
    y = np.zeros((len(nodes), 3))
    s = np.zeros((len(nodes), 3))
    tets = np.nonzero(np.isin(mesh.tet10, nodes).any(axis=1))[0]
    Ke, Me = assemble.element_matrices(mesh, case.mat, case.tet_mat, tets)
    Ae = cM * Me + cK * Ke
    fsel = np.nonzero(np.isin(mesh.tri6, nodes).any(axis=1) & np.isin(mesh.face_role, (1, 2)))[0]
    vp, vs, rho = (a[fsel] for a in assemble.face_materials(mesh, case.mat, case.tet_mat))
    Cf = cC * fem.face_dashpot(mesh.xyz[mesh.tri6[fsel, :3]], vp, vs, rho)
    for k, n in enumerate(nodes):
        for mats, conn in ((Ae, mesh.tet10[tets]), (Cf, mesh.tri6[fsel])):
            for j in np.nonzero((conn == n).any(axis=1))[0]:
                loc = int(np.nonzero(conn[j] == n)[0][0])
                xe = x[(3 * conn[j][:, None] + np.arange(3)).ravel()]
                rows = mats[j][3 * loc:3 * loc + 3]
                y[k] += rows @ xe
                s[k] += np.abs(rows) @ np.abs(xe)
    return y, s


def check_rows(gc, mesh, case, seed=11):
    """Largest error of the case's FP64 and FP32 operator passes at the
    sample nodes, relative to |A| |x| of each row."""
    import torch
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(3 * mesh.n_nodes)
    x32 = x.astype(np.float32)
    nodes = sample_nodes(mesh)
    dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
    y64 = gc.apply("A", torch.from_numpy(x)).cpu().numpy()[dofs].reshape(-1, 3)
    y32 = gc.apply_f32("A", torch.from_numpy(x32)).cpu().numpy()[dofs].reshape(-1, 3).astype(np.float64)
    ref64, s64 = oracle_rows(mesh, case, nodes, x)
    ref32, s32 = oracle_rows(mesh, case, nodes, x32.astype(np.float64))
    return float(np.max(np.abs(y64 - ref64) / s64)), float(np.max(np.abs(y32 - ref32) / s32)), len(nodes)
