"""sw_misfit_noalloc, the misfit entry point for callers that cannot
allocate device memory, against sw_misfit (which takes a caller-owned
workspace): the same ERR and pair count on two calls in a row, the second
smaller than the first, so the second reuses the static scratch the first
left behind; and the host rejection of receiver counts beyond its limit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2404_17754_amd as sw
    from paper_2404_17754_amd import _lib as L
    ctx = sw.Context(0)
    return torch, L, ctx


def _inputs(torch, n_steps, n_rec, seed, silent=()):
    rng = np.random.default_rng(seed)
    obs = rng.standard_normal((n_steps, n_rec, 3))
    U = obs + 0.1 * rng.standard_normal((n_steps, n_rec, 3))
    for r, c in silent:
        obs[:, r, c] = 0.0
    dev = lambda a: torch.from_numpy(a).to("cuda:0").contiguous()  # noqa: E731
    return dev(U), dev(obs)


def _with_workspace(torch, L, ctx, U, obs):
    n_steps, n_rec = U.shape[0], U.shape[1]
    nb = C.c_size_t()
    L.check(ctx.lib.sw_misfit_workspace_bytes(n_rec, C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    e, n = C.c_double(), C.c_int32()
    L.check(ctx.lib.sw_misfit(ctx.h, n_rec, n_steps, C.c_void_p(U.data_ptr()), C.c_void_p(obs.data_ptr()),
                              C.c_void_p(ws.data_ptr()), nb.value, C.byref(e), C.byref(n)))
    return e.value, n.value


def _noalloc(L, ctx, U, obs):
    n_steps, n_rec = U.shape[0], U.shape[1]
    e, n = C.c_double(), C.c_int32()
    L.check(ctx.lib.sw_misfit_noalloc(ctx.h, n_rec, n_steps, C.c_void_p(U.data_ptr()),
                                      C.c_void_p(obs.data_ptr()), C.byref(e), C.byref(n)))
    return e.value, n.value


def test_noalloc_matches_workspace_entry_point_twice(env):
    torch, L, ctx = env
    # first call: 2500 receivers (a 50 x 50 grid), 300 steps, two silent pairs
    U1, o1 = _inputs(torch, 300, 2500, 11, silent=((3, 1), (2400, 2)))
    # second call: fewer receivers and steps; the first call's pair sums
    # beyond the second's range are left in the scratch and must not count
    U2, o2 = _inputs(torch, 120, 400, 12)
    for U, o, pairs in ((U1, o1, 3 * 2500 - 2), (U2, o2, 3 * 400)):
        ref = _with_workspace(torch, L, ctx, U, o)
        got = _noalloc(L, ctx, U, o)
        assert got[1] == ref[1] == pairs
        assert abs(got[0] - ref[0]) <= 1e-14 * abs(ref[0])
        # and the definition (Eq. eqerr) on the host, FP64
        Uh, oh = U.cpu().numpy(), o.cpu().numpy()
        d = np.sqrt(((Uh - oh) ** 2).sum(0))
        on = np.sqrt((oh ** 2).sum(0))
        used = on > 1e-12 * on.max()
        assert abs(got[0] - (d[used] / on[used]).mean()) <= 1e-12 * got[0]


def test_noalloc_rejects_beyond_limit(env):
    torch, L, ctx = env
    n_rec = L.MISFIT_NOALLOC_MAX_REC + 1
    U = torch.zeros((1, n_rec, 3), dtype=torch.float64, device="cuda:0")
    e, n = C.c_double(), C.c_int32()
    rc = ctx.lib.sw_misfit_noalloc(ctx.h, n_rec, 1, C.c_void_p(U.data_ptr()), C.c_void_p(U.data_ptr()),
                                   C.byref(e), C.byref(n))
    assert rc == L.SW_EINVAL
    assert b"static scratch limit" in ctx.lib.sw_last_error()
