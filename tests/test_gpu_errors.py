"""Error paths of the C-ABI: host validation rejects bad meshes, parameters
and workspaces before any device work; non-convergence is flagged, not
raised."""
import ctypes as C

import numpy as np
import pytest

import casegen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    return sw.Context(0)


def _mesh():
    return cg.box_mesh(30.0, 20.0, 20.0, 10.0)


def test_inverted_tet_rejected(sw, ctx):
    m = _mesh()
    m.tet10 = m.tet10.copy()
    t = m.tet10[5].copy()
    # swap two vertices (and their edge nodes consistently) -> negative volume
    m.tet10[5, [1, 2]] = t[[2, 1]]
    with pytest.raises(sw.SwError, match="SW_EMESH"):
        sw.Mesh(ctx, m)


def test_curved_edge_rejected(sw, ctx):
    m = _mesh()
    m.xyz = m.xyz.copy()
    m.xyz[m.tet10[3, 6]] += 0.5
    with pytest.raises(sw.SwError, match="SW_EMESH"):
        sw.Mesh(ctx, m)


def test_index_out_of_range_rejected(sw, ctx):
    m = _mesh()
    m.tet10 = m.tet10.copy()
    m.tet10[0, 9] = m.n_nodes
    with pytest.raises(sw.SwError, match="SW_EMESH"):
        sw.Mesh(ctx, m)


def test_bad_case_params_rejected(sw, ctx):
    m = _mesh()
    gm = sw.Mesh(ctx, m)
    c = cg.make_case(m, cg.CONFIGS["small"], n_steps=5, n_rec=1)
    for kw, match in [({"rtol": 0.0}, "rtol"), ({"poly_order": 7}, "poly_order"), ({"max_iter": 0}, "max_iter")]:
        with pytest.raises(sw.SwError, match="SW_EINVAL"):
            sw.Case(ctx, gm, c, **kw)
    bad = cg.make_case(m, cg.CONFIGS["small"], n_steps=5, n_rec=1)
    bad.tet_mat = np.full(m.n_tets, 3, np.uint8)
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, bad)
    bad = cg.make_case(m, cg.CONFIGS["small"], n_steps=5, n_rec=1)
    bad.dt = -1.0
    with pytest.raises(sw.SwError, match="SW_EINVAL"):
        sw.Case(ctx, gm, bad)


def test_small_workspace_rejected(sw, ctx):
    import torch
    from paper_2404_17754_amd import _lib as L
    m = _mesh()
    lib = L.load()
    xyz = np.ascontiguousarray(m.xyz)
    tet = np.ascontiguousarray(m.tet10)
    tri = np.ascontiguousarray(m.tri6)
    ft = np.ascontiguousarray(m.face_tet)
    fr = np.ascontiguousarray(m.face_role)
    d = L.MeshDesc(m.n_nodes, m.n_tets, m.n_faces, xyz.ctypes.data, tet.ctypes.data, tri.ctypes.data,
                   ft.ctypes.data, fr.ctypes.data)
    nb = C.c_size_t()
    L.check(lib.sw_mesh_workspace_bytes(C.byref(d), C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    rc = lib.sw_mesh_create(ctx.h, C.byref(d), C.c_void_p(ws.data_ptr()), nb.value - 1, C.byref(h))
    assert rc == L.SW_ENOWS
    rc = lib.sw_mesh_create(ctx.h, C.byref(d), C.c_void_p(ws.data_ptr() + 8), nb.value - 8, C.byref(h))
    assert rc == L.SW_ENOWS


def test_max_iter_flags_nonconvergence(sw, ctx):
    m = _mesh()
    c = cg.make_case(m, cg.CONFIGS["small"], n_steps=30, n_rec=1)
    gc = sw.Case(ctx, sw.Mesh(ctx, m), c, max_iter=2)
    gc.step(30)
    st = gc.stats()
    assert st["flags"] & 1 and st["steps"] == 30


def test_step_beyond_capacity(sw, ctx):
    m = _mesh()
    c = cg.make_case(m, cg.CONFIGS["small"], n_steps=3, n_rec=1)
    gc = sw.Case(ctx, sw.Mesh(ctx, m), c)
    gc.step(3)
    with pytest.raises(sw.SwError, match="SW_ESTATE"):
        gc.step(1)
