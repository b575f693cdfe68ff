"""The optional kernel profiler of the C-ABI: HIP events bracket only the
kernel classes asked for, one launch in `every` of each, and bad requests
are rejected before any device work."""
import ctypes as C

import pytest

import casegen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


def _case(sw, ctx):
    cfg = cg.CONFIGS["small"]
    mesh = cg.config_mesh(cfg)
    return sw.Case(ctx, sw.Mesh(ctx, mesh), cg.make_case(mesh, cfg, n_steps=12), precision="mixed", guess="poly")


def test_profile_classes_and_sampling(sw):
    ctx = sw.Context(0)
    gc = _case(sw, ctx)
    ctx.profile(True, kinds=("tile_f32",))
    gc.step(3)
    tile, upd = ctx.profile_read("tile_f32"), ctx.profile_read("update_f32")
    assert tile[1] > 0 and tile[0] > 0.0 and upd[1] == 0
    # both classes launch once per CG iteration: the same count at any stride
    ctx.profile(True, kinds=("tile_f32", "update_f32"))
    gc.step(3)
    n1 = ctx.profile_read("tile_f32")[1]
    assert n1 > 0 and ctx.profile_read("update_f32")[1] == n1
    ctx.profile(True, kinds=("tile_f32", "update_f32"), every=3)
    gc.step(3)
    n3 = ctx.profile_read("tile_f32")[1]
    assert n3 > 0 and ctx.profile_read("update_f32")[1] == n3
    assert n3 < n1
    ctx.profile(True)
    gc.step(3)
    assert ctx.profile_read("dir_f32")[1] == ctx.profile_read("tile_f32")[1] > 0
    ctx.profile(False)


def test_profile_rejects_bad_requests(sw):
    from paper_2404_17754_amd import _lib as L
    ctx = sw.Context(0)
    lib = ctx.lib
    assert lib.sw_ctx_profile_kinds(ctx.h, C.c_uint32(1 << 6), 1) == L.SW_EINVAL
    assert lib.sw_ctx_profile_kinds(ctx.h, C.c_uint32(2), 0) == L.SW_EINVAL
    assert lib.sw_ctx_profile_kinds(None, C.c_uint32(2), 1) == L.SW_EINVAL
    assert lib.sw_ctx_profile_kinds(ctx.h, C.c_uint32(0), 1) == 0
