"""Every row of the persistent FP32 operator passes against the oracle when
each workgroup walks many tiles, as on the full-size meshes: the next tile's
node ids and values are loaded behind the current tile's element work and
handed over through LDS between tiles (single case, and the lane pass of a
batch over (lane, tile) work items).

The meshes are built with small tiles (at most 64 nodes) and the context
caps the persistent grid at 8 workgroups (one per XCD), so that every
workgroup walks at least four tiles or work items; a march in that
configuration is compared with the oracle's exact solves.  A wrong FP32
operator would be hidden by the FP64 refinement (more CG iterations, the
same waveforms), so the operator rows are compared directly."""
import numpy as np
import pytest

import casegen as cg
from oracle import march

pytestmark = pytest.mark.gpu

TILE_NODES = 64
GRID = 8


@pytest.fixture(scope="module")
def sw():
    import paper_2404_17754_amd as sw
    return sw


@pytest.fixture(scope="module")
def ctx(sw):
    c = sw.Context(0)
    c.set_grid_cap(GRID)
    return c


def _meshes():
    return {"small": cg.config_mesh(cg.CONFIGS["small"]),
            "jitter": cg.box_mesh(80.0, 60.0, 40.0, 10.0, jitter=0.22, seed=3),
            "graded": cg.box_mesh(80.0, 60.0, 40.0, 10.0, jitter=0.15, seed=4,
                                  z_levels=cg.graded_levels(40.0, 2.5, 1.5))}


MESHES = _meshes()


def _case_for(name, mesh, seed=5):
    if name == "small":
        return cg.make_case(mesh, cg.CONFIGS["small"])
    c = cg.make_case(mesh, cg.CONFIGS["small"], n_rec=2)
    c.tet_mat = np.random.default_rng(seed).integers(0, 2, mesh.n_tets).astype(np.uint8)
    return c


def _step_operator(S, case):
    dt = case.dt
    cM = 4 / dt ** 2 + 2 * case.ray_alpha / dt
    cK = 1 + 2 * case.ray_beta / dt
    return cM * S.M + cK * S.K + (2 / dt) * S.Cabs


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def gpu_meshes(sw, ctx):
    out = {}
    for name, mesh in MESHES.items():
        gm = sw.Mesh(ctx, mesh, tile_nodes=TILE_NODES)
        n_tiles, mx = gm.info()
        print(f"{name}: {mesh.n_tets} tets in {n_tiles} tiles of at most {mx} nodes", flush=True)
        assert mx <= TILE_NODES and n_tiles >= 4 * GRID
        out[name] = gm
    return out


@pytest.mark.parametrize("name", list(MESHES))
def test_single_case_pass_all_rows(sw, ctx, gpu_meshes, name):
    import torch
    mesh = MESHES[name]
    case = _case_for(name, mesh)
    A = _step_operator(march.build_system(mesh, case), case)
    gc = sw.Case(ctx, gpu_meshes[name], case, precision="mixed", guess="proj")
    for seed in (2, 3):
        x = cg.random_vector(3 * mesh.n_nodes, seed)
        y = gc.apply_f32("A", torch.from_numpy(x).float()).double().cpu().numpy()
        assert _rel(y, A @ x) < 2e-5, (name, seed, _rel(y, A @ x))


def test_lane_pass_all_rows(sw, ctx, gpu_meshes):
    """Five lanes over the three meshes (two models on two of them): each
    lane's rows through the batch's lane pass against its own operator."""
    import torch
    lanes, refs = [], []
    for k, name in enumerate(("small", "jitter", "graded", "small", "jitter")):
        mesh = MESHES[name]
        case = _case_for(name, mesh, seed=10 + k)
        if name == "small" and k:
            case = cg.make_case(mesh, cg.CONFIGS["small"], seed=7)
        refs.append((mesh, _step_operator(march.build_system(mesh, case), case)))
        lanes.append(sw.Case(ctx, gpu_meshes[name], case, precision="mixed", guess="proj"))
    b = sw.Batch(ctx, lanes)
    xs = [torch.from_numpy(cg.random_vector(3 * m.n_nodes, 20 + k)).float() for k, (m, _) in enumerate(refs)]
    ys = b.apply_f32(xs)
    for k, ((mesh, A), x, y) in enumerate(zip(refs, xs, ys)):
        ref = A @ x.double().numpy()
        e = _rel(y.double().cpu().numpy(), ref)
        assert e < 2e-5, (k, e)


def test_march_with_walking_workgroups(sw, ctx, gpu_meshes):
    """The small case (50 steps) in mixed precision with the projected
    guess, alone and as two batch lanes, against the oracle's exact
    solves."""
    mesh = MESHES["small"]
    case = cg.make_case(mesh, cg.CONFIGS["small"])
    ref = march.run_case(mesh, case, solver="lu").rec_v
    alone = sw.Case(ctx, gpu_meshes["small"], case, precision="mixed", guess="proj")
    alone.step(case.n_steps)
    lanes = [sw.Case(ctx, gpu_meshes["small"], case, precision="mixed", guess=g) for g in ("proj", "poly")]
    sw.Batch(ctx, lanes).step(case.n_steps)
    for gc in [alone] + lanes:
        w = gc.waveforms()
        st = gc.stats()
        err = np.linalg.norm(w - ref) / np.linalg.norm(ref)
        assert err < 1e-6 and st["max_true_rel_res"] <= 1e-8 and not st["flags"] & 3, (err, st)
