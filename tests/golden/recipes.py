"""Recipes of the stored oracle receiver records (tests/golden/*.npz) that
the config-size GPU parity tests compare against.  Each recipe names the
seeded inputs only (casegen); the records are written by make_golden.py,
which runs the oracle and nothing else.

Every recipe is one analysis of one candidate model:
  config   casegen configuration (mesh, materials law, input wavelet, dt)
  seed     the model's interface-field seed
  steps    steps marched
  start    "rest" (zero state at step 0) or "smooth": u = a = 0 and the
           seeded smooth velocity field casegen.smooth_field(mesh,
           state_seed, corr, amp) at step `step0`, so that every element is
           in motion from the first step (windows of the large meshes,
           where marching from rest to the arrival of the wave at the
           surface is beyond the oracle's CPU time)
  rec      receivers kept: every rec-th receiver of the config's grid in
           each direction
"""

SMOOTH = dict(corr=40.0, amp=1e-3)

RECIPES = {
    # the batched uneven workload: one model per mesh size, from rest until
    # the main pulse has crossed the soft layer (arrival ~ step 170)
    "c2_200m_seed1000": dict(config="batch200", seed=1000, steps=240, start="rest", rec=2),
    "c2_300m_seed1001": dict(config="batch300", seed=1001, steps=240, start="rest", rec=2),
    "c2_400m_seed1002": dict(config="batch400", seed=1002, steps=240, start="rest", rec=2),
    # two held-out models of the learned-guess workload (300 m mesh)
    "c3_300m_seed2000": dict(config="batch300", seed=2000, steps=240, start="rest", rec=2),
    "c3_300m_seed2001": dict(config="batch300", seed=2001, steps=240, start="rest", rec=2),
    # the large single case (39 M DOF): a window with the input at its peak
    "c1_window": dict(config="large", seed=1, steps=6, start="smooth", state_seed=71, step0=80, rec=1),
    # three sampled models of the full sweep (19.8 M DOF each)
    "c4_seed3000_window": dict(config="sweep", seed=3000, steps=6, start="smooth", state_seed=72, step0=200, rec=5),
    "c4_seed3500_window": dict(config="sweep", seed=3500, steps=6, start="smooth", state_seed=72, step0=200, rec=5),
    "c4_seed3999_window": dict(config="sweep", seed=3999, steps=6, start="smooth", state_seed=72, step0=200, rec=5),
}


def receiver_subset(n_side, every):
    """Indices into the config's n_side x n_side receiver list kept in the
    stored records (receiver (i, j) is entry i * n_side + j)."""
    return [i * n_side + j for i in range(0, n_side, every) for j in range(0, n_side, every)]


def inputs(name, mesh=None):
    """(mesh, case, u0, v0, a0, step0) of a recipe, from casegen only."""
    import numpy as np

    import casegen as cg
    r = RECIPES[name]
    cfg = cg.CONFIGS[r["config"]]
    if mesh is None:
        mesh = cg.config_mesh(cfg)
    step0 = r.get("step0", 0)
    case = cg.make_case(mesh, cfg, seed=r["seed"], n_steps=step0 + r["steps"])
    n3 = 3 * mesh.n_nodes
    if r["start"] == "rest":
        v0 = np.zeros(n3)
    else:
        v0 = cg.smooth_field(mesh, r["state_seed"], **SMOOTH)
    return mesh, case, np.zeros(n3), v0, np.zeros(n3), step0
