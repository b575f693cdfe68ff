"""Writes tests/golden/<recipe>.npz: receiver velocity records of the
oracle (the assembled FP64 block-sparse solver, oracle/bsr.py, each step
solved to a true relative residual of 1e-12) for the recipes in recipes.py.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_golden.py [recipe ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import casegen as cg  # noqa: E402
from oracle import bsr  # noqa: E402
from recipes import RECIPES, inputs, receiver_subset  # noqa: E402

RTOL = 1e-12


def make(name):
    t0 = time.time()
    mesh, case, u0, v0, a0, step0 = inputs(name)
    r = RECIPES[name]
    n_side = cg.CONFIGS[r["config"]].n_rec
    keep = np.array(receiver_subset(n_side, r["rec"]))
    print(f"{name}: {mesh.n_tets} tets, {3 * mesh.n_nodes} DOF, {r['steps']} steps from step {step0}", flush=True)
    S = bsr.System(mesh, case.mat, case.tet_mat)
    t1 = time.time()
    print(f"  assembled {S.blocks} blocks on {S.threads} threads in {t1 - t0:.0f} s", flush=True)
    out = S.march(case.dt, case.ray_alpha, case.ray_beta, case.v_in[step0:], r["steps"], case.rec_node[keep],
                  u0=u0, v0=v0, a0=a0, rtol=RTOL)
    t2 = time.time()
    print(f"  marched in {t2 - t1:.0f} s, CG iterations {out['iters'].min()}..{out['iters'].max()}, "
          f"max true residual {out['relres'].max():.2e}", flush=True)
    np.savez_compressed(os.path.join(HERE, name + ".npz"), rec_v=out["rec_v"], receivers=keep,
                        iters=out["iters"], relres=out["relres"], rtol=RTOL, threads=S.threads,
                        march_s=t2 - t1, u_norm=np.linalg.norm(out["u"]), v_norm=np.linalg.norm(out["v"]))


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(RECIPES)):
        make(n)
