#!/usr/bin/env python3
"""Benchmark of the implicit wave-propagation hot path on one MI355X.

A step is one Newmark time step of the whole path: right-hand side, initial
guess, preconditioned CG to a true relative residual of 1e-8 (FP32 inner CG
inside FP64 iterative refinement by default), Newmark update and receiver
recording.  The workload is the single large case: a 1000 x 1000 x 200 m
two-layer box with 5 m cells split into 9.6 M quadratic tetrahedra
(13.0 M nodes, 39.07 M DOF), dt = 0.005 s, 2.5 Hz Ricker input.  Inputs are
synthetic (seeded interface field, seeded wavelet) and resident in HBM
before timing starts.

Prints one JSON line with the metric, the roofline of the dominant kernel
(algorithmic bytes / HIP-event-timed average duration inside the timed
region), the plain FP64 PCG comparison on the same workload and the CPU
oracle timed on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "case-timesteps/s at rel. residual 1e-8; learned vs plain CG; EBE HBM GB/s"
HBM_PEAK_GBS = 8000.0

# the HBM-traffic figure is only used while the operator kernel's sources are
# unchanged since the counters were taken
from paper_2404_17754_amd.profsum import kernel_hash  # noqa: E402


def algorithmic_bytes(mesh, word):
    """Bytes one application of the element-by-element operator must move
    in the reference layout: 10 int32 node ids + 1 material byte per tet,
    the input vector read once and the output written once per node, and
    the coordinates of every vertex node read once."""
    n_vert = len(set(mesh.tet10[:, :4].ravel().tolist())) if mesh.n_tets < 200000 else None
    if n_vert is None:
        nx, ny, nz = mesh.ncell
        n_vert = (nx + 1) * (ny + 1) * (nz + 1)
    return mesh.n_tets * (40 + 1) + mesh.n_nodes * 2 * 3 * word + n_vert * 3 * 8


def read_traffic(kind):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    when it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kind}_large_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_sources_sha256_16:\s*(\w+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


def cpu_baseline(cfg_name, dof_target, steps=4):
    """The CPU oracle (FP64, assembled sparse matrices, conjugate gradients
    with a Jacobi preconditioner to the same 1e-8 relative residual) timed on
    a bounded sample of the workload: a 100 x 100 x 50 m box with the same
    5 m cells, material law, time step and input, marched `steps` steps.
    The rate is scaled to the workload by the DOF ratio."""
    import numpy as np  # noqa: F401
    import casegen as cg
    from oracle import march
    base = cg.CONFIGS[cfg_name]
    cfg = cg.BoxConfig("sample", (100.0, 100.0, 50.0), base.cell, min(base.h0, 25.0), base.amp, base.corr,
                       base.freqs, base.t0, base.dt, steps, 4, base.seed)
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg, n_steps=steps)
    sys_ = march.build_system(mesh, case)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = march.run(sys_, case.dt, case.v_in, steps, case.rec_node, solver="cg", rtol=1e-8)
        dt_wall = time.perf_counter() - t0
    dof = 3 * mesh.n_nodes
    rate = steps / dt_wall * dof / dof_target
    return {"value": rate, "unit": "case-timesteps/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 sparse CG (Jacobi, rtol 1e-8) on a 100x100x50 m box of the same 5 m cells "
                       f"({mesh.n_tets} tets, {dof} DOF), {steps} steps in {dt_wall:.1f} s "
                       f"(mean {np.mean(r.iters):.0f} CG iterations/step), scaled by DOF ratio {dof}/{dof_target}; "
                       f"one thread (BLAS limited to 1), host has {os.cpu_count()} logical CPUs")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="large")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--guess", default="poly", choices=["zero", "poly"])
    ap.add_argument("--plain-steps", type=int, default=6, help="steps of the plain FP64 PCG comparison (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the analyses of different candidate models are "
                                   "independent, so N GPUs would each march their own share of cases; "
                                   "only --gpus 1 is measured"}))
        sys.exit(2)

    import numpy as np
    import torch

    import casegen as cg
    import paper_2404_17754_amd as sw

    cfg = cg.CONFIGS[args.config]
    n_total = args.warmup + args.steps + 1
    t_gen = time.perf_counter()
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg, n_steps=max(n_total, args.warmup + args.plain_steps + 1))
    t_gen = time.perf_counter() - t_gen
    dof = 3 * mesh.n_nodes

    ctx = sw.Context(0)
    t_up = time.perf_counter()
    gmesh = sw.Mesh(ctx, mesh)
    gc = sw.Case(ctx, gmesh, case, rtol=1e-8, precision=args.precision, guess=args.guess)
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t_up

    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    gc.step(args.warmup)
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    gc.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    kernels = {k: ctx.profile_read(k) for k in ("tile_f64", "tile_f32", "update_f64", "update_f32",
                                                "dir_f64", "dir_f32")}
    ctx.profile(False)
    it, rel = gc.step_log(args.warmup, args.steps)
    stats = gc.stats()
    value = 1000.0 / ms_per_step  # one case

    # dominant kernel of the timed region
    dom = max(kernels, key=lambda k: kernels[k][0])
    tot_ms, n_launch, full_ms, n_full = kernels[dom]
    avg_s = full_ms / 1e3  # full launches (early exits after convergence left out)
    if dom.startswith("tile"):
        word = 4 if dom.endswith("f32") else 8
        abytes = algorithmic_bytes(mesh, word)
    else:
        word = 4 if dom.endswith("f32") else 8
        abytes = {"update": (4 * 3 * word + 6 * word + 4 * 3 * word),
                  "dir": 3 * 3 * word}[dom.split("_")[0]] * mesh.n_nodes
    achieved = abytes / avg_s / 1e9
    traffic = read_traffic(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 1), "launches": n_full,
                "launches_incl_early_exit": n_launch,
                "algorithmic_bytes_per_launch": abytes}

    plain = None
    if args.plain_steps > 0:
        del gc
        torch.cuda.empty_cache()
        gp = sw.Case(ctx, gmesh, case, rtol=1e-8, precision="fp64", guess="zero")
        gp.step(args.warmup)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        gp.step(args.plain_steps)
        p1.record()
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1) / args.plain_steps
        pit, _ = gp.step_log(args.warmup, args.plain_steps)
        plain = {"value": round(1000.0 / pms, 3), "ms_per_step": round(pms, 2),
                 "cg_iters_per_step": float(np.mean(pit)), "speedup_of_value": round(value / (1000.0 / pms), 3),
                 "method": "FP64 block-Jacobi PCG, zero initial guess, same steps"}
        del gp

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.config, dof)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "case-timesteps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": (f"{args.config}: {cfg.box[0]:.0f}x{cfg.box[1]:.0f}x{cfg.box[2]:.0f} m, "
                                f"{cfg.cell:g} m cells, {mesh.n_tets} P2 tets, {dof} DOF, dt {cfg.dt} s, "
                                f"Ricker {cfg.freqs} Hz, one case"),
                   "precision": args.precision, "guess": args.guess, "rtol": 1e-8,
                   "parallelism": "single GPU"},
        "cg_iters_per_step": float(np.mean(it)), "max_true_rel_res": float(np.max(rel)),
        "flags": stats["flags"], "wall_s_timed": round(wall, 3),
        "setup_s": {"host_generation": round(t_gen, 2), "upload_and_setup": round(t_up, 2)},
        "kernels_ms": {k: {"total_ms": round(v[0], 3), "launches": v[1], "full_launch_us": round(1e3 * v[2], 1)}
                       for k, v in kernels.items() if v[1]},
        "roofline": roofline, "plain_fp64": plain, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
