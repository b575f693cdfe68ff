#!/usr/bin/env python3
"""Benchmark of the implicit wave-propagation hot path on one MI355X.

A step is one Newmark time step of the whole path: right-hand side, initial
guess, preconditioned CG to a true relative residual of 1e-8 (FP32 inner CG
inside FP64 iterative refinement), Newmark update and receiver recording.
The workload is the single large case: a 1000 x 1000 x 200 m two-layer box
with 5 m cells split into 9.6 M quadratic tetrahedra (13.0 M nodes,
39.07 M DOF), dt = 0.005 s, 2.5 Hz Ricker input; the timed region is the
whole analysis (400 steps from rest by default).  Inputs are synthetic
(seeded interface field, seeded wavelet) and resident in HBM before timing
starts.

Each step starts by default from the projection guess: the Galerkin
projection of its solution onto the span of the last 6 increments.  The
same run times, on a common window of steps from rest, the polynomial
guess, the learned guess (a network trained before timing on solution
histories that the solver generates for separate training models, 200 x
200 x 100 m boxes of the same cells, time step and input, marched together
as one batch) and the plain FP64 PCG (zero guess), and the CPU oracle on a
bounded sample of the workload.  --batched K (default 8) adds a study of K
candidate models per mesh on the three uneven meshes of the batched
workload, marched case by case, as one batch and case by case with plain
FP64 PCG; --guess-study N marches N held-out models of
the 300 x 300 x 100 m mesh with the extrapolated, learned and projected
guesses; --fit-study S runs the input estimation of Section 2.

Prints one JSON line with the metric, the roofline of the dominant kernel
(algorithmic flops and bytes / HIP-event-timed mean duration of its full
launches inside the timed region) and the comparisons.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "case-timesteps/s at rel. residual 1e-8; learned vs plain CG; EBE HBM GB/s"
HBM_PEAK_GBS = 8000.0
# FP32 vector arithmetic without packed FP32 instructions (the build
# disables them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
# the kernel class whose launches the timed region brackets with HIP events
DOMINANT = "tile_f32"
PROFILE_EVERY = 4
# FP32 flops of the element-by-element operator per tetrahedron: the
# element arithmetic's stiffness and mass action (element_apply counted on a
# counting number type, tests/flop_count.cpp), the fourth vertex gradient
# (6), and p.Ap taken from the tile's node values (3 products and 3 sums per
# node, 1.36 nodes per tet: 8).  Boundary faces and the input scaling of
# the gathered values are left out (under 2 % of a pass).
ELEMENT_FLOPS = 1143
FLOPS_PER_TET = ELEMENT_FLOPS + 6 + 8

# guesses that use the trained network
LEARNED = ("mlp", "proj_mlp")
# steps per call of a long batched march (one progress line each)
CHUNK_STEPS = 50


def progress(msg):
    """One line on stderr per phase (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# the HBM-traffic figure is only used while the operator kernel's sources are
# unchanged since the counters were taken
from paper_2404_17754_amd.profsum import kernel_hash  # noqa: E402


def algorithmic_bytes(mesh, word):
    """Bytes one application of the element-by-element operator must move
    in the reference layout: 10 int32 node ids + 1 material byte per tet,
    the input vector read once and the output written once per node, and
    the three coordinates of every vertex node read once, all values in the
    pass's word size (FP32: about 76 bytes per tet, 726 MB on the large
    case)."""
    nx, ny, nz = mesh.ncell
    n_vert = (nx + 1) * (ny + 1) * (nz + 1)
    return mesh.n_tets * (40 + 1) + mesh.n_nodes * 2 * 3 * word + n_vert * 3 * word


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg_name, dof_target, steps=20, step0=80):
    """The CPU oracle as it stands (oracle/bsr.py: FP64 symmetric 3x3
    block-sparse matrices assembled in C++, block-Jacobi CG with OpenMP on
    every host core, each step to the same 1e-8 true relative residual,
    zero initial guess) timed on a bounded sample of the workload: a
    100 x 100 m column of the large case's full depth with the same cells,
    material law, time step and input, over a window of `steps` steps from
    step `step0` (the input near its peak) with every element in motion
    (seeded smooth initial velocity field).  The rate is scaled to the
    workload by the DOF ratio (the per-iteration work of CG is proportional
    to the DOF; iteration counts depend on the cells and time step, which
    are the workload's)."""
    import numpy as np
    import casegen as cg
    from oracle import bsr
    base = cg.CONFIGS[cfg_name]
    Lz = base.box[2]
    cfg = cg.BoxConfig("sample", (100.0, 100.0, Lz), base.cell, base.h0, base.amp, base.corr,
                       base.freqs, base.t0, base.dt, step0 + steps, 4, base.seed)
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg)
    v0 = cg.smooth_field(mesh, 71, corr=40.0, amp=1e-3)
    t0 = time.perf_counter()
    S = bsr.System(mesh, case.mat, case.tet_mat)
    t_asm = time.perf_counter() - t0
    progress(f"CPU baseline: sample assembled in {t_asm:.1f} s on {S.threads} threads")
    out = S.march(case.dt, case.ray_alpha, case.ray_beta, case.v_in[step0:], steps, case.rec_node, v0=v0,
                  rtol=1e-8, guess="zero")
    dt_wall = float(out["secs"].sum())
    dof = 3 * mesh.n_nodes
    rate = steps / dt_wall * dof / dof_target
    return {"value": rate, "unit": "case-timesteps/s", "cores": S.threads, "kind": "oracle",
            "scaled": "by DOF ratio (extrapolated from the sample)",
            "host": {"logical_cpus": os.cpu_count(), "cpu_model": cpu_model(),
                     "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"), "omp_threads_used": S.threads},
            "sample": (f"native oracle (C++/OpenMP, FP64 3x3 block-sparse, block-Jacobi CG, rtol 1e-8, zero guess) "
                       f"on a 100x100x{Lz:.0f} m column of the same {base.cell:g} m cells ({mesh.n_tets} tets, "
                       f"{dof} DOF), steps {step0}-{step0 + steps} from a seeded smooth velocity field: "
                       f"{steps} steps in {dt_wall:.1f} s (mean {np.mean(out['iters']):.0f} CG iterations/step; "
                       f"assembly {t_asm:.1f} s, not timed), scaled by DOF ratio {dof}/{dof_target}")}


def train_network(sw, cg, ctx, n_cases, n_steps, train_steps, per_step=4096, batch=8192,
                  box=(200.0, 200.0, 100.0)):
    """Histories of `n_cases` training models of the batched workload
    (boxes of `box`, 5 m cells, its 2 Hz input and time step; seeded
    interface fields of amplitude 5-20 m and correlation 50-200 m, seeds
    500 on, none of them a held-out model) marched together as one batch
    with the polynomial guess, `per_step` DOFs sampled per model and step,
    then `train_steps` Adam steps on minibatches of `batch` rows on the
    GPU."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    base = cg.CONFIGS["batch200"]
    tcfg = cg.BoxConfig("train", box, base.cell, base.h0, base.amp, base.corr, base.freqs, base.t0, base.dt,
                        n_steps, 4, 500)
    tmesh = cg.config_mesh(tcfg)
    gtm = sw.Mesh(ctx, tmesh)
    lanes = []
    for k in range(n_cases):
        c = sw.Case(ctx, gtm, cg.make_case(tmesh, tcfg, seed=500 + k), precision="mixed", guess="poly")
        c.set_sampler(capacity=n_steps * per_step, per_step=per_step, seed=k)
        lanes.append(c)
    sw.Batch(ctx, lanes).step(n_steps)
    S = torch.cat([c.samples() for c in lanes])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = sw.Mlp(ctx, seed=1)
    losses = net.train(S, steps=train_steps, batch=batch, lr=2e-3, seed=5)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"training_models": n_cases, "mesh": f"{box[0]:.0f}x{box[1]:.0f}x{box[2]:.0f} m, {tmesh.n_tets} tets",
            "steps_each": n_steps,
            "rows": int(S.shape[0]), "adam_steps": train_steps, "batch": batch,
            "loss_first20": float(np.mean(losses[:20])), "loss_last20": float(np.mean(losses[-20:])),
            "collect_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
            "training_cg_iters_per_step": float(np.mean([c.step_log()[0].mean() for c in lanes]))}
    del lanes, S
    torch.cuda.empty_cache()
    return net, info


def batched_study(sw, cg, ctx, per_mesh, steps, proj_dim, legs=("seq", "batched", "plain"), sample=None):
    """Candidate models on the three uneven meshes of the batched workload
    (200/300/400 x 100 m boxes, 5 m cells; seeded interface fields), marched
    `steps` steps from rest with the projection guess: as one batch of all
    `per_mesh` models per mesh ("batched"), and case by case ("seq") and case
    by case with plain FP64 PCG and a zero guess ("plain") on the first
    `sample` models of each mesh (all of them if sample is None), the legs
    asked for.  Every case of one mesh costs the same per step, and the
    sample keeps the mix of meshes, so the rates in case-timesteps/s
    compare."""
    import numpy as np
    import torch
    meshes, cases, in_sample = [], [], []
    sample = per_mesh if sample is None else min(sample, per_mesh)
    for name in ("batch200", "batch300", "batch400"):
        cfg = cg.CONFIGS[name]
        m = cg.config_mesh(cfg)
        gm = sw.Mesh(ctx, m)
        meshes.append((name, m.n_tets))
        for k in range(per_mesh):
            cases.append((gm, cg.make_case(m, cfg, seed=cfg.seed + 3 * k + len(cases), n_steps=steps)))
            in_sample.append(k < sample)
        progress(f"batched study: {per_mesh} models of {name} generated")

    tuned = {}

    def run(batched, precision="mixed", guess="proj"):
        sel = cases if batched else [c for c, s in zip(cases, in_sample) if s]
        lanes = [sw.Case(ctx, gm, c, precision=precision, guess=guess, proj_dim=proj_dim) for gm, c in sel]
        b = None
        if batched:
            # set-up-time choice of the lane pass's schedule (not timed)
            b = sw.Batch(ctx, lanes)
            choice, ms = b.autotune(reps=3)
            tuned.update({"choice": int(choice), "candidates_ms": [round(float(v), 4) for v in ms],
                          "candidates": ["mesh after mesh, 3 workgroups/CU", "mesh after mesh, 2/CU",
                                         "meshes interleaved tile by tile, 3/CU", "interleaved, 2/CU"]})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            # chunks of steps with a progress line each (a long march is
            # otherwise silent for minutes)
            done = 0
            while done < steps:
                n = min(CHUNK_STEPS, steps - done)
                b.step(n)
                done += n
                if done < steps:
                    progress(f"batched study: {len(sel)} models at step {done} of {steps}")
        else:
            for k, lane in enumerate(lanes):
                lane.step(steps)
                if steps > CHUNK_STEPS:
                    progress(f"batched study ({precision}/{guess}, case by case): model {k + 1} of {len(lanes)}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        progress(f"batched study leg ({'batched' if batched else 'case by case'}, {precision}/{guess}): "
                 f"{len(sel)} models x {steps} steps in {dt:.1f} s")
        its = np.concatenate([lane.step_log()[0] for lane in lanes]).astype(np.float64)
        worst = float(max(lane.stats()["max_true_rel_res"] for lane in lanes))
        del lanes, b
        torch.cuda.empty_cache()
        return len(sel) * steps / dt, float(its.mean()), worst

    out = {"meshes": [f"{n}: {t} tets" for n, t in meshes], "cases": len(cases), "steps": steps,
           "sequential_and_plain_sample": f"{sample} models per mesh ({3 * sample})",
           "guess": f"proj (L={proj_dim})", "cg_iters_per_step": {}}
    worst = 0.0
    if "seq" in legs:
        seq, its, w = run(False)
        out["sequential_case_timesteps_per_s"] = round(seq, 2)
        out["cg_iters_per_step"]["sequential"] = round(its, 2)
        worst = max(worst, w)
    if "batched" in legs:
        bat, its, w = run(True)
        out["batched_case_timesteps_per_s"] = round(bat, 2)
        out["cg_iters_per_step"]["batched"] = round(its, 2)
        worst = max(worst, w)
    if "plain" in legs:
        plain, its, _ = run(False, precision="fp64", guess="zero")
        out["plain_fp64_sequential_case_timesteps_per_s"] = round(plain, 2)
        out["cg_iters_per_step"]["plain_fp64"] = round(its, 2)
    if "seq" in legs and "batched" in legs:
        out["speedup"] = round(bat / seq, 3)
    if "plain" in legs and "batched" in legs:
        out["batched_vs_plain_fp64"] = round(bat / plain, 3)
    out["max_true_rel_res"] = worst
    if tuned:
        out["batch_autotune"] = tuned
    return out


def guess_study(sw, cg, ctx, net, n_models, steps, proj_dim):
    """The learned guess on held-out candidate models: `n_models` models of
    the 300 x 300 x 100 m mesh (5 m cells; seeded interface fields of the
    batched workload, seeds unseen in training), each marched `steps` steps
    from rest once per guess (extrapolation, the trained network, the
    projection, the projection with the network's direction), every guess
    as one batch.  CG iterations per step (mean, median, 95th percentile
    over models and steps), the worst true relative residual and the
    batch's case-timesteps/s; and the network's loss on rows sampled from
    the held-out marches against the extrapolation's."""
    import numpy as np
    import torch
    cfg = cg.CONFIGS["batch300"]
    mesh = cg.config_mesh(cfg)
    gm = sw.Mesh(ctx, mesh)
    models = [cg.make_case(mesh, cfg, seed=2000 + k, n_steps=steps) for k in range(n_models)]
    progress(f"learned-guess study: {n_models} held-out models generated")
    out = {"mesh": f"300x300x100 m, {mesh.n_tets} tets, {3 * mesh.n_nodes} DOF", "models": n_models,
           "seeds": f"2000-{2000 + n_models - 1}", "steps": steps}
    for g in ("poly", "mlp", "proj", "proj_mlp"):
        lanes = [sw.Case(ctx, gm, c, precision="mixed", guess=g, proj_dim=proj_dim) for c in models]
        if g in LEARNED:
            for lane in lanes:
                lane.attach_mlp(net)
        if g == "poly":
            # rows of the held-out marches, for the network's loss on them
            for k, lane in enumerate(lanes):
                lane.set_sampler(capacity=steps * 512, per_step=512, seed=7000 + k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw.Batch(ctx, lanes).step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        progress(f"learned-guess study: guess {g} done in {dt:.1f} s")
        its = np.concatenate([lane.step_log()[0] for lane in lanes]).astype(np.float64)
        if g == "poly":
            S = torch.cat([lane.samples() for lane in lanes])
            _, l_net = net.gradient(S)
            _, l_ext = sw.Mlp(ctx, seed=1).gradient(S)  # zero output layer: the extrapolation itself
            out["heldout_loss"] = {"rows": int(S.shape[0]), "trained": l_net, "extrapolation": l_ext,
                                   "note": "loss of the guess's correction (sum s^2 (y - t)^2 / sum s^2) on rows "
                                           "sampled from the held-out marches"}
            del S
        out[g] = {"cg_iters_per_step": round(float(its.mean()), 2), "p50": float(np.percentile(its, 50)),
                  "p95": float(np.percentile(its, 95)),
                  "max_true_rel_res": float(max(lane.stats()["max_true_rel_res"] for lane in lanes)),
                  "fallback_models": int(sum(1 for lane in lanes if lane.stats()["flags"] & 4)),
                  "case_timesteps_per_s": round(n_models * steps / dt, 2)}
        del lanes
        torch.cuda.empty_cache()
    for a, b in (("mlp", "poly"), ("proj", "poly"), ("proj_mlp", "poly"), ("proj_mlp", "proj")):
        out[f"{a}_vs_{b}_iters"] = round(out[a]["cg_iters_per_step"] / out[b]["cg_iters_per_step"], 4)
    return out


def sweep_study(sw, cg, ctx, n_models, steps, proj_dim):
    """The full sweep's batch shape: the sweep's reference model (seed 2999)
    and `n_models` - 1 candidates (seeds 3000 on) of the 1000 x 1000 x 100 m
    mesh (5 m cells, 19.78 M DOF; 50 x 50 receivers; Ricker 1 + 2 + 4 Hz,
    t0 = 1 s) marched `steps` steps from rest as one batch; each candidate's
    ERR against the reference model's surface velocities over those steps
    and the ranking; the batch's throughput, and the time of the whole sweep
    (1000 models x 2000 steps in batches of this size) at that rate, which
    is an extrapolation (later steps, with the wave in the model, need
    fewer CG iterations than the first ones)."""
    import numpy as np
    import torch
    cfg = cg.CONFIGS["sweep"]
    mesh = cg.config_mesh(cfg)
    gm = sw.Mesh(ctx, mesh)
    seeds = [cfg.seed - 1] + [cfg.seed + k for k in range(n_models - 1)]
    lanes = [sw.Case(ctx, gm, cg.make_case(mesh, cfg, seed=sd, n_steps=steps), precision="mixed", guess="proj",
                     proj_dim=proj_dim) for sd in seeds]
    progress(f"sweep study: {n_models} models of the sweep mesh set up")
    b = sw.Batch(ctx, lanes)
    choice, ms = b.autotune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(CHUNK_STEPS, steps - done)
        b.step(n)
        done += n
        progress(f"sweep study: step {done} of {steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    obs = lanes[0].waveform_device()
    errs = [lane.misfit(obs)[0] for lane in lanes[1:]]
    order = np.argsort(errs)
    its = np.concatenate([lane.step_log()[0] for lane in lanes]).astype(np.float64)
    rate = n_models * steps / dt
    out = {"mesh": f"1000x1000x100 m, {mesh.n_tets} tets, {3 * mesh.n_nodes} DOF", "models": n_models,
           "reference_seed": seeds[0], "candidate_seeds": f"{seeds[1]}-{seeds[-1]}", "steps": steps,
           "receivers": len(lanes[0].waveforms(0, 1)[0]), "case_timesteps_per_s": round(rate, 2),
           "dof_steps_per_s": float(f"{rate * 3 * mesh.n_nodes:.4g}"),
           "cg_iters_per_step": round(float(its.mean()), 2), "p95": float(np.percentile(its, 95)),
           "max_true_rel_res": float(max(lane.stats()["max_true_rel_res"] for lane in lanes)),
           "flags": int(np.bitwise_or.reduce([lane.stats()["flags"] for lane in lanes])),
           "err_best5": [(int(seeds[1 + i]), round(float(errs[i]), 4)) for i in order[:5]],
           "err_median": round(float(np.median(errs)), 4),
           "batch_autotune_choice": int(choice), "batch_autotune_ms": [round(float(v), 3) for v in ms],
           "whole_sweep_h_extrapolated": round(1000 * 2000 / rate / 3600.0, 2)}
    del lanes, b, obs
    torch.cuda.empty_cache()
    return out


def fit_study(sw, cg, ctx, n_steps, stride, proj_dim):
    """Section 2's input estimation for one candidate model of the batched
    workload (300 x 300 x 100 m, 5 m cells, 20 x 20 receivers): the model's
    three Green's runs (unit Hann impulse along x1, x2, x3) marched as one
    batch, a reference model driven by the Ricker input as the observation,
    then the fit (weighted normal equations on the GPU, pseudo-inverse on
    the host, response and ERR on the GPU)."""
    import torch
    cfg = cg.CONFIGS["batch300"]
    mesh = cg.config_mesh(cfg)
    gm = sw.Mesh(ctx, mesh)
    model = cg.make_case(mesh, cfg, seed=cfg.seed, n_steps=n_steps)
    ref = cg.make_case(mesh, cfg, seed=cfg.seed - 1, n_steps=n_steps)
    lanes = []
    for v_in in cg.impulse_inputs(n_steps, stride):
        c = cg.Case(mat=model.mat, tet_mat=model.tet_mat, rec_node=model.rec_node, v_in=v_in, dt=model.dt,
                    n_steps=n_steps, ray_alpha=model.ray_alpha, ray_beta=model.ray_beta, meta={})
        lanes.append(sw.Case(ctx, gm, c, precision="mixed", guess="proj", proj_dim=proj_dim))
    obs_case = sw.Case(ctx, gm, ref, precision="mixed", guess="proj", proj_dim=proj_dim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sw.Batch(ctx, lanes + [obs_case]).step(n_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    green = [torch.from_numpy(l.waveforms()).cuda() for l in lanes]
    obs = torch.from_numpy(obs_case.waveforms()).cuda()
    n_shift = n_steps // stride
    sw.fit_input(ctx, green, obs, stride, n_shift)          # warm-up
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    c, e, used, rank = sw.fit_input(ctx, green, obs, stride, n_shift)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    del lanes, obs_case
    torch.cuda.empty_cache()
    return {"mesh": f"batch300: {mesh.n_tets} tets, {3 * mesh.n_nodes} DOF", "steps": n_steps,
            "receivers": int(obs.shape[1]), "stride_steps": stride, "shifts": n_shift,
            "runs_s (3 Green's + 1 observation, one batch)": round(t1 - t0, 2),
            "fit_ms": round(1e3 * (t3 - t2), 2), "err_vs_other_model": round(e, 4), "pairs": used, "rank": rank}


def solver_study(sw, ctx, gmesh, case, steps, guess, proj_dim, windows=(20, 100, 400)):
    """The two outer solvers around the FP32 inner CG on the workload from
    rest: iterative refinement ("mixed") and the flexible CG ("flex"), each
    marched `steps` steps with per-step HIP-event timing; ms per step, CG
    iterations and FP64 operator passes per step over the windows of steps
    0-w."""
    import numpy as np
    import torch
    out = {"steps": steps, "guess": guess}
    for prec in ("mixed", "flex"):
        progress(f"outer-solver study: {prec}")
        c = sw.Case(ctx, gmesh, case, rtol=1e-8, precision=prec, guess=guess, proj_dim=proj_dim)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        outer = []
        for k in range(steps):
            c.step(1)
            ev[k + 1].record()
            outer.append(c.stats()["ir_outer"])
        torch.cuda.synchronize()
        ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        it, rel = c.step_log(0, steps)
        outer = np.diff(np.concatenate([[0], outer]))
        out[prec] = {f"0-{w}": {"ms_per_step": round(float(ms[:w].mean()), 3),
                                "cg_iters_per_step": round(float(it[:w].mean()), 2),
                                "fp64_passes_per_step": round(float(outer[:w].mean()), 3)}
                     for w in windows if w <= steps}
        out[prec]["max_true_rel_res"] = float(rel.max())
        del c
        torch.cuda.empty_cache()
    return out


def timed_window(sw, ctx, gmesh, case, n, **kw):
    """A fresh case marched `n` steps from rest; ms per step and the step
    log."""
    import torch
    c = sw.Case(ctx, gmesh, case, rtol=1e-8, **{k: v for k, v in kw.items() if k != "net"})
    if kw.get("net") is not None:
        c.attach_mlp(kw["net"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    c.step(n)
    e1.record()
    torch.cuda.synchronize()
    it, rel = c.step_log()
    st = c.stats()
    del c
    torch.cuda.empty_cache()
    return e0.elapsed_time(e1) / n, it, rel, st


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed steps (from rest; 400 = the whole analysis)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed steps on a separate copy of the case")
    ap.add_argument("--config", default="large")
    ap.add_argument("--guess", default="proj", choices=["zero", "poly", "mlp", "proj", "proj_mlp"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "flex", "fp16"],
                    help="outer solver around the FP32 inner CG: iterative refinement, flexible CG, or "
                         "refinement with the inner CG's direction stored in 16 bits")
    ap.add_argument("--proj-dim", type=int, default=6, help="past increments spanned by the projection guess")
    ap.add_argument("--inner-rtol", type=float, default=0.0,
                    help="floor of the inner FP32 CG tolerance (0 = the library default)")
    ap.add_argument("--compare-steps", type=int, default=100,
                    help="window (from rest) on which the other guesses and plain FP64 PCG are timed (0 = skip)")
    ap.add_argument("--no-mlp-compare", action="store_true", help="leave the trained-network leg out")
    ap.add_argument("--batched", type=int, default=86,
                    help="cases per mesh of the batched study on the 200/300/400 m meshes (0: none)")
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--batched-sample", type=int, default=8,
                    help="cases per mesh marched case by case (sequential and plain FP64 legs)")
    ap.add_argument("--batched-legs", default="seq,batched,plain",
                    help="legs of the batched study: seq, batched, plain (comma separated)")
    ap.add_argument("--guess-study", type=int, default=64,
                    help="held-out models of the 300 m mesh for the learned-guess study (0: none)")
    ap.add_argument("--guess-study-steps", type=int, default=100)
    ap.add_argument("--solver-study", type=int, default=0,
                    help="steps (from rest) of the outer-solver study: refinement vs flexible CG (0 = skip)")
    ap.add_argument("--sweep-study", default="",
                    help="models,steps of an extra sweep study (reference + candidates of the 1000 m sweep mesh "
                         "in one batch; empty = skip)")
    ap.add_argument("--fit-study", type=int, default=0,
                    help="steps of an extra input-estimation study (Green's runs + fit) on the 300 m mesh (0 = skip)")
    ap.add_argument("--train-cases", type=int, default=16)
    ap.add_argument("--train-box", default="200,200,100", help="training models' box (m)")
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--adam-steps", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: the analyses of different candidate models are "
                                   "independent, so N GPUs would each march their own share of cases; "
                                   "only --gpus 1 is measured"}))
        sys.exit(2)

    import numpy as np
    import torch

    import casegen as cg
    import paper_2404_17754_amd as sw

    cfg = cg.CONFIGS[args.config]
    cmp_n = min(args.compare_steps, args.steps)
    t_gen = time.perf_counter()
    mesh = cg.config_mesh(cfg)
    case = cg.make_case(mesh, cfg, n_steps=max(args.steps, args.warmup, cmp_n) + 1)
    t_gen = time.perf_counter() - t_gen
    dof = 3 * mesh.n_nodes

    progress("mesh generated")
    ctx = sw.Context(0)
    t_up = time.perf_counter()
    gmesh = sw.Mesh(ctx, mesh)
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t_up

    net, train_info = None, None
    if args.guess in LEARNED or args.guess_study > 0 or (args.compare_steps > 0 and not args.no_mlp_compare):
        net, train_info = train_network(sw, cg, ctx, args.train_cases, args.train_steps, args.adam_steps,
                                        box=tuple(float(v) for v in args.train_box.split(",")))

    progress("network trained")
    # warm-up on a separate copy of the case
    if args.warmup > 0:
        w = sw.Case(ctx, gmesh, case, rtol=1e-8, precision=args.precision, guess=args.guess,
                    proj_dim=args.proj_dim, inner_rtol=args.inner_rtol)
        if args.guess in LEARNED:
            w.attach_mlp(net)
        w.step(args.warmup)
        torch.cuda.synchronize()
        del w
        torch.cuda.empty_cache()

    gc = sw.Case(ctx, gmesh, case, rtol=1e-8, precision=args.precision, guess=args.guess, proj_dim=args.proj_dim,
                 inner_rtol=args.inner_rtol)
    if args.guess in LEARNED:
        gc.attach_mlp(net)
    # set-up-time choice of the FP32 pass's workgroups per CU (not timed)
    tune_choice, tune_ms = gc.autotune(reps=5)
    case_tune = {"choice": ["3 workgroups/CU", "2/CU", "1/CU"][int(tune_choice)],
                 "candidates_ms": [round(float(v), 4) for v in tune_ms]}
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    # HIP events bracket launches of the dominant kernel only (the FP32
    # element-by-element pass: about half of the kernel time in the
    # rocprofv3 trace of this run, the rest split over many smaller
    # kernels), one in PROFILE_EVERY of them (every launch does the same
    # work); each event pair adds several microseconds to the timed work
    ctx.profile(True, kinds=(DOMINANT,), every=PROFILE_EVERY)
    torch.cuda.synchronize()
    e0, em, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    w0 = time.perf_counter()
    e0.record()
    gc.step(cmp_n)
    em.record()
    gc.step(args.steps - cmp_n)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    ms_window = e0.elapsed_time(em) / cmp_n if cmp_n > 0 else None
    kernels = {DOMINANT: ctx.profile_read(DOMINANT)}
    ctx.profile(False)
    it, rel = gc.step_log(0, args.steps)
    stats = gc.stats()
    value = 1000.0 / ms_per_step  # one case
    del gc
    torch.cuda.empty_cache()

    progress("timed region done")
    # the dominant kernel of the timed region: the FP32 element-by-element pass
    dom = DOMINANT
    tot_ms, n_launch, full_ms, n_full = kernels[dom]
    avg_s = full_ms / 1e3  # full launches (early exits after convergence left out)
    abytes = algorithmic_bytes(mesh, 4)
    aflops = FLOPS_PER_TET * mesh.n_tets
    traffic = read_traffic(dom)
    tflops = aflops / avg_s / 1e12
    gbs = abytes / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 1), "launches": n_full,
                "launches_incl_early_exit": n_launch, "timed_one_launch_in": PROFILE_EVERY,
                "algorithmic_bytes_per_launch": abytes,
                "bytes_per_tet": round(abytes / mesh.n_tets, 2),
                "counter_traffic_GBs": None if traffic is None else round(traffic / avg_s / 1e9, 1),
                "alu": {"achieved": round(tflops, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / ALU_PEAK_TFLOPS, 4), "algorithmic_flops_per_launch": aflops,
                        "flops_per_tet": FLOPS_PER_TET, "intensity_flop_per_byte": round(aflops / abytes, 2),
                        "ridge_flop_per_byte": round(ALU_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS, 2),
                        "peak_note": "FP32 vector FMA without packed instructions (the build disables them)"}}

    # comparisons on the common window of steps from rest
    compare = None
    if cmp_n > 0:
        compare = {"window_steps": cmp_n,
                   args.guess: {"ms_per_step": round(ms_window, 2), "value": round(1000.0 / ms_window, 3),
                                "cg_iters_per_step": float(np.mean(it[:cmp_n]))}}
        legs = [(g, dict(precision=args.precision, guess=g, proj_dim=args.proj_dim,
                         net=net if g in LEARNED else None))
                for g in ("poly", "mlp", "proj", "proj_mlp") if g != args.guess and (g not in LEARNED or net is not None)]
        for other in ("mixed", "flex", "fp16"):
            if other != args.precision:
                legs.append((f"{other}_{args.guess}", dict(precision=other, guess=args.guess, proj_dim=args.proj_dim,
                                                            net=net if args.guess in LEARNED else None)))
        legs.append(("plain_fp64", dict(precision="fp64", guess="zero")))
        for name, kw in legs:
            ms, pit, prel, pst = timed_window(sw, ctx, gmesh, case, cmp_n, **kw)
            compare[name] = {"ms_per_step": round(ms, 2), "value": round(1000.0 / ms, 3),
                             "cg_iters_per_step": float(np.mean(pit)), "max_true_rel_res": float(np.max(prel)),
                             "flags": pst["flags"]}
        compare["speedup_vs_plain_fp64"] = round(compare["plain_fp64"]["ms_per_step"] / ms_window, 3)
        compare["plain_fp64"]["method"] = "FP64 block-Jacobi PCG, zero initial guess"

    progress("comparison legs done")
    solvers = None
    if args.solver_study > 0:
        case_s = cg.make_case(mesh, cfg, n_steps=args.solver_study + 1)
        solvers = solver_study(sw, ctx, gmesh, case_s, args.solver_study, args.guess, args.proj_dim)

    batched = None
    if args.batched > 0:
        gmesh = None
        torch.cuda.empty_cache()
        batched = batched_study(sw, cg, ctx, args.batched, args.batched_steps, args.proj_dim,
                                tuple(args.batched_legs.split(",")), sample=args.batched_sample)

    progress("batched study done")
    gstudy = None
    if args.guess_study > 0:
        torch.cuda.empty_cache()
        gstudy = guess_study(sw, cg, ctx, net, args.guess_study, args.guess_study_steps, args.proj_dim)

    fit = None
    if args.fit_study > 0:
        torch.cuda.empty_cache()
        fit = fit_study(sw, cg, ctx, args.fit_study, 20, args.proj_dim)

    sweep = None
    if args.sweep_study:
        gmesh = None
        torch.cuda.empty_cache()
        k, n = (int(v) for v in args.sweep_study.split(","))
        sweep = sweep_study(sw, cg, ctx, k, n, args.proj_dim)

    progress("studies done; CPU baseline next")
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.config, dof)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "case-timesteps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32+f64" if args.precision == "fp16" else "f32+f64", "data": "synthetic",
        "config": {"workload": (f"{args.config}: {cfg.box[0]:.0f}x{cfg.box[1]:.0f}x{cfg.box[2]:.0f} m, "
                                f"{cfg.cell:g} m cells, {mesh.n_tets} P2 tets, {dof} DOF, dt {cfg.dt} s, "
                                f"Ricker {cfg.freqs} Hz, one case, steps 0-{args.steps} from rest"),
                   "precision": {"mixed": "FP32 inner CG in FP64 refinement",
                                 "flex": "FP32 inner CG preconditioning FP64 flexible CG",
                                 "fp16": "FP32 inner CG with a bfloat16 direction vector in FP64 refinement"}[
                                     args.precision],
                   "guess": args.guess, "rtol": 1e-8,
                   "parallelism": "single GPU"},
        "cg_iters_per_step": float(np.mean(it)), "refinement_rounds_per_step": round(stats["ir_outer"] / stats["steps"], 3),
        "max_true_rel_res": float(np.max(rel)),
        "flags": stats["flags"], "wall_s_timed": round(wall, 3),
        "setup_s": {"host_generation": round(t_gen, 2), "mesh_upload_and_layout": round(t_up, 2)},
        "autotune": case_tune,
        "learned_guess_training": train_info,
        "kernels_ms": {k: {"total_ms": round(v[0], 3), "launches": v[1], "full_launch_us": round(1e3 * v[2], 1),
                           "timed_one_launch_in": PROFILE_EVERY}
                       for k, v in kernels.items() if v[1]},
        "roofline": roofline, "compare": compare, "outer_solvers": solvers, "batched": batched,
        "learned_guess_study": gstudy,
        "input_estimation": fit, "sweep": sweep, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
