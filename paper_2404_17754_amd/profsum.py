"""Text summaries of rocprofv3 result databases (kernel traces and HBM
counter runs) for the profiles/ folder.

    python -m paper_2404_17754_amd.profsum trace <results.db> <out.txt> "<command>"
    python -m paper_2404_17754_amd.profsum traffic <fetch.db> <write.db> <kernel substring> \
        <calibration MiB> <out.txt> "<fetch command>" "<write command>"
    python -m paper_2404_17754_amd.profsum counters <db1,db2,...> <kernel substring> \
        <elements per launch> <out.txt> "<command>" ...

The traffic summary scales FETCH_SIZE and WRITE_SIZE by what the same
counters read for the calibration copy of known size made in the same run
(bench.py --calibrate-copy-mib), and averages over full launches of the
kernel (launches that returned early after convergence are left out: their
counters are under half of the kernel's largest).
"""
from __future__ import annotations

import collections
import hashlib
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources that define the operator kernels and the layout they read
KERNEL_SOURCES = ["sw_tile.hip", "sw_elem.h", "sw_device.h", "sw_layout.h", "sw_mesh.cpp", "sw_bf16.h"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2404_17754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace(db, out, command, top=16):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(end - start), min(end - start), max(end - start), "
                       "sum(end - start) from kernels group by name order by sum(end - start) desc").fetchall()
    total = sum(r[5] for r in rows)
    lines = [f"# rocprofv3 kernel trace summary", f"command: {command}", "",
             f"{'kernel':62s} {'calls':>7s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>9s} {'total_ms':>10s} {'pct':>6s}"]
    for name, n, avg, mn, mx, tot in rows[:top]:
        short = name.split("(")[0].replace("void ", "")[:62]
        lines.append(f"{short:62s} {n:7d} {avg / 1e3:10.1f} {mn / 1e3:9.1f} {mx / 1e3:9.1f} {tot / 1e6:10.2f} "
                     f"{100.0 * tot / total:6.1f}")
    lines.append(f"(total kernel time {total / 1e6:.1f} ms over {sum(r[1] for r in rows)} dispatches)")
    # full launches of the tile kernels (early exits after convergence left out)
    for pat in ("k_tile_pipe<", "k_tile_lanes_pipe<", "k_tile<float", "k_tile<double"):
        d = [r[0] for r in con.execute("select end - start from kernels where name like ?", (f"%{pat}%",))]
        if d:
            mx = max(d)
            full = [x for x in d if x >= 0.5 * mx]
            lines.append(f"{pat}: {len(d)} launches, mean over all {sum(d) / len(d) / 1e3:.1f} us, "
                         f"mean over {len(full)} full launches {sum(full) / len(full) / 1e3:.1f} us")
    # device busy fraction over the march: the union of every kernel's
    # interval within the span from the first to the last launch of the
    # operator pass (host decisions, synchronisations and launch gaps are
    # the idle rest)
    for pat in ("k_tile_pipe<", "k_tile_lanes_pipe<"):
        w = con.execute("select min(start), max(end) from kernels where name like ?", (f"%{pat}%",)).fetchone()
        if not w or w[0] is None:
            continue
        t0, t1 = w
        iv = con.execute("select start, end from kernels where end > ? and start < ? order by start",
                         (t0, t1)).fetchall()
        busy, cur_s, cur_e = 0, None, None
        for a, b in iv:
            a, b = max(a, t0), min(b, t1)
            if cur_e is None or a > cur_e:
                if cur_e is not None:
                    busy += cur_e - cur_s
                cur_s, cur_e = a, b
            else:
                cur_e = max(cur_e, b)
        if cur_e is not None:
            busy += cur_e - cur_s
        lines.append(f"device busy over the span of the {pat} launches ({(t1 - t0) / 1e6:.1f} ms): "
                     f"{100.0 * busy / (t1 - t0):.1f} % (idle {100.0 * (1 - busy / (t1 - t0)):.1f} %)")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(db, name):
    con = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
        if c == name:
            agg[k].append(v)
    return agg


def traffic(fetch_db, write_db, pat, calib_mib, out, cmd_f, cmd_w):
    calib = calib_mib * 1024.0  # KiB
    fetch = _counter(fetch_db, "FETCH_SIZE")
    write = _counter(write_db, "WRITE_SIZE")
    # calibration: largest single copy read / largest single write of the run
    f_cal = max(max(v) for k, v in fetch.items() if "copyBuffer" in k or "elementwise" in k)
    w_cal = max(max(v) for k, v in write.items() if "copyBuffer" in k or "elementwise" in k)
    sf, sw = calib / f_cal, calib / w_cal
    kf = [v for k, vs in fetch.items() if pat in k for v in vs]
    kw = [v for k, vs in write.items() if pat in k for v in vs]
    ff = [x for x in kf if x >= 0.5 * max(kf)]
    fw = [x for x in kw if x >= 0.5 * max(kw)]
    fkib = sum(ff) / len(ff)
    wkib = sum(fw) / len(fw)
    hbm = (fkib * sf + wkib * sw) * 1024.0
    lines = ["# HBM traffic of one launch from rocprofv3 counters",
             f"kernel: {pat}", f"fetch command: {cmd_f}", f"write command: {cmd_w}",
             f"calibration copy: {calib_mib} MiB; FETCH_SIZE read {f_cal:.0f} KiB -> fetch scale {sf:.4f}; "
             f"WRITE_SIZE read {w_cal:.0f} KiB -> write scale {sw:.4f}",
             f"FETCH_SIZE per full launch: {fkib:.0f} KiB (mean of {len(ff)} of {len(kf)} launches)",
             f"WRITE_SIZE per full launch: {wkib:.0f} KiB (mean of {len(fw)} of {len(kw)} launches)",
             f"hbm_bytes_per_launch: {hbm:.6e}",
             f"kernel_sources_sha256_16: {kernel_hash()}"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


# shares of the waves' cycles (ratios of counters of the same block)
WAVE_SHARES = [("SQ_WAIT_ANY", "waiting for anything (memory or LDS results, barriers, dependencies)"),
               ("SQ_WAIT_INST_ANY", "waiting to issue any instruction"),
               ("SQ_ACTIVE_INST_VALU", "issuing VALU instructions"),
               ("SQ_ACTIVE_INST_LDS", "issuing LDS instructions"),
               ("SQ_WAIT_INST_LDS", "waiting to issue LDS instructions"),
               ("SQ_ACTIVE_INST_VMEM", "issuing vector memory instructions"),
               ("SQ_ACTIVE_INST_ANY", "issuing any instruction")]


def counters(dbs, pat, n_elems, out, cmds):
    """Mean per full launch of every counter the runs took on the kernels
    matching `pat` (launches under half a counter's largest value are left
    out), with the shares of SQ_WAVE_CYCLES and per-element figures."""
    vals = collections.defaultdict(list)
    for db in dbs:
        con = sqlite3.connect(db)
        for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
            if pat in k:
                vals[c].append(v)
    mean = {}
    lines = ["# rocprofv3 SQ counters of one launch", f"kernel: {pat}"] + [f"command: {c}" for c in cmds] + [""]
    for c in sorted(vals):
        v = vals[c]
        full = [x for x in v if x >= 0.5 * max(v)] if max(v) > 0 else v
        mean[c] = sum(full) / len(full)
        lines.append(f"{c:28s} {mean[c]:16.6e}   (mean of {len(full)} of {len(v)} launches)")
    lines.append("")
    wc = mean.get("SQ_WAVE_CYCLES")
    if wc:
        for c, what in WAVE_SHARES:
            if c in mean:
                lines.append(f"share of wave cycles {what}: {100.0 * mean[c] / wc:.1f} % ({c})")
    if "SQ_INSTS_VALU" in mean and n_elems > 0:
        lines.append(f"VALU instructions per wave step of 64 elements: {mean['SQ_INSTS_VALU'] * 64.0 / n_elems:.0f}")
    if "SQ_INSTS_LDS" in mean and n_elems > 0:
        lines.append(f"LDS instructions per wave step of 64 elements: {mean['SQ_INSTS_LDS'] * 64.0 / n_elems:.0f}")
    if "SQ_LDS_BANK_CONFLICT" in mean and mean.get("SQ_ACTIVE_INST_LDS"):
        lines.append(f"LDS bank-conflict cycles per LDS issue cycle: "
                     f"{mean['SQ_LDS_BANK_CONFLICT'] / mean['SQ_ACTIVE_INST_LDS']:.2f}")
    lines.append(f"kernel_sources_sha256_16: {kernel_hash()}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6], sys.argv[7], sys.argv[8])
    elif sys.argv[1] == "counters":
        # counters <db1,db2,...> <kernel substring> <elements per launch> <out.txt> "<command>" ...
        counters(sys.argv[2].split(","), sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6:])
    else:
        raise SystemExit(__doc__)
