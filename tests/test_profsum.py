"""The profile summariser (paper_2404_17754_amd/profsum.py) and the bench's
reader of its HBM-traffic summary, on synthetic rocprofv3 result databases
with known answers: counters are scaled by the calibration copy of the same
run, launches that returned early (under half the largest) are left out,
and a traffic summary counts only while it was taken on the current kernel
sources."""
import os
import re
import sqlite3

import pytest

import bench
from paper_2404_17754_amd import profsum


def _counter_db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", [(k, counter, v) for k, v in rows])
    con.commit()
    con.close()


def _value(txt, key):
    return float(re.search(key + r":\s*([0-9.eE+-]+)", txt).group(1))


def test_traffic_scaling_and_full_launches(tmp_path):
    # a 1 MiB calibration copy: FETCH_SIZE reads half its bytes (scale 2),
    # WRITE_SIZE all of them (scale 1); one early-exit launch per counter
    tile = "void sw::k_tile_pipe<256, 5, false>(sw::MeshDev, ...)"
    f = tmp_path / "fetch.db"
    w = tmp_path / "write.db"
    _counter_db(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 512.0), ("__amd_rocclr_copyBuffer", 3.0),
                                  (tile, 10.0), (tile, 1000.0), (tile, 1002.0), (tile, 998.0)])
    _counter_db(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1024.0), (tile, 5.0), (tile, 400.0), (tile, 400.0)])
    out = tmp_path / "traffic.txt"
    profsum.traffic(str(f), str(w), "k_tile_pipe", 1, str(out), "fetch cmd", "write cmd")
    txt = out.read_text()
    # (1000 KiB x 2 + 400 KiB x 1) per full launch
    assert _value(txt, "hbm_bytes_per_launch") == pytest.approx((1000.0 * 2 + 400.0) * 1024, rel=1e-6)
    assert "mean of 3 of 4 launches" in txt and "mean of 2 of 3 launches" in txt
    assert re.search(r"kernel_sources_sha256_16:\s*" + profsum.kernel_hash(), txt)


def test_trace_full_launch_mean(tmp_path):
    db = tmp_path / "trace.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = [("void sw::k_tile_pipe<256, 5, false>(...)", 0, 400_000), ("void sw::k_tile_pipe<256, 5, false>(...)", 0, 440_000),
            ("void sw::k_tile_pipe<256, 5, false>(...)", 0, 1_000), ("sw::k_newmark(...)", 0, 500_000)]
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    out = tmp_path / "trace.txt"
    profsum.trace(str(db), str(out), "trace cmd")
    txt = out.read_text()
    # full launches: 400 and 440 us (the 1 us early exit is left out)
    assert "k_tile_pipe<: 3 launches" in txt and "mean over 2 full launches 420.0 us" in txt
    assert "(total kernel time 1.3 ms over 4 dispatches)" in txt


def test_bench_reads_traffic_only_for_current_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("tile_f32") is None          # no summary
    os.makedirs(tmp_path / "profiles")
    p = tmp_path / "profiles" / "tile_f32_large_hbm_traffic.txt"
    p.write_text(f"hbm_bytes_per_launch: 1.25e+09\nkernel_sources_sha256_16: {profsum.kernel_hash()}\n")
    assert bench.read_traffic("tile_f32") == 1.25e9
    p.write_text("hbm_bytes_per_launch: 1.25e+09\nkernel_sources_sha256_16: 0000000000000000\n")
    assert bench.read_traffic("tile_f32") is None          # taken on other sources


def test_trace_device_busy_fraction(tmp_path):
    # operator passes span 0 .. 1000 us; kernels cover 0-300, 250-400 (an
    # overlap), 600-700 and 900-1000 us: busy 600 of 1000 us.  A kernel
    # outside the span does not count.
    db = tmp_path / "trace.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer)")
    tile = "void sw::k_tile_pipe<256, 5, false>(...)"
    rows = [(tile, 0, 300_000), ("sw::k_cg_update(...)", 250_000, 400_000), ("sw::k_cg_dir(...)", 600_000, 700_000),
            (tile, 900_000, 1_000_000), ("sw::k_newmark(...)", 2_000_000, 2_500_000)]
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    out = tmp_path / "trace.txt"
    profsum.trace(str(db), str(out), "trace cmd")
    txt = out.read_text()
    assert "device busy over the span of the k_tile_pipe< launches (1.0 ms): 60.0 % (idle 40.0 %)" in txt


def test_counter_summary_shares_and_per_element(tmp_path):
    tile = "void sw::k_tile_pipe<256, 5, false>(...)"
    a = tmp_path / "p1.db"
    b = tmp_path / "p2.db"
    _counter_db(a, "SQ_WAVE_CYCLES", [(tile, 1000.0), (tile, 1000.0), (tile, 3.0), ("other", 5.0)])
    con = sqlite3.connect(a)
    con.executemany("insert into counters_collection values (?, ?, ?)",
                    [(tile, "SQ_INSTS_VALU", 7000.0), (tile, "SQ_INSTS_VALU", 7000.0)])
    con.commit()
    con.close()
    _counter_db(b, "SQ_ACTIVE_INST_VALU", [(tile, 200.0), (tile, 200.0)])
    out = tmp_path / "c.txt"
    profsum.counters([str(a), str(b)], "k_tile_pipe", 640, str(out), ["cmd1", "cmd2"])
    txt = out.read_text()
    # 7000 VALU instructions over 640 elements = 10 wave steps: 700 per step
    assert "VALU instructions per wave step of 64 elements: 700" in txt
    assert "issuing VALU instructions: 20.0 %" in txt
    assert "(mean of 2 of 3 launches)" in txt
