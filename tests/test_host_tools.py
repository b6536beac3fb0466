"""Host-side logic on the CPU: workload shapes, the bench contract's
multi-GPU refusal, and the counter-summary arithmetic."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import scenarios

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_workload_shapes():
    c1 = scenarios.c1()
    assert c1.cells == 65536 and c1.steps == 1000 and c1.dt == 1.0
    c2 = scenarios.c2()
    assert [(lv["nx"], lv["ny"]) for lv in c2.levels] == [(1200, 1000), (900, 900), (1500, 1500), (2400, 2400)]
    assert c2.cells == 10_020_000 and c2.steps == 18000 and c2.dt == 0.2
    assert [c2.level_dx(k) for k in range(4)] == [810.0, 270.0, 90.0, 30.0]
    land = [float((lv["h"] <= 0).mean()) for lv in c2.levels]
    assert 0.3 < land[3] < 0.7 and max(lv["h"].max() for lv in c2.levels[3:]) < 1146.0


@pytest.mark.slow
def test_c3_matches_table1_shapes():
    c3 = scenarios.c3()
    assert c3.levels[0]["nx"] * c3.levels[0]["ny"] == 2_012_940          # Table 1, level 1
    assert c3.cells == 47_218_698 and c3.steps == 108_000
    assert [c3.level_dx(k) for k in range(5)] == [810.0, 270.0, 90.0, 30.0, 10.0]
    for lv in c3.levels[2:]:
        assert 0.35 < float((lv["h"] <= 0).mean()) < 0.45
    assert c3.levels[4]["h"].max() <= 100.0


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_summary(tmp_path):
    sys.path.insert(0, ROOT)
    from bench import COPY_PROBE_BYTES, source_hash
    kib = COPY_PROBE_BYTES / 1024

    def write(path, counter, copy_factor, fused_kib):
        with open(path, "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for d in range(3):
                f.write(f'{d},"void (anonymous namespace)::k_stream_copy(double const*, double*, long)",'
                        f'{counter},{kib * copy_factor}\n')
            for d in range(3, 7):
                f.write(f"{d},\"(anonymous namespace)::k_fused(DomainDev, int)\",{counter},{fused_kib}\n")
    write(tmp_path / "f.csv", "FETCH_SIZE", 1.25, 1000.0)
    write(tmp_path / "w.csv", "WRITE_SIZE", 0.5, 300.0)
    out = tmp_path / "traffic.json"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench_traffic.py"), str(tmp_path / "f.csv"),
                        str(tmp_path / "w.csv"), "--cells", "1000", "--workload", "w", "--out", str(out)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    e = json.loads(out.read_text())["k_fused"]
    assert e["copy_factor_fetch"] == pytest.approx(1.25) and e["copy_factor_write"] == pytest.approx(0.5)
    assert e["bytes_per_cell"] == pytest.approx((1000 * 1024 / 1.25 + 300 * 1024 / 0.5) / 1000)
    assert e["source_hash"] == source_hash()
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench_traffic.py"), str(tmp_path / "f.csv"),
                        str(tmp_path / "w.csv"), "--cells", "1000", "--workload", "w", "--tile-rows", "12",
                        "--out", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    t = json.loads(out.read_text())
    assert set(t) == {"k_fused", "k_fused@12"} and t["k_fused@12"]["tile_rows"] == 12


def test_step_times_from_a_trace(tmp_path):
    """bench_steps.py groups dispatches into steps at each k_active, starts the
    run after the reset gap and averages each kernel over a window."""
    import sqlite3
    sys.path.insert(0, ROOT)
    import bench_steps
    db = tmp_path / "run_results.db"
    c = sqlite3.connect(db)
    c.execute("create table kernels (name text, start integer, duration integer)")
    t = 0
    rows = []
    for s in range(400):
        if s == 40:
            t += 10_000_000                      # the reset to t = 0 before the timed run
        small = 40 <= s < 140
        for name, dur in (("k_active<double>", 5000), ("k_fused_loop<double>" if small else "k_fused<double>", 7000),
                          ("k_fused_split<double>", 3000)):
            rows.append((f"(anonymous namespace)::{name}(DomainDev, int)", t, dur))
            t += dur
        t += 1000
    rows.insert(0, ("__amd_rocclr_copyBuffer", 0, 100))
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    c.commit()
    steps = bench_steps.steps_of(str(db))
    assert len(steps) == 360
    av, tot, period, nsmall = bench_steps.window(steps, 0, 200)
    assert av["active"] == pytest.approx(5.0) and av["split"] == pytest.approx(3.0)
    assert av["loop"] == pytest.approx(3.5) and av["fused"] == pytest.approx(3.5) and nsmall == 100
    assert tot == pytest.approx(15.0) and period == pytest.approx(16.0)
