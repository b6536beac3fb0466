#!/usr/bin/env python
"""Throughput of the nested long-wave time step on one MI355X.

One bench step = one time step of the whole nested domain (mass, child->parent
level, momentum, parent->child flux, open sides, maxima on every level).
Default workload: the 4-level nest at 810/270/90/30 m (1200x1000, 900^2,
1500^2, 2400^2 = 10.02 M cells) over a seeded synthetic coast, dt = 0.2 s,
3 m elliptic uplift, run for the whole 3600 s (18,000 steps) from t = 0,
inputs resident in HBM.  Prints one JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell for each kernel kind, FP64 (read + write of the
# arrays the kernel must touch once per cell; stencil neighbours not counted).
BYTES_PER_CELL = {
    "k_mass": 8 * (4 + 1),          # eta, M, N, h in; eta out
    "k_momentum": 8 * (5 + 3),      # eta, h, M, N, max in; M, N, max out
    "k_fused": 8 * (4 + 3 + 2),     # eta, M, N, h in; eta, M, N out; max in+out
}
# FP32-bulk: eta in and out FP64 (16 B); M, N, h in and M, N out FP32 (20 B); max in+out FP32 (8 B)
BYTES_PER_CELL_FP32_BULK = {"k_fused": 16 + 20 + 8}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for p in ("paper_2408_07609_amd/csrc/rti_kernels.hip", "paper_2408_07609_amd/csrc/rti_fused.hip",
              "paper_2408_07609_amd/csrc/rti_device.h", "paper_2408_07609_amd/csrc/rti_internal.h"):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, cells_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json, written by bench_traffic.py): the measured bytes
    per computed cell of this kernel on this workload, times the cells one
    launch computes here.  None when the counters were taken on another
    kernel source or workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel)
    if not e or e.get("source_hash") != source_hash() or e.get("workload") != workload:
        return None
    return e["bytes_per_cell"] * cells_per_launch


COPY_PROBE_BYTES = 1 << 30


def copy_probe():
    """A plain 1 GiB device-to-device copy by torch's copy kernel: rocprofv3's
    FETCH_SIZE / WRITE_SIZE readings of it give the factor between the
    counters and real bytes."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 copies of {COPY_PROBE_BYTES} bytes")


def cpu_baseline(sc, seconds):
    import oracle
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    t0 = time.perf_counter()
    o.step(1)
    done = 1
    el = time.perf_counter() - t0
    per = el
    while el + per < seconds:
        o.step(1)
        done += 1
        el = time.perf_counter() - t0
        per = el / done
    return dict(value=sc.cells * done / el, unit="cell-updates/s", cores=oracle.threads(), kind="oracle",
                sample=f"{sc.name}: all {sc.cells} cells, steps 1..{done} from t=0 ({el:.1f} s of CPU work)")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the whole configuration)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--flags", type=int, default=0, help="RTI_FLAG_* bits for the domain")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32-bulk"])
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenarios
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64, Domain

    sc = {"c1": scenarios.c1, "c2": scenarios.c2, "c3": scenarios.c3}[args.config]()
    steps = args.steps if args.steps is not None else sc.steps
    log(f"workload {sc.name}: {len(sc.levels)} levels, {sc.cells} cells, {steps} timed steps")
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, flags=args.flags, device="cuda:0",
               precision=RTI_FP32_BULK if args.precision == "fp32-bulk" else RTI_FP64)
    bpc = BYTES_PER_CELL_FP32_BULK if args.precision == "fp32-bulk" else BYTES_PER_CELL
    d.set_source(*sc.source.astuple())
    init = [d.get_state(k) for k in range(len(sc.levels))]
    zinit = [d.max_inundation(k) for k in range(len(sc.levels))]
    d.step(args.warmup)
    d.sync()
    # back to t = 0: the timed run is the configuration itself
    for k, (e, M, N) in enumerate(init):
        d.set_state(k, e, M, N)
        d.set_max(k, zinit[k])
    log("warmup done")

    stream = d.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    d.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    log(f"timed {steps} steps: {wall:.3f} s wall, {ev_ms / 1e3:.3f} s by events")
    e_last = d.get_state(len(sc.levels) - 1)[0]
    assert np.all(np.isfinite(e_last)), "non-finite state after the timed run"
    active, total, active_cells = d.active_tiles()

    prof, prof_cells = d.profile(args.profile_steps)
    dom = max((k for k in prof if k in bpc), key=lambda k: prof[k])
    launch_ms = prof[dom]
    # algorithmic bytes of one launch: the per-cell figure times the cells the
    # launch computes (skipped quiescent tiles move no data)
    units = prof_cells if dom == "k_fused" else sc.cells
    alg = bpc[dom] * units
    achieved = alg / (launch_ms * 1e-3) / 1e9
    log(f"kernel times (ms/launch): {prof}; cells per launch {units:.0f}")
    if args.copy_probe:
        copy_probe()

    value = sc.cells * steps / wall
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-bulk (f64 water level)",
        "data": "synthetic",
        "config": {
            "workload": sc.name,
            "cells": sc.cells,
            "levels": [[lv["nx"], lv["ny"]] for lv in sc.levels],
            "dx_m": [sc.level_dx(k) for k in range(len(sc.levels))],
            "dt_s": sc.dt,
            "simulated_s": steps * sc.dt,
            "active_tiles": [active, total],
            "active_cells_last_step": active_cells,
            "flags": args.flags,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom + ("" if args.precision == "fp64" else "_fp32bulk"), sc.name, units),
            "bytes_per_cell": bpc[dom],
            "cells_per_launch": units,
            "launch_ms": launch_ms,
            "kernel_ms": prof,
        },
    }
    d.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
