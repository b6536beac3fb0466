#!/usr/bin/env python
"""Throughput of the nested long-wave time step on one MI355X.

One bench step = one time step of the whole nested domain (mass, child->parent
level, momentum, parent->child flux, open sides, maxima on every level), FP64.
Default workload: configuration 3, the 5-level nest at 810/270/90/30/10 m
(1266x1590, 1305^2, 1494^2, 3141^2, 5604^2 = 47.2 M cells, the shapes of the
paper's Table 1) over a seeded synthetic coast with 40 % dry coastal plains,
dt = 0.2 s, 3 m elliptic uplift, inputs resident in HBM.

Timed window: with no --steps, the whole configuration (108,000 steps = 6 h
simulated) from t = 0 with stationary tiles skipped ("full_run"); with
--steps K shorter than that, K steps with every tile computed ("dense": no
counted cell is skipped), after --warmup steps.  Graph capture and the first
steps' set-up always happen before the timed window.  In the dense case the
whole 6-hour run is measured too, in the same process, and reported as
"full_run".  Prints one JSON line on stdout; progress on stderr.
--config c1/c2: the smaller configurations; c3b: C3 split into the 84 blocks
of the paper's Table 1, each in its own parent block; c3t: the same block
counts as touching rectangles, one masked level per resolution; c4: the batched ensemble (48 uneven scenarios,
FP32-bulk, one batch); c5: forecast serving (Poisson arrivals, continuous
batching, p50/p99 time to forecast).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
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


def measured_traffic(kernel, workload, cells_per_launch, tile_rows=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json, written by bench_traffic.py): the measured bytes
    per computed cell of this kernel on this workload, times the cells one
    launch computes here.  None when the counters were taken on another
    kernel source, workload or tile height."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    # One entry per kernel and tile height ("k_fused@12"); the plain kernel
    # name holds the entry of one height, stated in its tile_rows.
    keys = ([f"{kernel}@{tile_rows}"] if tile_rows is not None else []) + [kernel]
    for e in (t.get(k) for k in keys):
        if not e or e.get("source_hash") != source_hash() or e.get("workload") != workload:
            continue
        if tile_rows is not None and e.get("tile_rows") not in (None, tile_rows):
            continue
        return e["bytes_per_cell"] * cells_per_launch
    return None


COPY_PROBE_BYTES = 1 << 30
MIX_PROBE_DOUBLES = 1 << 26      # 512 MiB per array


def copy_probe():
    """Project-written streams (rti_stream_probe), timed with HIP events on
    torch's stream: a plain 1 GiB copy (k_stream_copy; rocprofv3's FETCH_SIZE
    and WRITE_SIZE readings of it give the factor between the counters and
    real bytes), and the FP64 step's mix of 5 reads and 4 writes per element
    (k_stream_probe), the practical HBM ceiling for the step's kernels."""
    import torch
    from paper_2408_07609_amd import rti
    out = {}
    src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    ins = [torch.full((MIX_PROBE_DOUBLES,), float(k + 1), dtype=torch.float64, device="cuda:0") for k in range(5)]
    outs = [torch.empty(MIX_PROBE_DOUBLES, dtype=torch.float64, device="cuda:0") for _ in range(4)]
    for name, fn, nbytes in (("copy", lambda: rti.stream_probe([src], [dst]), 2 * COPY_PROBE_BYTES),
                             ("mix_5r4w", lambda: rti.stream_probe(ins, outs), 9 * 8 * MIX_PROBE_DOUBLES)):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(3):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        s = ev0.elapsed_time(ev1) / 3e3
        out[name] = {"bytes": nbytes, "ms": s * 1e3, "GB_per_s": nbytes / s / 1e9,
                     "frac_of_peak": nbytes / s / 1e9 / HBM_PEAK_GBS}
    log(f"stream probes: {out}")
    del src, dst, ins, outs
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(sc, seconds):
    """The oracle (as it stands) stepping the configuration from t = 0 for
    about `seconds` of CPU work; returns (cell-updates/s, steps, seconds, threads)."""
    import oracle
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    t0 = time.perf_counter()
    o.step(1)
    done = 1
    el = time.perf_counter() - t0
    while el + el / done < seconds:
        o.step(1)
        done += 1
        el = time.perf_counter() - t0
    return sc.cells * done / el, done, el, oracle.threads()


SCENARIOS = ("c1", "c2", "c3", "c3b", "c3t")


def scenario(name):
    import scenarios
    return {"c1": scenarios.c1, "c2": scenarios.c2, "c3": scenarios.c3, "c3b": scenarios.c3_blocks,
            "c3t": scenarios.c3_touching}[name]()


def cpu_baseline(sc, seconds, config=None):
    """The oracle on the host's cores (OpenMP over rows, all cores), and, when
    the configuration is named, the same on one thread in a child process."""
    v, done, el, threads = _oracle_rate(sc, seconds)
    out = dict(value=v, unit="cell-updates/s", cores=threads, kind="oracle",
               sample=f"{sc.name}: all {sc.cells} cells, steps 1..{done} from t=0 ({el:.1f} s of CPU work)",
               cpu_model=cpu_model(), nproc=os.cpu_count())
    if config is not None:
        import subprocess
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", config,
                            "--cpu-seconds", str(seconds)], env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0 and r.stdout.strip():
            out["one_thread"] = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            out["one_thread"] = {"error": (r.stderr or "")[-300:]}
    return out


def cpu_child(config, seconds):
    """Child process of cpu_baseline (OMP_NUM_THREADS=1): no GPU is touched."""
    sc = scenario(config)
    v, done, el, threads = _oracle_rate(sc, seconds)
    print(json.dumps(dict(value=v, unit="cell-updates/s", cores=threads,
                          sample=f"{sc.name}: all {sc.cells} cells, steps 1..{done} from t=0 ({el:.1f} s)")))


def make_domain(sc, precision, flags=0):
    from paper_2408_07609_amd import Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, flags=flags, device="cuda:0", precision=precision)
    d.set_source(*sc.source.astuple())
    return d


def bench_batch(args):
    """The batched ensemble (C4): 48 uneven scenarios stepped as one batch
    (one active-list launch and one fused launch per step over all members'
    tiles, HIP graphs), tile heights autotuned per member."""
    import collections

    import numpy as np
    import torch

    import scenarios
    from paper_2408_07609_amd import (RTI_FLAG_NO_ACTIVE, RTI_FLAG_NO_GRAPH, RTI_FLAG_PERSISTENT, RTI_FP32_BULK, RTI_FP64,
                                      Batch, autotune_batch_rows)

    prec = RTI_FP32_BULK if args.precision == "fp32-bulk" else RTI_FP64
    scs = scenarios.c4()
    cells = sum(sc.cells for sc in scs)
    steps = args.steps if args.steps is not None else 2000
    log(f"c4: {len(scs)} members, {cells} cells, {steps} timed steps, {args.precision}")

    # the members get the same skipping and graph choices as the batch, for the one-after-another comparison
    member_flags = args.flags & (RTI_FLAG_NO_ACTIVE | RTI_FLAG_NO_GRAPH)

    def build(precision, tune):
        ds = [make_domain(sc, precision, member_flags) for sc in scs]
        rows = []
        if tune and args.tile_rows:
            for d in ds:
                d.set_tile_rows(args.tile_rows)
                rows.append(args.tile_rows)
        elif tune:
            # one height for the whole batch, tuned on throwaway copies of the members
            copies = [make_domain(sc, precision, member_flags) for sc in scs]
            best, ms = autotune_batch_rows(copies, 8)
            for c in copies:
                c.close()
            del copies
            log(f"batch autotuner: {best} rows ({ms:.3f} ms per step, every tile computed)")
            for d in ds:
                d.set_tile_rows(best)
                rows.append(best)
        return ds, rows

    ds, rows = build(prec, True)
    log(f"tile rows: {dict(collections.Counter(rows))}")
    batch = Batch(ds, flags=(RTI_FLAG_PERSISTENT if args.persistent else 0)
                  | (args.flags & (RTI_FLAG_NO_ACTIVE | RTI_FLAG_NO_GRAPH)))
    batch.step(args.warmup)
    batch.sync()
    stream = batch.stream
    all0, comp0 = batch.cell_updates()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    all1, comp1 = batch.cell_updates()
    assert all1 - all0 == cells * steps
    log(f"timed {steps} batch steps: {wall:.3f} s")
    fused_ms, active_ms, prof_cells = batch.profile(args.profile_steps)
    bpc = BYTES_PER_CELL_FP32_BULK["k_fused"] if prec == RTI_FP32_BULK else BYTES_PER_CELL["k_fused"]
    achieved = bpc * prof_cells / (fused_ms * 1e-3) / 1e9
    finest = [d.get_state(len(d.levels) - 1)[0] for d in ds]
    assert all(np.all(np.isfinite(e)) for e in finest), "non-finite state after the timed run"
    done = ds[0].steps
    batch.close()

    # the same members one after another (each replays its own graphs)
    seq_steps = max(20, min(steps, 400) // 20 * 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in ds:
        d.step(seq_steps)
    torch.cuda.synchronize()
    seq = cells * seq_steps / (time.perf_counter() - t0)
    log(f"members one after another: {seq:.4g} cell-updates/s ({seq_steps} steps each)")

    out = {
        "metric": "cell-updates/s",
        "value": cells * steps / wall,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == RTI_FP64 else "f32-bulk (f64 water level)",
        "data": "synthetic",
        "config": {
            "workload": "c4-ensemble48",
            "members": len(scs),
            "cells": cells,
            "member_cells": [sc.cells for sc in scs],
            "tile_rows": rows,
            "persistent": bool(args.persistent),
            "timed_steps_from": args.warmup,
            "computed_cell_updates": comp1 - comp0,
            "active_cell_updates_per_s": (comp1 - comp0) / wall,
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_fused_batch", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_cell": bpc, "cells_per_launch": prof_cells,
            "launch_ms": fused_ms, "kernel_ms": {"k_fused_batch": fused_ms, "k_active_batch": active_ms},
        },
        "one_after_another": {"value": seq, "unit": "cell-updates/s", "steps_each": seq_steps},
    }
    for d in ds:
        d.close()
    del ds, finest

    if prec == RTI_FP32_BULK and not args.no_fp64:
        # The same ensemble in FP64: the FP32-bulk error after compare_steps
        # steps from t = 0 (max and RMS |d eta| over all cells, max |d maxima|),
        # then the FP64 rate over the same number of timed steps.
        log(f"fp64 comparison: {args.compare_steps} steps of both precisions")
        d32, _ = build(RTI_FP32_BULK, False)
        d64, _ = build(RTI_FP64, False)
        for group in (d32, d64):
            with Batch(group) as b:
                b.step(args.compare_steps)
                b.sync()
        emax = zerr = 0.0
        esq = 0.0
        ncell = 0
        for a32, a64 in zip(d32, d64):
            for k in range(len(a32.levels)):
                e32, e64 = a32.get_state(k)[0], a64.get_state(k)[0]
                de = np.abs(e32 - e64)
                emax = max(emax, float(de.max()))
                esq += float(np.sum(de * de))
                ncell += de.size
                zerr = max(zerr, float(np.abs(a32.max_inundation(k) - a64.max_inundation(k)).max()))
            a32.close()
        b64 = Batch(d64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b64.step(steps)
        torch.cuda.synchronize()
        v64 = cells * steps / (time.perf_counter() - t0)
        b64.close()
        for d in d64:
            d.close()
        out["fp64"] = {"value": v64, "unit": "cell-updates/s", "steps": steps}
        out["fp32_bulk_error_vs_fp64"] = {"after_steps": args.compare_steps, "eta_max_m": emax,
                                          "eta_rms_m": math.sqrt(esq / max(1, ncell)), "maxima_max_m": zerr}
        log(f"fp64 {v64:.4g} cell-updates/s; fp32-bulk error {out['fp32_bulk_error_vs_fp64']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        small = min(scs, key=lambda sc: sc.cells if len(sc.levels) == 3 else 1 << 60)
        out["cpu_baseline"] = cpu_baseline(small, args.cpu_seconds)
        out["cpu_baseline"]["sample"] += " (the smallest nested member of c4)"
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Forecast serving (C5): Poisson arrivals (2 per minute) of requests on
    six nested sites of 1 M to 47 M cells, 1-6 h forecasts, admitted by
    device footprint into one running batch (continuous batching); with
    --time-scale s the clock and the durations are both divided by s (1, the
    default, is the stated configuration).  Runs the same request stream in
    FP32-bulk and in FP64 (unless --precision picks one) and reports p50/p99
    time to forecast, concurrency, and the cost model's predictions."""
    import torch

    import scenarios
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64
    import numpy as np

    from paper_2408_07609_amd.serve import ForecastServer, Request, fit_cost_model, percentiles, predict

    sites = scenarios.c5_sites()
    stream = scenarios.c5_requests(sites, count=args.requests, time_scale=args.time_scale)
    reqs = [Request(i, sites[k], src, steps, t) for i, (k, src, steps, t) in enumerate(stream)]
    free, total = torch.cuda.mem_get_info()
    budget = int(min(free * 0.8, args.hbm_gib * 2**30)) if args.hbm_gib else int(free * 0.8)
    log(f"c5: {len(reqs)} requests over {reqs[-1].arrival:.1f} s, sites {[sc.cells for sc in sites]}, "
        f"budget {budget / 2**30:.1f} GiB")
    runs = {}
    precs = {"fp32-bulk": RTI_FP32_BULK, "fp64": RTI_FP64}
    order = [args.precision] if "--precision" in sys.argv else ["fp32-bulk", "fp64"]
    for name in order:
        srv = ForecastServer(budget, precs[name], chunk_steps=args.chunk)
        res = srv.run(reqs, log=log)
        srv.close()
        q = percentiles(res)
        # the cost model: step time = a * computed cells + b, fitted on the run's chunks; then the
        # whole stream replayed through the server's policy with that model
        a, b = fit_cost_model(srv.chunks)
        frac = sum(c[3] for c in srv.chunks) / max(1, sum(c[0] * c[2] for c in srv.chunks))
        pred = predict(reqs, a, b, frac, budget, precs[name], args.chunk)
        rel = [abs(pred[r.rid] - r.time_to_forecast) / r.time_to_forecast for r in res]
        qp = np.percentile([pred[r.rid] for r in res], [50, 99])
        runs[name] = {"p50_time_to_forecast_s": q["p50"], "p99_time_to_forecast_s": q["p99"],
                      "cell_updates_per_s": srv.cell_updates / srv.makespan, "makespan_s": srv.makespan,
                      "cell_updates": srv.cell_updates, "peak_concurrent": srv.peak_members,
                      "mean_concurrent": float(sum(r.time_to_forecast for r in res) / srv.makespan),
                      "peak_gib": srv.peak_bytes / 2**30, "computed_fraction": frac,
                      "cost_model": {"a_s_per_computed_cell": a, "b_s_per_step": b,
                                     "predicted_p50_s": float(qp[0]), "predicted_p99_s": float(qp[1]),
                                     "median_rel_error": float(np.median(rel)), "max_rel_error": float(max(rel))},
                      "requests": [{"rid": r.rid, "cells": r.cells, "steps": r.steps, "arrival_s": r.arrival,
                                    "time_to_forecast_s": r.time_to_forecast, "predicted_s": pred[r.rid]}
                                   for r in sorted(res, key=lambda r: r.rid)]}
        log(f"{name}: " + json.dumps({k: v for k, v in runs[name].items() if k != "requests"}))
    first = runs[order[0]]
    out = {
        "metric": "cell-updates/s",
        "value": first["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": int(sum(r.steps for r in reqs)),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-bulk (f64 water level)" if order[0] == "fp32-bulk" else "f64",
        "data": "synthetic",
        "config": {"workload": "c5-serving", "requests": len(reqs), "sites_cells": [sc.cells for sc in sites],
                   "arrival_rate_per_min": 2.0, "time_scale": args.time_scale, "chunk_steps": args.chunk,
                   "hbm_budget_gib": budget / 2**30},
        "serving": runs,
    }
    print(json.dumps(out), flush=True)


GRAPH_STEPS = 20      # steps per captured HIP graph in the library


def timed_steps(d, steps, torch):
    """Time `steps` steps of domain d on its stream: wall clock around the
    enqueue and a synchronisation, and HIP events recorded on d's stream."""
    stream = d.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    all0, comp0 = d.cell_updates()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    d.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    all1, comp1 = d.cell_updates()
    return wall, ev0.elapsed_time(ev1) / 1e3, all1 - all0, comp1 - comp0


def tile_rows(d, args):
    """The tile height: --tile-rows if given, else the library's autotuner
    (every candidate height timed from the current state with every tile
    computed; the state is restored exactly)."""
    if args.tile_rows:
        d.set_tile_rows(args.tile_rows)
        return args.tile_rows
    rows, ms = d.autotune(8)
    log(f"autotuned tile rows: {rows} ({ms:.4f} ms per step, every tile computed)")
    return rows


def full_run(sc, prec, flags, torch, np, args):
    """The whole configuration from t = 0 with stationary tiles skipped: the
    graph is captured by untimed steps first, then the state goes back to
    t = 0 (which, like a new domain, computes every tile in the first two
    steps) and all sc.steps steps are timed."""
    d = make_domain(sc, prec, flags)
    rows = tile_rows(d, args)
    init = [d.get_state(k) for k in range(len(sc.levels))]
    zinit = [d.max_inundation(k) for k in range(len(sc.levels))]
    d.step(2 * GRAPH_STEPS)
    d.sync()
    for k, (e, M, N) in enumerate(init):
        d.set_state(k, e, M, N)
        d.set_max(k, zinit[k])
    d.sync()
    log(f"full run: {sc.steps} steps ({sc.steps * sc.dt:.0f} s simulated)")
    wall, ev_s, all_, comp = timed_steps(d, sc.steps, torch)
    assert all_ == sc.cells * sc.steps
    for k in range(len(sc.levels)):
        assert np.all(np.isfinite(d.get_state(k)[0])), "non-finite state after the full run"
    log(f"full run: {wall:.2f} s wall, {ev_s:.2f} s by events, computed fraction {comp / all_:.3f}")
    return d, dict(steps=sc.steps, simulated_s=sc.steps * sc.dt, tile_rows=rows, wall_s=wall, events_s=ev_s,
                   value=sc.cells * sc.steps / wall, unit="cell-updates/s", computed_cell_updates=comp,
                   computed_fraction=comp / all_, active_cell_updates_per_s=comp / wall)


def bench_single(args):
    import numpy as np
    import torch

    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FP32_BULK, RTI_FP64

    sc = scenario(args.config)
    prec = RTI_FP32_BULK if args.precision == "fp32-bulk" else RTI_FP64
    bpc = BYTES_PER_CELL_FP32_BULK if prec == RTI_FP32_BULK else BYTES_PER_CELL
    dense = args.steps is not None and args.steps < sc.steps
    steps = args.steps if dense else sc.steps
    log(f"workload {sc.name}: {len(sc.levels)} levels, {sc.cells} cells, "
        f"{'dense window of ' + str(steps) if dense else 'full run of ' + str(steps)} steps, {args.precision}")

    full = None
    if dense:
        # every tile computed; warmup (at least one graph's worth, rounded up
        # to whole graphs so the timed window starts on a captured graph)
        d = make_domain(sc, prec, args.flags | RTI_FLAG_NO_ACTIVE)
        rows = tile_rows(d, args)
        prep = max(args.warmup, GRAPH_STEPS)
        prep = (prep + GRAPH_STEPS - 1) // GRAPH_STEPS * GRAPH_STEPS
        d.step(prep)
        d.sync()
        log(f"warmup: {prep} untimed steps (graph captured)")
        wall, ev_s, all_, comp = timed_steps(d, steps, torch)
        assert all_ == comp == sc.cells * steps, "the dense window skipped cells"
        window = "dense"
        untimed = prep
    else:
        d, full = full_run(sc, prec, args.flags, torch, np, args)
        rows = full["tile_rows"]
        wall, ev_s, all_, comp = full["wall_s"], full["events_s"], sc.cells * steps, full["computed_cell_updates"]
        window = "full_run"
        untimed = 2 * GRAPH_STEPS
    log(f"timed {steps} steps: {wall:.3f} s wall, {ev_s:.3f} s by events")
    active, total, active_cells = d.active_tiles()

    # kernel durations with HIP events on the domain's stream, launched one by one
    prof, prof_cells = d.profile(args.profile_steps)
    dom = max((k for k in prof if k in bpc), key=lambda k: prof[k])
    launch_ms = prof[dom]
    units = prof_cells if dom == "k_fused" else sc.cells
    alg = bpc[dom] * units
    achieved = alg / (launch_ms * 1e-3) / 1e9
    log(f"kernel times (ms/launch): {prof}; cells per launch {units:.0f}")
    d.close()
    del d
    probes = copy_probe() if args.copy_probe else None
    if dense and not args.no_full_run:
        dfull, full = full_run(sc, prec, args.flags, torch, np, args)
        fprof, fcells = dfull.profile(args.profile_steps)
        full["kernel_ms_at_end"] = fprof
        full["cells_per_launch_at_end"] = fcells
        dfull.close()
        del dfull

    out = {
        "metric": "cell-updates/s",
        "value": sc.cells * steps / wall,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == RTI_FP64 else "f32-bulk (f64 water level)",
        "data": "synthetic",
        "config": {
            "workload": sc.name,
            "timed_window": window,
            "untimed_steps_before_window": untimed,
            "cells": sc.cells,
            "levels": [[lv["nx"], lv["ny"]] for lv in sc.levels],
            "dx_m": [sc.level_dx(k) for k in range(len(sc.levels))],
            "dt_s": sc.dt,
            "simulated_s": steps * sc.dt,
            "active_tiles_last_step": [active, total],
            "active_cells_last_step": active_cells,
            "computed_cell_updates": comp,
            "active_cell_updates_per_s": comp / wall,
            "flags": args.flags | (RTI_FLAG_NO_ACTIVE if dense else 0),
            "tile_rows": rows,
            "tile_rows_from": "--tile-rows" if args.tile_rows else "autotuner",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom + ("" if prec == RTI_FP64 else "_fp32bulk"), sc.name, units, rows)
            if dense else None,
            "bytes_per_cell": bpc[dom],
            "cells_per_launch": units,
            "launch_ms": launch_ms,
            "kernel_ms": prof,
        },
    }
    if full is not None and dense:
        out["full_run"] = full
    if probes is not None:
        out["stream_probes"] = probes
    if prec == RTI_FP32_BULK and not args.no_fp64:
        out["fp32_bulk_error_vs_fp64"] = fp32_error(sc, args.flags, steps if dense else sc.steps, np)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds, config=args.config)
    print(json.dumps(out), flush=True)


def fp32_error(sc, flags, steps, np):
    """FP32-bulk against FP64 on the same GPU after `steps` steps from the
    same source: max and RMS |d eta| over every cell of every level, max
    |d maxima|, and the inundated land cells (maxima above 1 cm) of each."""
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64
    a, b = make_domain(sc, RTI_FP32_BULK, flags), make_domain(sc, RTI_FP64, flags)
    a.step(steps)
    b.step(steps)
    emax = zmax = esq = 0.0
    n = 0
    inund = [0, 0]
    for k, lv in enumerate(sc.levels):
        de = np.abs(a.get_state(k)[0] - b.get_state(k)[0])
        za, zb = a.max_inundation(k), b.max_inundation(k)
        emax = max(emax, float(de.max()))
        esq += float(np.sum(de * de))
        n += de.size
        zmax = max(zmax, float(np.abs(za - zb).max()))
        land = lv["h"] <= 0
        inund[0] += int(np.count_nonzero(land & (za > 0.01)))
        inund[1] += int(np.count_nonzero(land & (zb > 0.01)))
    a.close()
    b.close()
    out = {"after_steps": steps, "eta_max_m": emax, "eta_rms_m": math.sqrt(esq / max(1, n)), "maxima_max_m": zmax,
           "inundated_cells_fp32_bulk": inund[0], "inundated_cells_fp64": inund[1]}
    log(f"fp32-bulk error vs fp64: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the whole configuration)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c3b", "c3t", "c4", "c5"])
    ap.add_argument("--flags", type=int, default=0, help="RTI_FLAG_* bits for the domain")
    ap.add_argument("--tile-rows", type=int, default=0, help="tile height of the fused kernel (0: the library's default)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32-bulk"])
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run the stream probes (1 GiB copy for counter calibration, 5-read/4-write ceiling)")
    ap.add_argument("--persistent", action="store_true", help="c4: persistent grid for the batched kernel")
    ap.add_argument("--no-fp64", action="store_true", help="c4: skip the FP64 comparison run")
    ap.add_argument("--compare-steps", type=int, default=600, help="c4: steps before the FP32-bulk error is taken")
    ap.add_argument("--requests", type=int, default=24, help="c5: forecast requests")
    ap.add_argument("--time-scale", type=float, default=1.0,
                    help="c5: compression of arrivals and durations (1: the stated 2 requests/min and 1-6 h)")
    ap.add_argument("--chunk", type=int, default=200, help="c5: batch steps between admission points")
    ap.add_argument("--hbm-gib", type=float, default=0.0, help="c5: HBM budget (default 80%% of free memory)")
    ap.add_argument("--no-full-run", action="store_true", help="dense window only: skip the whole-run measurement")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.cpu_child:
        return cpu_child(args.cpu_child, args.cpu_seconds)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library drives one GPU)",
              file=sys.stderr)
        sys.exit(2)

    if args.config == "c5":
        return bench_serve(args)
    if args.config == "c4":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "fp32-bulk"          # the ensemble runs in FP32-bulk unless asked otherwise
        return bench_batch(args)

    return bench_single(args)


if __name__ == "__main__":
    main()
