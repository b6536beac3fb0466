#!/usr/bin/env python
"""Turn two rocprofv3 counter runs of bench.py into profiles/traffic.json.

Each run is `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) with csv output of
`bench.py --steps K ... --copy-probe --flags 1` (dense window: every launch
computes every cell; no graph).  FETCH_SIZE and WRITE_SIZE are in KiB per
dispatch.  The project's 1 GiB copy kernel (k_stream_copy) in the same run
calibrates each counter (reading / true bytes); the fused kernel's per-dispatch readings divided by
that factor and by the cells of the workload give its HBM bytes per computed
cell, stored with the kernel source hash so bench.py can tell when they are
stale.

    python bench_traffic.py FETCH_CSV WRITE_CSV --cells N --workload NAME [--tile-rows R] [--key k_fused_fp32bulk]
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
from bench import COPY_PROBE_BYTES, source_hash  # noqa: E402


def per_kernel(path, counter):
    vals = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"]
            vals.setdefault(name, []).append(float(row["Counter_Value"]))
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--cells", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernel", default="k_fused", help="substring of the kernel name")
    ap.add_argument("--key", default=None,
                    help="entry name in the json (default: --kernel, or --kernel@ROWS with --tile-rows)")
    ap.add_argument("--tile-rows", type=int, default=None, help="tile height of the counted runs")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    out = {}
    factors = {}
    per = {}
    for which, path, counter in (("fetch", args.fetch_csv, "FETCH_SIZE"), ("write", args.write_csv, "WRITE_SIZE")):
        vals = per_kernel(path, counter)
        copy = [v for k, vs in vals.items() if "k_stream_copy" in k for v in vs]
        big = [v for v in copy if v * 1024 > 0.1 * COPY_PROBE_BYTES]
        if not big:
            sys.exit(f"no copy-probe dispatch in {path}")
        factors[which] = (sum(big) / len(big)) * 1024 / COPY_PROBE_BYTES
        ker = [v for k, vs in vals.items() if args.kernel in k for v in vs]
        if not ker:
            sys.exit(f"no {args.kernel} dispatch in {path}")
        per[which] = (sum(ker) / len(ker)) * 1024 / factors[which]
    key = args.key or (f"{args.kernel}@{args.tile_rows}" if args.tile_rows else args.kernel)
    out[key] = {
        "bytes_per_cell": (per["fetch"] + per["write"]) / args.cells,
        "fetch_bytes_per_launch": per["fetch"],
        "write_bytes_per_launch": per["write"],
        "copy_factor_fetch": factors["fetch"],
        "copy_factor_write": factors["write"],
        "cells": args.cells,
        "workload": args.workload,
        "tile_rows": args.tile_rows,
        "source_hash": source_hash(),
    }
    path = args.out
    old = {}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
    old.update(out)
    with open(path, "w") as f:
        json.dump(old, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
