#!/usr/bin/env python
"""The per-step floor: a domain at rest (lake at rest, no source), so every
tile is stationary after two steps and nothing is computed; the time per
graph-replayed step is then the launches alone.

    python bench_floor.py [--configs c2 c3] [--persistent]

Prints one JSON line per domain: k_fused and k_active by HIP events (launches
one by one, rti_profile) and the wall time per step of 400 graph-replayed
steps around a synchronisation.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", nargs="+", default=["c2", "c3"])
    ap.add_argument("--persistent", action="store_true", help="also each domain with RTI_FLAG_PERSISTENT")
    ap.add_argument("--tile-rows", type=int, default=16)
    args = ap.parse_args()
    import torch

    import scenarios
    from paper_2408_07609_amd import RTI_FLAG_PERSISTENT, Domain
    for name in args.configs:
        for flags in ((0, RTI_FLAG_PERSISTENT) if args.persistent else (0,)):
            sc = getattr(scenarios, name)()
            d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
                       flags=flags)
            d.set_tile_rows(args.tile_rows)
            d.step(4)
            prof, _ = d.profile(50)
            active, tiles, _ = d.active_tiles()
            torch.cuda.synchronize()
            t = time.perf_counter()
            d.step(400)
            torch.cuda.synchronize()
            per = (time.perf_counter() - t) / 400 * 1e6
            print(json.dumps({"workload": sc.name, "flags": flags, "tiles": tiles, "active_tiles": active,
                              "k_fused_us": prof.get("k_fused", 0.0) * 1e3, "k_active_us": prof.get("k_active", 0.0) * 1e3,
                              "graph_us_per_step": per}), flush=True)
            d.close()


if __name__ == "__main__":
    main()
