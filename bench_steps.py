#!/usr/bin/env python
"""Per-step kernel times of a whole run traced with rocprofv3.

Input: the run_results.db of
    rocprofv3 --kernel-trace --stats -d DIR -o run -- python -u bench.py --config c2 --no-cpu-baseline
Dispatches are taken in start order from the `kernels` view; a step starts at
each k_active dispatch (the active-list launch) and takes the fused launch
(k_fused, or k_fused_loop on the small grid) and the split kernel after it.
The timed run starts after the longest gap among the first 300 steps (the
reset to t = 0 after the untimed graph-capture steps); the averages are over
windows of that run's steps.

    python bench_steps.py DIR/run_results.db [--steps 18000]
"""
from __future__ import annotations

import argparse
import sqlite3


def kind(name):
    for k, tag in (("k_active", "active"), ("k_fused_split", "split"), ("k_fused_loop", "loop"), ("k_fused", "fused")):
        if k in name:
            return tag
    return None


def steps_of(db):
    rows = sqlite3.connect(db).execute("select name, start, duration from kernels order by start").fetchall()
    steps, cur = [], None
    for name, start, dur in rows:
        k = kind(name)
        if k is None:
            continue
        if k == "active":
            cur = {"start": start, "active": 0.0, "fused": 0.0, "loop": 0.0, "split": 0.0, "small": False}
            steps.append(cur)
        elif cur is None:
            continue
        cur[k] += dur / 1000.0
        cur["small"] |= k == "loop"
    first_split = next(i for i, s in enumerate(steps) if s["split"] > 0)
    steps = steps[first_split:]
    gap, i_run = max((steps[i]["start"] - steps[i - 1]["start"], i) for i in range(1, min(300, len(steps))))
    return steps[i_run:]


def window(steps, a, b):
    w = steps[a:b]
    n = len(w)
    av = {k: sum(s[k] for s in w) / n for k in ("active", "fused", "loop", "split")}
    period = (w[-1]["start"] - w[0]["start"]) / (n - 1) / 1000.0
    return av, sum(av.values()), period, sum(1 for s in w if s["small"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--steps", type=int, default=18000, help="steps of the timed run")
    args = ap.parse_args()
    steps = steps_of(args.db)[:args.steps]
    print("| steps | k_active µs | k_fused µs | k_fused_loop µs | k_fused_split µs | sum µs | step period µs | on the small grid |")
    print("|---|---|---|---|---|---|---|---|")
    for a, b in ((0, 200), (0, 2000), (1800, 2000), (0, len(steps))):
        av, tot, per, small = window(steps, a, min(b, len(steps)))
        print(f"| {a + 1}-{min(b, len(steps))} | {av['active']:.2f} | {av['fused']:.2f} | {av['loop']:.2f} | "
              f"{av['split']:.2f} | {tot:.2f} | {per:.2f} | {small} |")


if __name__ == "__main__":
    main()
