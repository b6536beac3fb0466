"""Write tests/golden/c2_full_run.npz: sampled outputs of the CPU oracle after
the whole of configuration 2 (4 levels, 10.02 M cells, 3 m uplift, 18,000
steps of 0.2 s = 3600 s), for the GPU full-run parity test.

Only the oracle and the seeded generator are called.  Per level the file holds
the seeded sample of cell indices, eta, the maxima, M and N at those indices,
and whole-level sums and extrema.  The oracle source hash is stored so a test
can tell a stale file.

    python tests/golden/make_golden.py          # about an hour on 8 cores
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenarios  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_full_run.npz")
SAMPLES = 4096


def oracle_hash():
    with open(os.path.join(ROOT, "oracle", "rti_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main():
    sc = scenarios.c2()
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    t0 = time.time()
    chunk = 500
    while o.steps < sc.steps:
        o.step(min(chunk, sc.steps - o.steps))
        print(f"{o.steps}/{sc.steps} steps, {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(2024)
    out = dict(steps=np.int64(o.steps), oracle_sha256=np.array(oracle_hash()), threads=np.int64(oracle.threads()))
    for k, lv in enumerate(sc.levels):
        e, M, N = o.get_state(k)
        z = o.max_inundation(k)
        ny, nx = e.shape
        idx = rng.choice(nx * ny, size=min(SAMPLES, nx * ny), replace=False)
        j, i = np.divmod(idx, nx)
        out[f"l{k}_i"], out[f"l{k}_j"] = i, j
        out[f"l{k}_eta"], out[f"l{k}_zmax"] = e[j, i], z[j, i]
        out[f"l{k}_M"], out[f"l{k}_N"] = M[j, i], N[j, i]
        out[f"l{k}_stats"] = np.array([e.sum(), np.abs(e).max(), z.max(), np.abs(M).max(), np.abs(N).max()])
        land = lv["h"] <= 0
        out[f"l{k}_inundated"] = np.int64(np.count_nonzero(land & (z > 0.01)))
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
