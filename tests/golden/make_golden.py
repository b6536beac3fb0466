"""Write the oracle references of the GPU full-run parity tests.

Only the oracle and the seeded generators are called.  Each file holds, per
level, the SHA-256 of the whole final eta, M, N and maxima arrays (float64,
row-major, as the oracle's arrays are laid out), the values at a stratified
sample of cells and faces (every parent cell of every child's ring, every
child edge face, the cells within 2 of the final shoreline, and random cells),
whole-level sums and extrema, and the count of inundated land cells; and the
SHA-256 of the oracle source that wrote it.

    python tests/golden/make_golden.py c2    # configuration 2, all 18,000 steps (about 1.5 h on 8 cores)
    python tests/golden/make_golden.py c3w   # configuration 3's grid, near-shore source, 3000 steps (about 1 h)
    python tests/golden/make_golden.py c3tw  # the same as touching blocks (masked levels), 3000 steps (about 1.5 h)

On a masked level (touching blocks) the ring cells and the injected faces
are those of the covered region (oracle.coverage), and cells outside are
not sampled.
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

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = {
    # name: (scenario, steps (None: the configuration's whole run), file)
    "c2": (lambda: scenarios.c2(), None, "c2_full_run.npz"),
    "c3w": (lambda: scenarios.c3_nearshore(), 3000, "c3_nearshore_3000.npz"),
    "c3tw": (lambda: scenarios.c3_touching_nearshore(), 3000, "c3_touching_nearshore_3000.npz"),
}
RANDOM = 4096
SHORE_CAP = 8192


def oracle_hash():
    with open(os.path.join(ROOT, "oracle", "rti_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def ring_cells(sc, k):
    """(i, j) of level k's cells on the ring of every child's footprint: the
    covered parent cells with an uncovered one among their 8 neighbours (a
    rectangle's outermost ring)."""
    out = []
    for c, lv in enumerate(sc.levels):
        if lv["parent"] != k:
            continue
        cov = np.pad(oracle.coverage(lv), 1)
        fh, fw = cov.shape[0] - 2, cov.shape[1] - 2
        for J in range(fh):
            for I in range(fw):
                if cov[J + 1, I + 1] and not cov[J:J + 3, I:I + 3].all():
                    out.append((lv["off_i"] + I, lv["off_j"] + J))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def injected_faces(lv):
    """Flat indices into M (ny x nx+1) and N (ny+1 x nx) of a child's faces that
    its parent injects: those on a parent face between a covered and an
    uncovered parent cell (a rectangle's four edges)."""
    ny, nx = lv["ny"], lv["nx"]
    cov = np.pad(oracle.coverage(lv), 1)
    xs = cov[1:-1, :-1] != cov[1:-1, 1:]            # (fh, fw + 1): x-face I between parent cells I-1, I
    ys = cov[:-1, 1:-1] != cov[1:, 1:-1]            # (fh + 1, fw)
    J, I = np.nonzero(xs)
    mx = ((3 * J)[:, None] + np.arange(3)) * (nx + 1) + (3 * I)[:, None]
    J, I = np.nonzero(ys)
    ny_ = (3 * J)[:, None] * nx + (3 * I)[:, None] + np.arange(3)
    return mx.ravel(), ny_.ravel()


def shoreline_band(h, e, eps, rng):
    """Cells within 2 cells of a wet/dry change in the final state (at most SHORE_CAP, drawn at random)."""
    wet = (h + e) > eps
    ny, nx = wet.shape
    pad = np.pad(wet, 2, mode="edge")
    anyw = np.zeros_like(wet)
    allw = np.ones_like(wet)
    for dj in range(5):
        for di in range(5):
            w = pad[dj:dj + ny, di:di + nx]
            anyw |= w
            allw &= w
    idx = np.flatnonzero(anyw & ~allw)
    if idx.size > SHORE_CAP:
        idx = np.sort(rng.choice(idx, size=SHORE_CAP, replace=False))
    return idx


def main(name):
    make, steps, fname = CASES[name]
    sc = make()
    steps = sc.steps if steps is None else steps
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    t0 = time.time()
    while o.steps < steps:
        o.step(min(250, steps - o.steps))
        print(f"{name}: {o.steps}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(2025)
    out = dict(steps=np.int64(o.steps), oracle_sha256=np.array(oracle_hash()), threads=np.int64(oracle.threads()),
               scenario=np.array(sc.name), seconds=np.float64(time.time() - t0))
    for k, lv in enumerate(sc.levels):
        e, M, N = o.get_state(k)
        z = o.max_inundation(k)
        h = lv["h"]
        ny, nx = e.shape
        out[f"l{k}_sha"] = np.array([sha(e), sha(M), sha(N), sha(z)])
        rc = ring_cells(sc, k)
        inside = oracle.level_mask(lv).ravel()
        cells = np.concatenate([rc[:, 1] * nx + rc[:, 0],
                                shoreline_band(h, e, sc.dry_eps, rng),
                                rng.choice(np.flatnonzero(inside), size=min(RANDOM, int(inside.sum())), replace=False)])
        cells = np.unique(cells)
        j, i = np.divmod(cells, nx)
        out[f"l{k}_cell"] = cells
        out[f"l{k}_eta"], out[f"l{k}_zmax"] = e[j, i], z[j, i]
        # faces: a child's edge faces (those the parent injects) and random interior faces
        if lv["parent"] >= 0:
            mx, ny_ = injected_faces(lv)
        else:
            mx, ny_ = np.zeros(0, np.int64), np.zeros(0, np.int64)
        mx = np.unique(np.concatenate([mx, rng.choice(M.size, size=RANDOM, replace=False)]))
        ny_ = np.unique(np.concatenate([ny_, rng.choice(N.size, size=RANDOM, replace=False)]))
        out[f"l{k}_mface"], out[f"l{k}_M"] = mx, M.reshape(-1)[mx]
        out[f"l{k}_nface"], out[f"l{k}_N"] = ny_, N.reshape(-1)[ny_]
        out[f"l{k}_stats"] = np.array([e.sum(), np.abs(e).max(), z.max(), np.abs(M).max(), np.abs(N).max()])
        out[f"l{k}_inundated"] = np.int64(np.count_nonzero((h <= 0) & (z > 0.01)))
        print(f"level {k}: {rc.shape[0]} ring cells, {cells.size} cells, {mx.size} + {ny_.size} faces, "
              f"{int(out[f'l{k}_inundated'])} inundated", flush=True)
    path = os.path.join(HERE, fname)
    np.savez_compressed(path, **out)
    print(f"wrote {path} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
