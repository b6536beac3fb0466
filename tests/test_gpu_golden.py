"""Whole runs at full size on the GPU, in the benchmark's launch configuration
(fused kernel, active tiles, HIP graphs), against stored oracle references
written by tests/golden/make_golden.py (which calls only the oracle):

- configuration 2 (4 levels, 10.02 M cells, 3 m uplift), all 18,000 steps of
  0.2 s = 3600 s;
- configuration 3's grid (5 levels, 47.2 M cells) with the uplift 10 km
  offshore, so that the 30 m and 10 m levels flood within the window, 3000
  steps;
- the same coast and uplift on the paper's block counts as touching blocks
  (one masked level per resolution, 47.0 M cells), 3000 steps.

Both sides start from the oracle's initial level (the source's exp, sin and
cos are not correctly rounded on either side, so rti_set_source matches the
oracle's within a few ulp only; that is tested in test_gpu_parity).

FP64 bar: max |d eta| <= 1e-9 m and the same on the maxima at every stored
cell (every ring cell, every child edge face, the final shoreline band,
random cells), fluxes within 1e-9 of their scale; then every level's whole
eta, M, N and maxima arrays must have the oracle's SHA-256 (bitwise equality
of every cell and face), and the level sums and inundated counts must match.
FP32-bulk: the stated error of that precision against the FP64 oracle after
the run, printed and asserted.  The stored cells lean towards the shoreline
(every cell within 2 of a final wet/dry change, up to 8192 per level), where
FP32-bulk's error concentrates: a wet/dry test that flips a step earlier or
later moves a thin film.  Measured on C2's whole run: max |d eta| 3.4 cm (at
a shoreline cell of the 270 m level), RMS over the stored cells 5.7e-4 m,
maxima within 2.7e-4 m, the same inundated cells.
"""
import hashlib
import os

import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SRC = os.path.join(os.path.dirname(HERE), "oracle", "rti_oracle.c")
CASES = {
    "c2": (lambda: scenarios.c2(), "c2_full_run.npz"),
    "c3w": (lambda: scenarios.c3_nearshore(), "c3_nearshore_3000.npz"),
    "c3tw": (lambda: scenarios.c3_touching_nearshore(), "c3_touching_nearshore_3000.npz"),
}


def load_golden(name):
    path = os.path.join(HERE, "golden", CASES[name][1])
    if not os.path.exists(path):
        pytest.skip(f"tests/golden/{CASES[name][1]} not generated")
    g = np.load(path, allow_pickle=False)
    with open(ORACLE_SRC, "rb") as f:
        if str(g["oracle_sha256"]) != hashlib.sha256(f.read()).hexdigest():
            pytest.fail("the golden file was written by another oracle source; rerun tests/golden/make_golden.py")
    return g


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def run(name, precision, steps):
    from paper_2408_07609_amd import Domain
    sc = CASES[name][0]()
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, precision=precision)
    for k in range(len(sc.levels)):
        d.set_eta(k, o.get_state(k)[0])
    del o
    print(f"[{name}] {sc.cells} cells, {steps} steps", flush=True)
    d.run(steps * sc.dt)
    return sc, d


def compare(sc, d, g):
    res = []
    for k in range(len(sc.levels)):
        e, M, N = d.get_state(k)
        z = d.max_inundation(k)
        cells = g[f"l{k}_cell"]
        fs = max(1.0, float(g[f"l{k}_stats"][3]), float(g[f"l{k}_stats"][4]))
        de = np.abs(e.reshape(-1)[cells] - g[f"l{k}_eta"])
        res.append(dict(
            eta_max=float(de.max()), eta_rms=float(np.sqrt(np.mean(de ** 2))),
            zmax=float(np.abs(z.reshape(-1)[cells] - g[f"l{k}_zmax"]).max()),
            M=float(np.abs(M.reshape(-1)[g[f"l{k}_mface"]] - g[f"l{k}_M"]).max() / fs),
            N=float(np.abs(N.reshape(-1)[g[f"l{k}_nface"]] - g[f"l{k}_N"]).max() / fs),
            eta_sum_rel=float(abs(e.sum() - g[f"l{k}_stats"][0]) / max(1.0, np.abs(e).sum())),
            inundated=int(np.count_nonzero((sc.levels[k]["h"] <= 0) & (z > 0.01))),
            inundated_oracle=int(g[f"l{k}_inundated"]),
            sha_equal=[sha(a) == str(h) for a, h in zip((e, M, N, z), g[f"l{k}_sha"])],
            sums_equal=bool(e.sum() == g[f"l{k}_stats"][0] and z.max() == g[f"l{k}_stats"][2])))
        print(f"level {k}: {res[-1]}", flush=True)
    return res


@pytest.mark.timeout(1100)
@pytest.mark.parametrize("name", ["c2", "c3w", "c3tw"])
def test_full_run_fp64_matches_oracle(name):
    from paper_2408_07609_amd import RTI_FP64
    g = load_golden(name)
    sc, d = run(name, RTI_FP64, int(g["steps"]))
    assert d.steps == int(g["steps"])
    res = compare(sc, d, g)
    for k, r in enumerate(res):
        assert r["eta_max"] <= 1e-9 and r["zmax"] <= 1e-9, f"level {k}: {r}"
        assert r["M"] <= 1e-9 and r["N"] <= 1e-9, f"level {k}: {r}"
        assert r["eta_sum_rel"] <= 1e-12 and r["inundated"] == r["inundated_oracle"], f"level {k}: {r}"
    for k, r in enumerate(res):
        assert all(r["sha_equal"]) and r["sums_equal"], f"level {k}: eta/M/N/max not bitwise equal: {r}"
    assert max(int(g[f"l{k}_inundated"]) for k in range(len(sc.levels))) > 0, "the run never inundated land"


@pytest.mark.timeout(1100)
@pytest.mark.parametrize("name", ["c2", "c3w", "c3tw"])
def test_full_run_fp32_bulk_error(name):
    """FP32-bulk against the FP64 oracle after the run: max |d eta| <= 0.1 m,
    RMS over the stored (shoreline-heavy) cells <= 2e-3 m, maxima within
    1e-3 m, inundated land cells within 0.1 %."""
    from paper_2408_07609_amd import RTI_FP32_BULK
    g = load_golden(name)
    sc, d = run(name, RTI_FP32_BULK, int(g["steps"]))
    for k, r in enumerate(compare(sc, d, g)):
        assert r["eta_max"] <= 0.1 and r["eta_rms"] <= 2e-3 and r["zmax"] <= 1e-3, f"level {k}: {r}"
        assert abs(r["inundated"] - r["inundated_oracle"]) <= 0.001 * max(1, r["inundated_oracle"])
