"""Levels made of several rectangular blocks (each block an entry of the
level table with its own parent) on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu


def gpu(sc, flags=0):
    from paper_2408_07609_amd import Domain
    return Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
                  x0=sc.x0, y0=sc.y0, flags=flags)


def compare(d, o, n, tol, what):
    for k in range(n):
        e, M, N = d.get_state(k)
        eo, Mo, No = o.get_state(k)
        fs = max(1.0, np.abs(Mo).max(), np.abs(No).max())
        err = (np.abs(e - eo).max(), np.abs(M - Mo).max() / fs, np.abs(N - No).max() / fs,
               np.abs(d.max_inundation(k) - o.max_inundation(k)).max())
        assert max(err) <= tol, f"{what}: block {k}: {err}"
        for name, x, y in (("eta", e, eo), ("M", M, Mo), ("N", N, No),
                           ("max", d.max_inundation(k), o.max_inundation(k))):
            assert np.array_equal(x, y), f"{what}: block {k}: {name} not bitwise equal"


def test_blocks_one_step_random_state():
    sc = scenarios.small_blocks()
    d, o = gpu(sc), oracle.OracleDomain(**sc.oracle_kwargs())
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, 8, flux=5.0)):
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        d.set_state(k, e, M, N)
        d.set_max(k, z)
        o.set_state(k, eta=e, M=M, N=N, zmax=z)
    d.step(1)
    o.step(1)
    compare(d, o, len(sc.levels), 1e-9, "one step")


def test_blocks_source_run():
    sc = scenarios.small_blocks()
    d, o = gpu(sc), oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    for k in range(len(sc.levels)):                # the oracle's initial level (bitwise runs)
        d.set_eta(k, o.get_state(k)[0])
    d.step(600)
    o.step(600)
    compare(d, o, len(sc.levels), 1e-9, "600 steps")
    for k in (6, 7):
        land = sc.levels[k]["h"] <= 0
        assert (o.max_inundation(k)[land] > 0.05).any(), f"no inundation in finest block {k}"


def test_blocks_lake_at_rest_and_phased_agree():
    from paper_2408_07609_amd import RTI_FLAG_PHASED
    sc = scenarios.small_blocks()
    d = gpu(sc)
    before = [d.get_state(k) for k in range(len(sc.levels))]
    d.step(500)
    for k in range(len(sc.levels)):
        for x, y in zip(d.get_state(k), before[k]):
            assert np.array_equal(x, y), f"block {k} moved at rest"
    a, b = gpu(sc), gpu(sc, flags=RTI_FLAG_PHASED)
    for x in (a, b):
        x.set_source(*sc.source.astuple())
        x.step(150)
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k), b.get_state(k)):
            assert np.array_equal(x, y), f"block {k}: fused and per-phase differ"



def many_children(nchild=34):
    """A 230x24 root (land in the west, sea in the east) holding nchild
    children of 9x9 cells in a row, 3 parent cells apart: more children than
    the per-tile child masks describe (32); the wave starts near the last
    children."""
    levels = [dict(nx=230, ny=24, parent=-1, off_i=0, off_j=0, h=None)]
    for q in range(nchild):
        levels.append(dict(nx=9, ny=9, parent=0, off_i=3 + 6 * q, off_j=10, h=None))
    sc = scenarios.Scenario(f"children{nchild}", levels, dx0=810.0, dt=0.5, steps=0)
    for k in range(len(levels)):
        X, Y = sc.cell_centres(k)
        sc.levels[k]["h"] = np.ascontiguousarray(-20.0 + 60.0 * X / (230 * 810.0) + 3.0 * np.sin(Y / 2e3))
    sc.source = scenarios.Source(0.85 * 230 * 810.0, 12 * 810.0, 20e3, 6e3, 0.0, 2.0, scenarios.GAUSS)
    sc.check_cfl()
    return sc


def test_more_than_32_children():
    """Ring means and edge injection for children beyond the 32 a tile's
    child mask holds: one step from a random state against the oracle, and a
    source run bitwise against the per-phase kernels."""
    from paper_2408_07609_amd import RTI_FLAG_PHASED
    sc = many_children()
    d, o = gpu(sc), oracle.OracleDomain(**sc.oracle_kwargs())
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, 12, flux=3.0)):
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        d.set_state(k, e, M, N)
        d.set_max(k, z)
        o.set_state(k, eta=e, M=M, N=N, zmax=z)
    d.step(1)
    o.step(1)
    compare(d, o, len(sc.levels), 1e-9, "one step")
    a, b = gpu(sc), gpu(sc, flags=RTI_FLAG_PHASED)
    for x in (a, b):
        x.set_source(*sc.source.astuple())
        x.step(400)
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"level {k}: fused and per-phase differ"
