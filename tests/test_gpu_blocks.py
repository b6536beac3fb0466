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
    compare(d, o, len(sc.levels), 1e-12, "one step")


def test_blocks_source_run():
    sc = scenarios.small_blocks()
    d, o = gpu(sc), oracle.OracleDomain(**sc.oracle_kwargs())
    d.set_source(*sc.source.astuple())
    o.set_source(*sc.source.astuple())
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

