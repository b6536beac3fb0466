"""Levels of touching blocks (one masked level per resolution) on the GPU
against the oracle: an L-shaped level of two touching 270 m blocks with a
90 m block across their junction, and two separate blocks held as one masked
level.  Every comparison is bitwise; cells outside a level read back 0."""
import numpy as np
import pytest

import oracle
import pins
import scenarios

pytestmark = pytest.mark.gpu


def gpu(sc, flags=0, rows=None, precision=0):
    from paper_2408_07609_amd import Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, flags=flags, precision=precision)
    if rows is not None:
        d.set_tile_rows(rows)
    return d


def compare(d, o, n, what):
    for k in range(n):
        got = (*d.get_state(k), d.max_inundation(k))
        want = (*o.get_state(k), o.max_inundation(k))
        for name, x, y in zip(("eta", "M", "N", "max"), got, want):
            assert np.abs(x - y).max() <= 1e-9, f"{what}: level {k} {name} off by {np.abs(x - y).max():.3e}"
            assert np.array_equal(x, y), f"{what}: level {k} {name} not bitwise equal"


def from_source(sc, rows=None, flags=0):
    """GPU and oracle started from the oracle's initial level."""
    d, o = gpu(sc, flags=flags, rows=rows), oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    for k in range(len(sc.levels)):
        d.set_eta(k, o.get_state(k)[0])
    return d, o


def merged_blocks():
    sc = scenarios.small_blocks()
    levels, _, _ = pins.merge_siblings(sc.levels, 1, 2)
    out = scenarios.Scenario("merged-blocks", levels, dx0=sc.dx0, dt=sc.dt, steps=0, source=sc.source)
    out.check_cfl()
    return out


@pytest.mark.parametrize("rows", [4, 7, 12])
def test_union_one_step_random_state(rows):
    """One step from a random state with noise on the outside cells: every
    branch of the step next to the boundary of the covered region."""
    sc = scenarios.small_union()
    d, o = gpu(sc, rows=rows), oracle.OracleDomain(**sc.oracle_kwargs())
    rng = np.random.default_rng(5)
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, 8, flux=3.0)):
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        if sc.levels[k].get("mask") is not None:
            out = sc.levels[k]["mask"] == 0
            e = np.where(out, rng.uniform(-5, 5, size=e.shape), e)
            z = np.where(out, rng.uniform(-5, 5, size=e.shape), z)
        d.set_state(k, e, M, N)
        d.set_max(k, z)
        o.set_state(k, eta=e, M=M, N=N, zmax=z)
    for n in (1, 2):
        d.step(1)
        o.step(1)
        compare(d, o, len(sc.levels), f"step {n}, tile rows {rows}")


def test_union_source_run():
    """600 steps of a wave over the L-shaped level and its child across the
    junction; the union floods."""
    sc = scenarios.small_union()
    d, o = from_source(sc)
    d.step(600)
    o.step(600)
    d.sync()
    compare(d, o, len(sc.levels), "600 steps")
    land = (sc.levels[1]["h"] <= 0) & (sc.levels[1]["mask"] != 0)
    assert (o.max_inundation(1)[land] > 0.05).sum() > 10
    out = sc.levels[1]["mask"] == 0
    assert np.all(d.get_state(1)[0][out] == 0.0) and np.all(d.max_inundation(1)[out] == 0.0)


def test_touching_chain_source_run():
    """Levels of touching blocks inside levels of touching blocks (a 3 x 2
    grid of 90 m blocks in two stepped 270 m blocks): bitwise the oracle
    after 600 steps and after 3000 (the flood running up and draining back
    across the blocks' shared edges); every level floods."""
    sc = scenarios.small_touching()
    d, o = from_source(sc)
    for n in (600, 2400):
        d.step(n)
        o.step(n)
        compare(d, o, len(sc.levels), f"touching chain, {o.steps} steps")
    for k in (1, 2):
        land = (sc.levels[k]["h"] <= 0) & (sc.levels[k]["mask"] != 0)
        assert (o.max_inundation(k)[land] > 0.05).sum() > 10, f"level {k} does not flood"


def test_merged_blocks_match_oracle():
    """Two 270 m blocks held as one masked level (and their children
    re-parented to it): bitwise the oracle after 300 steps."""
    sc = merged_blocks()
    d, o = from_source(sc)
    d.step(300)
    o.step(300)
    compare(d, o, len(sc.levels), "merged blocks, 300 steps")


def test_union_lake_at_rest():
    sc = scenarios.small_union()
    d = gpu(sc)
    before = [d.get_state(k) for k in range(len(sc.levels))]
    d.step(500)
    for k in range(len(sc.levels)):
        for x, y in zip(d.get_state(k), before[k]):
            assert np.array_equal(x, y), f"level {k} moved at rest"


@pytest.mark.parametrize("name", ["small_union", "small_touching"])
def test_union_skipping_and_phased_are_exact(name):
    """The fused kernel with stationary tiles skipped, without skipping, and
    the per-phase kernels give bitwise the same run."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FLAG_PHASED
    sc = getattr(scenarios, name)()
    runs = []
    for flags in (0, RTI_FLAG_NO_ACTIVE, RTI_FLAG_PHASED):
        d = gpu(sc, flags=flags)
        d.set_source(*sc.source.astuple())
        d.step(420)
        runs.append([(*d.get_state(k), d.max_inundation(k)) for k in range(len(sc.levels))])
    for r in runs[1:]:
        for k in range(len(sc.levels)):
            for name, x, y in zip(("eta", "M", "N", "max"), runs[0][k], r[k]):
                assert np.array_equal(x, y), f"level {k} {name} differs between kernel paths"


def test_union_in_a_batch():
    """A masked domain batched with plain ones steps bitwise as alone."""
    from paper_2408_07609_amd import Batch
    scs = [scenarios.small_union(), scenarios.small_nested(seed=7, nlev=3), merged_blocks()]
    alone = []
    for sc in scs:
        d = gpu(sc)
        d.set_source(*sc.source.astuple())
        d.step(240)
        alone.append([(*d.get_state(k), d.max_inundation(k)) for k in range(len(sc.levels))])
    doms = []
    for sc in scs:
        d = gpu(sc)
        d.set_source(*sc.source.astuple())
        doms.append(d)
    b = Batch(doms)
    b.step(240)
    b.sync()
    for m, (sc, d) in enumerate(zip(scs, doms)):
        for k in range(len(sc.levels)):
            for name, x, y in zip(("eta", "M", "N", "max"), (*d.get_state(k), d.max_inundation(k)), alone[m][k]):
                assert np.array_equal(x, y), f"member {m} level {k} {name}: batch differs from alone"
    b.close()


def test_union_fp32_bulk_close_to_fp64():
    """FP32-bulk on a masked level: the step runs (outside cells stay put,
    the ground sentinel is exact in FP32) and stays close to FP64."""
    sc = scenarios.small_union()
    a, b = gpu(sc), gpu(sc, precision=1)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(300)
    for k in range(len(sc.levels)):
        ea, eb = a.get_state(k)[0], b.get_state(k)[0]
        assert np.abs(ea - eb).max() < 0.05, f"level {k}: FP32-bulk level off by {np.abs(ea - eb).max():.2e} m"
    out = sc.levels[1]["mask"] == 0
    assert np.all(b.get_state(1)[0][out] == 0.0)
