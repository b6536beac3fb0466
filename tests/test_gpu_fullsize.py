"""Parity at the full sizes of the workloads, in the launch configuration the
benchmark times (fused kernel, active tiles, HIP graphs).

The oracle computes every cell of a few steps from a seeded random state of
the full grid (wet/dry mix, both flux signs, every exchange), so every output
of those steps is compared, not a sample: within 1e-9 m first, then for
bitwise equality (every FP64 operation is correctly rounded on both sides).  Skipping stationary tiles is checked
to be exact at full size against the same run with skipping off.
"""
import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu


def gpu_domain(sc, flags=0):
    from paper_2408_07609_amd import Domain
    return Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
                  x0=sc.x0, y0=sc.y0, flags=flags)


def run_random(sc, steps, seed):
    d = gpu_domain(sc)
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed, flux=1.0)):
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        d.set_state(k, e, M, N)
        d.set_max(k, z)
        o.set_state(k, eta=e, M=M, N=N, zmax=z)
        print(f"level {k} loaded", flush=True)
    d.step(steps)
    d.sync()
    o.step(steps)
    worst = {}
    for k in range(len(sc.levels)):
        e, M, N = d.get_state(k)
        eo, Mo, No = o.get_state(k)
        z, zo = d.max_inundation(k), o.max_inundation(k)
        worst[k] = (float(np.abs(e - eo).max()), float(np.abs(M - Mo).max()), float(np.abs(N - No).max()),
                    float(np.abs(z - zo).max()))
        print(f"level {k}: max|d eta| {worst[k][0]:.2e} |dM| {worst[k][1]:.2e} |dN| {worst[k][2]:.2e} "
              f"|d max| {worst[k][3]:.2e}", flush=True)
        assert max(worst[k]) <= 1e-9, f"level {k}: {worst[k]}"
        for name, x, y in (("eta", e, eo), ("M", M, Mo), ("N", N, No), ("max", z, zo)):
            assert np.array_equal(x, y), f"level {k}: {name} not bitwise equal"
    d.close()
    return worst


@pytest.mark.timeout(1200)
def test_c3_blocks_full_size_steps():
    """The 84-block layout of the paper's Table 1 (3/9/11/60 blocks at
    270/90/30/10 m, each in its own parent block)."""
    sc = scenarios.c3_blocks()
    for k, w in run_random(sc, 2, seed=304).items():
        assert max(w) <= 1e-9, f"block {k}: {w}"


@pytest.mark.timeout(1200)
def test_c3_touching_full_size_steps():
    """The paper's 3/9/11/60 blocks at 270/90/30/10 m as touching
    rectangles, one masked level per resolution (46,983,789 cells)."""
    sc = scenarios.c3_touching()
    for k, w in run_random(sc, 2, seed=305).items():
        assert max(w) <= 1e-9, f"level {k}: {w}"


@pytest.mark.timeout(900)
def test_c2_full_size_steps():
    sc = scenarios.c2()
    for k, w in run_random(sc, 3, seed=202).items():
        assert max(w) <= 1e-9, f"level {k}: {w}"


@pytest.mark.timeout(1200)
def test_c3_full_size_steps():
    sc = scenarios.c3()
    for k, w in run_random(sc, 2, seed=303).items():
        assert max(w) <= 1e-9, f"level {k}: {w}"


@pytest.mark.timeout(900)
def test_c2_small_grid_is_exact():
    """The fused kernel on the small grid that loops over the active list
    (what RTI_FLAG_PERSISTENT asks for) computes, bit for bit, what one
    workgroup per tile computes:
    configuration 2 (14,000 tiles, more than the small grid's workgroups)
    from its source for 300 steps, and 40 steps with every tile computed."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FLAG_PERSISTENT
    sc = scenarios.c2()
    for base, steps in ((0, 300), (RTI_FLAG_NO_ACTIVE, 40)):
        a, b = gpu_domain(sc, flags=base), gpu_domain(sc, flags=base | RTI_FLAG_PERSISTENT)
        for d in (a, b):
            d.set_source(*sc.source.astuple())
            d.step(steps)
            d.sync()
        for k in range(len(sc.levels)):
            for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
                assert np.array_equal(x, y), f"flags {base}: level {k}"
        print(f"flags {base}: {steps} steps bitwise equal", flush=True)
        a.close()
        b.close()


@pytest.mark.timeout(900)
def test_c2_graph_kinds_are_exact():
    """Configuration 2 from its source for 2000 steps, one graph at a time
    (so each graph's kind follows the count of the one before): graphs of
    both kinds (both kernels while few tiles are active, the fused kernel
    alone once many are) give, bit for bit, the same steps as launched one by
    one."""
    from paper_2408_07609_amd import RTI_FLAG_NO_GRAPH
    sc = scenarios.c2()
    a, b = gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_GRAPH)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        for _ in range(100):
            d.step(20)
            d.sync()
    kinds = a.graph_launches()
    print(f"graphs launched (default, dense): {kinds}", flush=True)
    assert sum(kinds) == 100 and all(n > 0 for n in kinds), kinds
    assert b.graph_launches() == (0, 0)
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"level {k}"
    a.close()
    b.close()


@pytest.mark.timeout(900)
def test_c2_tile_skipping_is_exact():
    """Configuration 2 from its source for 600 steps: the run that skips
    stationary tiles (dry land, sea still at rest) equals, bit for bit, the run that computes every tile,
    and it did skip tiles."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE
    sc = scenarios.c2()
    a, b = gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_ACTIVE)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(600)
        d.sync()
    active, total, cells = a.active_tiles()
    print(f"active tiles {active} of {total} ({cells} of {sc.cells} cells)")
    assert active < 0.9 * total
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"level {k}"


@pytest.mark.timeout(900)
def test_c3_blocks_tile_skipping_is_exact():
    """The 84-block layout from its source for 1500 steps: most of the sea is
    still at rest, so tiles at the edges of blocks and over the footprints of
    child blocks are skipped while their coupled tiles on the other level are
    stationary.  The skipping run equals, bit for bit, the run that computes
    every tile."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE
    sc = scenarios.c3_blocks()
    a, b = gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_ACTIVE)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(1500)
        d.sync()
    all_, computed = a.cell_updates()
    print(f"computed {computed} of {all_} cell updates ({computed / all_:.3f})")
    assert computed < 0.9 * all_
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"block {k}"
    a.close()
    b.close()


@pytest.mark.timeout(900)
def test_c3_touching_tile_skipping_is_exact():
    """The touching-block layout from its source for 1500 steps, skipping
    stationary tiles (the tiles wholly outside the staircase bands among
    them) against computing every tile: bitwise equal."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE
    sc = scenarios.c3_touching()
    a, b = gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_ACTIVE)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(1500)
        d.sync()
    all_, computed = a.cell_updates()
    print(f"computed {computed} of {all_} cell updates ({computed / all_:.3f})")
    assert computed < 0.9 * all_
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"level {k}"
    a.close()
    b.close()
