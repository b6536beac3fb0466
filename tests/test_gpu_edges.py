"""Degenerate and boundary cases of the step on the GPU against the oracle:
the smallest levels the ABI allows (3 cells across, a 9x9 child in the
smallest parent), ragged tile tails at several tile heights, all-land and
all-sea domains, no friction, walls on every side, zero steps.  Compared
within 1e-9 m, then for bitwise equality."""
import numpy as np
import pytest

import oracle
import scenarios
from scenarios import Scenario, Source

pytestmark = pytest.mark.gpu

TOL = 1e-9


def gpu(sc, rows=None, precision=0):
    from paper_2408_07609_amd import Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, precision=precision)
    if rows is not None:
        d.set_tile_rows(rows)
    return d


def compare(d, o, nlev, what, tol=TOL):
    for k in range(nlev):
        e, M, N = d.get_state(k)
        eo, Mo, No = o.get_state(k)
        fs = max(1.0, np.abs(Mo).max(), np.abs(No).max())
        err = dict(eta=np.abs(e - eo).max(), M=np.abs(M - Mo).max() / fs, N=np.abs(N - No).max() / fs,
                   zmax=np.abs(d.max_inundation(k) - o.max_inundation(k)).max())
        assert all(v <= tol for v in err.values()), f"{what} level {k}: {err}"
        for name, x, y in (("eta", e, eo), ("M", M, Mo), ("N", N, No),
                           ("max", d.max_inundation(k), o.max_inundation(k))):
            assert np.array_equal(x, y), f"{what} level {k}: {name} not bitwise equal"


def run_both(sc, steps, source=None, state_seed=None, rows=None):
    d, o = gpu(sc, rows), oracle.OracleDomain(**sc.oracle_kwargs())
    if source is not None:                         # the oracle's initial level on both (bitwise runs)
        o.set_source(*source.astuple())
        for k in range(len(sc.levels)):
            d.set_eta(k, o.get_state(k)[0])
    if state_seed is not None:
        for k, (e, M, N) in enumerate(scenarios.random_state(sc, state_seed, flux=1.0)):
            h = sc.levels[k]["h"]
            z = np.where(h > 0, e, h + e)
            d.set_state(k, e, M, N)
            d.set_max(k, z)
            o.set_state(k, eta=e, M=M, N=N, zmax=z)
    d.step(steps)
    o.step(steps)
    return d, o


def single(nx, ny, depth, dx=810.0, dt=1.0, **kw):
    sc = Scenario(f"single-{nx}x{ny}", [dict(nx=nx, ny=ny, parent=-1, off_i=0, off_j=0, h=None)], dx0=dx, dt=dt,
                  steps=0, **kw)
    X, Y = sc.cell_centres(0)
    sc.levels[0]["h"] = np.ascontiguousarray(depth(X, Y), dtype=np.float64)
    return sc


@pytest.mark.parametrize("shape", [(3, 3), (3, 41), (41, 3), (61, 7), (121, 13), (7, 121)])
def test_thin_and_ragged_single_levels(shape):
    """Strips three cells across, and widths and heights one past a tile
    (60 columns; 12 rows, the default height, and 6) so the last tile is
    ragged."""
    nx, ny = shape
    L = max(nx, ny) * 810.0
    sc = single(nx, ny, lambda X, Y: 200.0 - 190.0 * (X + Y) / (2 * L) + 5.0 * np.sin(X / 3e3))
    src = Source(0.3 * nx * 810.0, 0.4 * ny * 810.0, 4e3, 3e3, 0.3, 1.5, scenarios.GAUSS)
    d, o = run_both(sc, 300, source=src)
    compare(d, o, 1, f"{nx}x{ny} source run")
    d, o = run_both(sc, 40, state_seed=3)
    compare(d, o, 1, f"{nx}x{ny} random state")


def test_smallest_nest():
    """A root of 15x15 cells holding a 9x9 child (3x3 footprint, 3 cells of
    margin on every side), random state with wet and dry cells on both."""
    sc = Scenario("smallest-nest", [dict(nx=15, ny=15, parent=-1, off_i=0, off_j=0, h=None),
                                    dict(nx=9, ny=9, parent=0, off_i=6, off_j=6, h=None)],
                  dx0=810.0, dt=0.2, steps=0)
    for k in range(2):
        X, Y = sc.cell_centres(k)
        sc.levels[k]["h"] = np.ascontiguousarray(30.0 - 40.0 * X / (15 * 810.0))
    for rows in (4, 6, 64):
        d, o = run_both(sc, 60, state_seed=9, rows=rows)
        compare(d, o, 2, f"smallest nest, tile rows {rows}")


def test_all_land_stays_still():
    """No water anywhere: nothing moves, bitwise."""
    sc = scenarios.small_nested(seed=7, nlev=3)
    for lv in sc.levels:
        lv["h"] = -np.abs(lv["h"]) - 1.0
    d = gpu(sc)
    before = [d.get_state(k) for k in range(3)]
    d.step(100)
    for k in range(3):
        for x, y in zip(d.get_state(k), before[k]):
            assert np.array_equal(x, y)
        assert np.array_equal(d.max_inundation(k), np.zeros_like(before[k][0]))


@pytest.mark.parametrize("case", ["no_friction", "walls", "all_sea"])
def test_special_physics(case):
    sc = scenarios.small_nested(seed=19, nlev=3)
    if case == "no_friction":
        sc.manning_n = 0.0
    elif case == "walls":
        sc.bc = (1, 1, 1, 1)
    else:
        for lv in sc.levels:
            lv["h"] = np.abs(lv["h"]) + 5.0
    d, o = run_both(sc, 400, source=sc.source)
    compare(d, o, 3, case)


def test_zero_steps_is_a_no_op():
    sc = scenarios.small_nested(seed=7, nlev=2)
    d = gpu(sc)
    d.set_source(*sc.source.astuple())
    before = [d.get_state(k) for k in range(2)]
    d.step(0)
    d.run(0.0)
    assert d.steps == 0
    for k in range(2):
        for x, y in zip(d.get_state(k), before[k]):
            assert np.array_equal(x, y)
