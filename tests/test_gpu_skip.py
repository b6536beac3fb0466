"""Tile skipping at nest boundaries on the GPU.

A tile next to a child's edge, or over a child's footprint boundary, reads
values that another level writes (the edge fluxes the parent injects; the
child blocks averaged into the parent's ring cells).  Such a tile is skipped
only while its coupled tiles on that level are stationary too.  The nest here
lies wholly on dry land, so its edge and ring tiles are skipped until a dam
break floods across its edges: the skipping run must equal, bit for bit, the
run that computes every tile, and the oracle.
"""
import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu

CHUNKS = (1500, 1500, 2000, 2000)      # the water crosses the child's edge near step 1500, its grandchild's by 3500


def gpu(sc, flags=0, rows=None, precision=None):
    from paper_2408_07609_amd import RTI_FP64, Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, flags=flags, precision=RTI_FP64 if precision is None else precision)
    if rows is not None:
        d.set_tile_rows(rows)
    return d


def load_dam(sc, *doms):
    for k in range(len(sc.levels)):
        e, M, N = scenarios.dam_state(sc, k)
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        for d in doms:
            if isinstance(d, oracle.OracleDomain):
                d.set_state(k, eta=e, M=M, N=N, zmax=z)
            else:
                d.set_state(k, e, M, N)
                d.set_max(k, z)


def same(a, b, nlev, what):
    for k in range(nlev):
        for name, x, y in zip(("eta", "M", "N", "max"), a.get_state(k) + (a.max_inundation(k),),
                              b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y), f"{what}: level {k} {name} differs (max {np.abs(x - y).max()})"


@pytest.mark.parametrize("rows", [4, 6, 13])
def test_skipping_exact_when_water_crosses_nest_edges(rows):
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE
    sc = scenarios.inland_nest()
    a, b = gpu(sc, rows=rows), gpu(sc, flags=RTI_FLAG_NO_ACTIVE, rows=rows)
    load_dam(sc, a, b)
    computed = []
    for n in CHUNKS:
        c0 = a.cell_updates()[1]
        a.step(n)
        b.step(n)
        computed.append((a.cell_updates()[1] - c0) / (n * sc.cells))
        same(a, b, len(sc.levels), f"tile rows {rows}, after {a.steps} steps")
    print(f"tile rows {rows}: computed fraction per chunk {['%.3f' % f for f in computed]}")
    assert computed[0] < 0.6, "the dry nest was not skipped before the water came"
    for k in (1, 2, 3):
        h = sc.levels[k]["h"]
        assert (a.max_inundation(k)[h <= 0] > 0.1).sum() > 1000, f"level {k} did not flood"


def test_skipping_run_matches_oracle():
    """The skipping run against the oracle through the whole dam break (7000
    steps: the water crosses the edges of both children by step 3500 and the
    bore keeps running on the root), compared after every chunk.  Every FP64
    operation of the step is correctly rounded on both sides, so the two are
    equal bit for bit; the bar of 1e-9 m is checked first and named."""
    sc = scenarios.inland_nest()
    d, o = gpu(sc), oracle.OracleDomain(**sc.oracle_kwargs())
    load_dam(sc, d, o)
    for n in CHUNKS:
        d.step(n)
        o.step(n)
        for k in range(len(sc.levels)):
            e, M, N = d.get_state(k)
            eo, Mo, No = o.get_state(k)
            z, zo = d.max_inundation(k), o.max_inundation(k)
            fs = max(1.0, np.abs(Mo).max(), np.abs(No).max())
            err = (np.abs(e - eo).max(), np.abs(M - Mo).max() / fs, np.abs(N - No).max() / fs, np.abs(z - zo).max())
            print(f"step {o.steps} level {k}: {err}")
            assert max(err) <= 1e-9, f"step {o.steps} level {k}: {err}"
            for name, x, y in (("eta", e, eo), ("M", M, Mo), ("N", N, No), ("max", z, zo)):
                assert np.array_equal(x, y), f"step {o.steps} level {k}: {name} not bitwise equal"
    for k in (1, 3):
        h = sc.levels[k]["h"]
        assert (o.max_inundation(k)[h <= 0] > 0.1).sum() > 500, f"level {k} not flooded"


@pytest.mark.parametrize("precision", ["fp32-bulk"])
def test_skipping_exact_fp32_bulk_and_batched(precision):
    """The same in FP32-bulk, and for the nest stepped inside a batch with
    another domain (the batch kernel tests the same coupled tiles)."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FP32_BULK, Batch
    sc = scenarios.inland_nest()
    a = gpu(sc, precision=RTI_FP32_BULK)
    b = gpu(sc, flags=RTI_FLAG_NO_ACTIVE, precision=RTI_FP32_BULK)
    c = gpu(sc, precision=RTI_FP32_BULK)
    other = gpu(scenarios.small_nested(seed=7, nlev=3), precision=RTI_FP32_BULK)
    load_dam(sc, a, b, c)
    n = sum(CHUNKS)
    a.step(n)
    b.step(n)
    with Batch([c, other]) as batch:
        batch.step(n)
    same(a, b, len(sc.levels), "FP32-bulk skip vs every tile")
    same(c, b, len(sc.levels), "FP32-bulk batched vs every tile")


def test_stored_ring_means_match_per_phase_kernels():
    """The active-list launch keeps a ring cell's stored child-to-parent mean
    while the tiles writing its inputs stay stationary (here: the nest's
    rings lie on dry land until the flood crosses them).  The per-phase
    kernels compute every ring mean afresh each step; the two paths must agree
    bit for bit through the flood, with and without tile skipping."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FLAG_PHASED
    sc = scenarios.inland_nest()
    fused, fused_all, phased = gpu(sc), gpu(sc, flags=RTI_FLAG_NO_ACTIVE), gpu(sc, flags=RTI_FLAG_PHASED)
    load_dam(sc, fused, fused_all, phased)
    for n in CHUNKS:
        for d in (fused, fused_all, phased):
            d.step(n)
        same(fused, phased, len(sc.levels), f"fused vs per-phase after {fused.steps} steps")
        same(fused_all, phased, len(sc.levels), f"fused (every tile) vs per-phase after {fused.steps} steps")
