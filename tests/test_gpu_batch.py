"""Tile shapes, the persistent grid, batches and the tile autotuner on the GPU.

The tile decomposition only decides which wavefront computes which cells,
never how a cell is computed, so every tile height, the persistent grid and
batched stepping must give bitwise the state and maxima of the default
single-domain run.  One batched member is also checked against the oracle.
"""
import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu


def members():
    """Uneven domains: 1 to 4 levels, a few hundred to ~100k cells."""
    return [
        scenarios.small_nested(seed=7, nlev=3),
        scenarios.small_nested(seed=11, nlev=2, base=(90, 72), child=(45, 54)),
        scenarios.small_nested(seed=5, nlev=1, base=(150, 40)),
        scenarios.small_nested(seed=13, nlev=3, base=(60, 66), child=(36, 30)),
        scenarios.c2(scale=10),
    ]


def make(sc, flags=0, precision=None, rows=None, source=True):
    from paper_2408_07609_amd import RTI_FP64, Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, flags=flags, precision=RTI_FP64 if precision is None else precision)
    if source:
        d.set_source(*sc.source.astuple())
    if rows is not None:
        d.set_tile_rows(rows)
    return d


def snapshot(d):
    return [(d.get_state(k), d.max_inundation(k)) for k in range(len(d.levels))]


def assert_same(a, b, what):
    assert len(a) == len(b)
    for k, ((sa, za), (sb, zb)) in enumerate(zip(a, b)):
        for name, x, y in zip(("eta", "M", "N"), sa, sb):
            assert np.array_equal(x, y), f"{what}: level {k} {name} differs (max {np.abs(x - y).max()})"
        assert np.array_equal(za, zb), f"{what}: level {k} maxima differ"


def test_tile_rows_and_persistent_grid_bitwise():
    from paper_2408_07609_amd import RTI_FLAG_NO_GRAPH, RTI_FLAG_PERSISTENT
    sc = scenarios.c2(scale=10)
    ref = make(sc)
    from paper_2408_07609_amd.rti import RTI_TILE_ROWS_DEFAULT
    assert ref.tile_rows == RTI_TILE_ROWS_DEFAULT
    ref.step(130)
    want = snapshot(ref)
    for rows in (4, 5, 6, 13, 24, 64):
        d = make(sc, rows=rows)
        assert d.tile_rows == rows
        d.step(130)
        assert_same(snapshot(d), want, f"tile rows {rows}")
    for flags in (RTI_FLAG_PERSISTENT, RTI_FLAG_PERSISTENT | RTI_FLAG_NO_GRAPH):
        d = make(sc, flags=flags)
        d.step(130)
        assert_same(snapshot(d), want, f"flags {flags}")
    # changing the height in the middle of a run
    d = make(sc)
    d.step(61)
    d.set_tile_rows(10)
    d.step(69)
    assert_same(snapshot(d), want, "height changed at step 61")


@pytest.mark.parametrize("precision", ["fp64", "fp32-bulk"])
@pytest.mark.parametrize("flags", [0, 0x8])
def test_batch_matches_alone_bitwise(precision, flags):
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64, Batch
    prec = RTI_FP64 if precision == "fp64" else RTI_FP32_BULK
    scs = members()
    rows = [6, 4, 9, 16, 6]
    alone = []
    for sc, r in zip(scs, rows):
        d = make(sc, precision=prec, rows=r)
        d.step(45)
        d.step(7)
        alone.append(snapshot(d))
        d.close()
    ds = [make(sc, precision=prec, rows=r) for sc, r in zip(scs, rows)]
    with Batch(ds, flags=flags) as b:
        assert len(b) == len(ds)
        b.step(45)          # two captured graphs of 20 steps and 5 single steps
        b.step(7)
        for d in ds:
            assert d.steps == 52
        for k, d in enumerate(ds):
            assert_same(snapshot(d), alone[k], f"member {k}")


def test_batch_membership_changes():
    from paper_2408_07609_amd import Batch
    scs = members()[:3]
    want = []
    for sc, n in zip(scs, (55, 75, 45)):
        d = make(sc)
        d.step(n)
        want.append(snapshot(d))
    a, bdom, c = (make(sc) for sc in scs)
    with Batch([a, bdom]) as b:
        b.step(30)
        b.add(c)            # joins from its own initial state
        b.step(25)
        b.remove(a)
        b.step(20)
        assert len(b) == 2
    assert (a.steps, bdom.steps, c.steps) == (55, 75, 45)
    for k, d in enumerate((a, bdom, c)):
        assert_same(snapshot(d), want[k], f"member {k}")
    # after the batch is gone the members step alone again, from either parity
    for sc, d, n in zip(scs, (a, bdom, c), (55, 75, 45)):
        ref = make(sc)
        ref.step(n + 23)
        d.step(23)
        assert_same(snapshot(d), snapshot(ref), "stepped alone after the batch")


def test_batched_member_against_oracle():
    from paper_2408_07609_amd import Batch
    scs = members()
    sc = scs[0]
    o = oracle.OracleDomain(**sc.oracle_kwargs())
    o.set_source(*sc.source.astuple())
    ds = [make(q) for q in scs]
    first = make(sc, source=False)
    for k in range(len(sc.levels)):              # the oracle's initial level (bitwise run)
        first.set_eta(k, o.get_state(k)[0])
    ds[0] = first
    with Batch(ds) as b:
        b.step(300)
    o.step(300)
    for k in range(len(sc.levels)):
        e, M, N = ds[0].get_state(k)
        eo, Mo, No = o.get_state(k)
        z, zo = ds[0].max_inundation(k), o.max_inundation(k)
        fs = max(1.0, np.abs(Mo).max(), np.abs(No).max())
        assert np.abs(e - eo).max() <= 1e-9
        assert np.abs(z - zo).max() <= 1e-9
        assert np.abs(M - Mo).max() / fs <= 1e-9 and np.abs(N - No).max() / fs <= 1e-9
        for name, x, y in (("eta", e, eo), ("M", M, Mo), ("N", N, No), ("max", z, zo)):
            assert np.array_equal(x, y), f"level {k}: {name} not bitwise equal"


def test_batch_rules():
    import torch
    from paper_2408_07609_amd import RTI_EINVAL, RTI_ESTATE, RTI_FP32_BULK, Batch, Domain, RtiError
    scs = members()
    a, b = make(scs[0]), make(scs[1])
    f32 = make(scs[2], precision=RTI_FP32_BULK)
    with Batch([a]) as batch:
        with pytest.raises(RtiError) as ei:
            a.step(1)                      # members step only through the batch
        assert ei.value.code == RTI_ESTATE
        with pytest.raises(RtiError) as ei:
            a.autotune(2)
        assert ei.value.code == RTI_ESTATE
        with pytest.raises(RtiError) as ei:
            batch.add(f32)                 # one precision per batch
        assert ei.value.code == RTI_EINVAL
        with pytest.raises(RtiError) as ei:
            Batch([a])                     # one batch per domain
        assert ei.value.code == RTI_ESTATE
        batch.add(b)
        batch.step(3)
        b.close()                          # a destroyed member leaves the batch
        assert len(batch) == 1
        batch.step(3)
        assert a.steps == 6


def test_autotune_restores_state():
    sc = scenarios.c2(scale=10)
    ref = make(sc)
    ref.step(100)
    want = snapshot(ref)
    d = make(sc)
    d.step(60)
    before = snapshot(d)
    rows, ms = d.autotune(5)
    assert rows in (4, 5, 6, 8, 10, 12, 16, 24) and ms > 0.0
    assert d.tile_rows == rows and d.steps == 60
    assert_same(snapshot(d), before, "state after autotune")
    d.step(40)
    assert_same(snapshot(d), want, "run continued after autotune")


def test_cell_update_counters():
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, Batch
    sc = scenarios.c2(scale=10)
    d = make(sc)
    d.step(200)                              # graph-replayed steps count too
    a0, c0 = d.cell_updates()
    assert a0 == sc.cells * 200 and 0 < c0 <= a0
    fused_avg_cells = d.profile(30)[1]       # eager steps, active cells read from each step's list
    a1, c1 = d.cell_updates()
    assert a1 - a0 == sc.cells * 30
    assert abs((c1 - c0) - fused_avg_cells * 30) < 0.5
    d.autotune(3)                            # the trials are not counted
    assert d.cell_updates() == (a1, c1)
    full = make(sc, flags=RTI_FLAG_NO_ACTIVE)
    full.step(25)
    assert full.cell_updates() == (sc.cells * 25, sc.cells * 25)
    scs = members()[:3]
    ds = [make(s) for s in scs]
    with Batch(ds) as b:
        b.step(40)
        ba, bc = b.cell_updates()
        assert ba == 40 * sum(s.cells for s in scs) and 0 < bc <= ba
        avg = b.profile(10)[2]
        ba2, bc2 = b.cell_updates()
        assert abs((bc2 - bc) - avg * 10) < 0.5
        b.add(make(members()[3]))            # the counter survives a rebuild of the tables
        b.step(5)
        assert b.cell_updates()[1] > bc2


def test_member_from_another_stream_is_adopted():
    import torch
    from paper_2408_07609_amd import Batch, Domain
    sc = members()[3]
    ref = make(sc)
    ref.step(90)
    other = torch.cuda.Stream()
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0, stream=other)
    d.set_source(*sc.source.astuple())
    d.step(21)                                # queued on its own stream
    with Batch([make(members()[0])]) as b:
        b.add(d)                              # waits for those steps, then runs on the batch's stream
        b.step(40)
        b.remove(d)
    d.step(29)                                # back on its own stream
    d.sync()
    assert d.steps == 90
    assert_same(snapshot(d), snapshot(ref), "adopted member")


def test_batch_autotuner_picks_one_height():
    """The batch-wide autotuner sets one candidate height on every member and
    reports a positive time; running the members at that height gives
    bitwise the results of the default height (the height changes only the
    decomposition)."""
    from paper_2408_07609_amd import Batch, autotune_batch_rows
    scs = members()[:3]
    copies = [make(sc) for sc in scs]
    rows, ms = autotune_batch_rows(copies, 3, candidates=(6, 12))
    assert rows in (6, 12) and ms > 0
    assert all(c.tile_rows == 12 for c in copies)          # the last candidate stays set
    a = [make(sc, rows=rows) for sc in scs]
    b = [make(sc) for sc in scs]
    with Batch(a) as ba:
        ba.step(60)
    with Batch(b) as bb:
        bb.step(60)
    for x, y in zip(a, b):
        assert_same(snapshot(x), snapshot(y), f"batch at {rows} rows vs the default")
