"""rti_domain_autotune_noalloc (the autotuner for callers that cannot
allocate device memory) against rti_domain_autotune, through the C ABI.

The tile height an autotuner picks depends on timings, so the comparison is
on what is exact: each call restores the state, the maxima and the step
count bit for bit, and after the call both domains, stepped at the same tile
height, stay bitwise equal to each other and to a domain never tuned.  Two
calls in a row go through the one static array, the second on a smaller
domain; a domain whose state exceeds the array is refused before anything
runs."""
import numpy as np
import pytest

import scenarios

pytestmark = pytest.mark.gpu


def make(sc):
    from paper_2408_07609_amd import Domain
    d = Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
               x0=sc.x0, y0=sc.y0)
    d.set_source(*sc.source.astuple())
    return d


def snap(d):
    return [d.get_state(k) + (d.max_inundation(k),) for k in range(len(d.levels))]


def same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        for name, u, v in zip(("eta", "M", "N", "max"), x, y):
            assert np.array_equal(u, v), f"{what}: level {k} {name} differs"


@pytest.mark.parametrize("sc", [scenarios.small_nested(seed=7, nlev=3),
                                scenarios.small_nested(seed=5, nlev=1, base=(150, 40))],
                         ids=["nest3", "single-smaller"])
def test_noalloc_autotune_matches_autotune(sc):
    from paper_2408_07609_amd import RTI_AUTOTUNE_NOALLOC_MAX_BYTES
    a, b, ref = make(sc), make(sc), make(sc)
    for d in (a, b, ref):
        d.step(37)                                   # odd: the tuned state sits in the second buffer
    before = snap(a)
    same(before, snap(b), "before tuning")
    ra, ma = a.autotune(3)
    rb, mb = b.autotune_noalloc(3)
    print(f"{sc.name}: autotune -> {ra} rows ({ma:.4f} ms), noalloc -> {rb} rows ({mb:.4f} ms)")
    assert a.steps == b.steps == 37
    same(snap(a), before, "state after autotune")
    same(snap(b), before, "state after autotune_noalloc")
    assert ma > 0 and mb > 0 and rb in (4, 5, 6, 8, 10, 12, 16, 24)
    b.set_tile_rows(ra)
    for d in (a, b, ref):
        d.step(55)
    same(snap(a), snap(ref), "autotuned vs untuned after 55 steps")
    same(snap(b), snap(ref), "noalloc-tuned vs untuned after 55 steps")
    # a second call on the same domain, from the new state
    now = snap(b)
    b.autotune_noalloc(2)
    same(snap(b), now, "state after a second autotune_noalloc")
    assert RTI_AUTOTUNE_NOALLOC_MAX_BYTES == 128 << 20
    for d in (a, b, ref):
        d.close()


def test_noalloc_autotune_refuses_a_state_above_the_array():
    from paper_2408_07609_amd import RTI_ENOMEM, RtiError
    sc = scenarios.c2(scale=2)                       # 2.5 M cells: about 200 MB of state
    d = make(sc)
    before = snap(d)
    with pytest.raises(RtiError) as ei:
        d.autotune_noalloc(2)
    assert ei.value.code == RTI_ENOMEM and "static staging array" in str(ei.value)
    same(snap(d), before, "state after the refused call")
    d.close()
