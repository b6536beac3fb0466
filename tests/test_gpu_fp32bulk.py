"""FP32-bulk precision (h, M, N, maxima in binary32; water level, continuity,
face depth and wet/dry tests in binary64) against the FP64 path.

Stated error after a run (checked, and printed per run): the water level
differs from FP64 by at most 1e-3 m (RMS 1e-4 m), the maxima by 1e-3 m.
Still water stays bitwise still, and skipping stationary tiles is exact in
this precision too.
"""
import numpy as np
import pytest

import scenarios

pytestmark = pytest.mark.gpu


def dom(sc, precision, flags=0):
    from paper_2408_07609_amd import Domain
    return Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
                  x0=sc.x0, y0=sc.y0, flags=flags, precision=precision)


def errors(a, b, nlev):
    out = []
    for k in range(nlev):
        ea, eb = a.get_state(k)[0], b.get_state(k)[0]
        za, zb = a.max_inundation(k), b.max_inundation(k)
        out.append(dict(eta_max=float(np.abs(ea - eb).max()), eta_rms=float(np.sqrt(np.mean((ea - eb) ** 2))),
                        zmax_max=float(np.abs(za - zb).max())))
    return out


def check(errs, what):
    for k, e in enumerate(errs):
        print(f"{what} level {k}: {e}")
        assert e["eta_max"] <= 1e-3 and e["eta_rms"] <= 1e-4 and e["zmax_max"] <= 1e-3, f"{what} level {k}: {e}"


def test_fp32_bulk_lake_at_rest_bitwise():
    from paper_2408_07609_amd import RTI_FP32_BULK
    sc = scenarios.small_nested(seed=11, nlev=3)
    d = dom(sc, RTI_FP32_BULK)
    before = [d.get_state(k)[0] for k in range(3)]
    d.step(1000)
    for k in range(3):
        e, M, N = d.get_state(k)
        assert np.array_equal(e, before[k]) and np.all(M == 0) and np.all(N == 0)


def test_fp32_bulk_c1_full_run():
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64
    sc = scenarios.c1()
    a, b = dom(sc, RTI_FP32_BULK), dom(sc, RTI_FP64)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.run(sc.steps * sc.dt)
    check(errors(a, b, 1), "c1 fp32-bulk vs fp64")


def test_fp32_bulk_nested_run():
    from paper_2408_07609_amd import RTI_FP32_BULK, RTI_FP64
    sc = scenarios.small_nested(seed=7, nlev=3)
    a, b = dom(sc, RTI_FP32_BULK), dom(sc, RTI_FP64)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(3000)
    check(errors(a, b, 3), "small nested fp32-bulk vs fp64")


def test_fp32_bulk_skipping_is_exact():
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FP32_BULK
    sc = scenarios.c2(scale=2)
    a, b = dom(sc, RTI_FP32_BULK), dom(sc, RTI_FP32_BULK, flags=RTI_FLAG_NO_ACTIVE)
    for d in (a, b):
        d.set_source(*sc.source.astuple())
        d.step(400)
    active, total, _ = a.active_tiles()
    print(f"fp32-bulk c2/2: active tiles {active} of {total}")
    for k in range(len(sc.levels)):
        for x, y in zip(a.get_state(k) + (a.max_inundation(k),), b.get_state(k) + (b.max_inundation(k),)):
            assert np.array_equal(x, y)
