"""The FP64 operations of the HIP step against IEEE binary64 (through the
C-ABI diagnostic rti_math_probe).  The step's FP64 results can match the
oracle bit for bit only because each operation is correctly rounded on both
sides: the reciprocal of a face depth and the square roots are IEEE division
and square root, and the Manning term's cube root (Eqs. 2-3, D^(-7/3)) is
correctly rounded by construction on each side."""
import numpy as np
import pytest

import oracle
import pins

pytestmark = pytest.mark.gpu


def probe(op, x):
    import torch
    from paper_2408_07609_amd import rti
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    y = rti.math_probe(op, xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def inputs(n=1_000_000, seed=11):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(0.01, 6000.0, size=n // 2)                 # face depths of the workloads
    wide = np.exp2(rng.uniform(-1000.0, 1000.0, size=n - n // 2))  # every binade of the normal range
    return np.concatenate([1.0 / depth, depth, wide])


def test_cbrt_is_correctly_rounded():
    from paper_2408_07609_amd import rti
    x = inputs()
    got = probe(rti.RTI_PROBE_CBRT, x)
    want = oracle.cbrt_rn(x)                       # pinned to mpmath on the CPU (pins.pin_cbrt_rn)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} of {x.size} differ, e.g. x={x[bad[0]]!r}: {got[bad[0]]!r} vs {want[bad[0]]!r}"
    # exact cubes and the inputs nearest to a midpoint (these take the exact integer test)
    rng = np.random.default_rng(12)
    k = rng.integers(1, 1 << 17, size=4096).astype(np.float64)
    e = rng.integers(-300, 300, size=4096)
    assert np.array_equal(probe(rti.RTI_PROBE_CBRT, np.ldexp(k ** 3, 3 * e)), np.ldexp(k, e))
    xs, w = pins.cbrt_hard_cases(20000, seed=13)
    got = probe(rti.RTI_PROBE_CBRT, xs)
    bad = np.nonzero(got != w)[0]
    assert bad.size == 0, f"near-midpoint: {bad.size} of {xs.size} differ, e.g. x={xs[bad[0]]!r}"


def test_reciprocal_and_sqrt_are_ieee():
    from paper_2408_07609_amd import rti
    x = inputs(seed=14)
    d = x[(x >= 2.0 ** -767) & (x < 2.0 ** 1022)]                 # the face-depth reciprocal's domain
    assert d.size > 0.9 * x.size
    assert np.array_equal(probe(rti.RTI_PROBE_RECIP, d), 1.0 / d)
    rng = np.random.default_rng(16)                                # near the ends of the domain and at powers of 2
    edge = np.concatenate([np.exp2(rng.uniform(-767.0, -700.0, 100_000)), np.exp2(rng.uniform(950.0, 1021.99, 100_000)),
                           np.exp2(np.arange(-767.0, 1022.0)), np.nextafter(np.exp2(np.arange(-766.0, 1022.0)), 0.0),
                           np.array([1e-12, 0.01, 1.0, 3.0, 6000.0])])
    assert np.array_equal(probe(rti.RTI_PROBE_RECIP, edge), 1.0 / edge)
    assert np.array_equal(probe(rti.RTI_PROBE_SQRT, x), np.sqrt(x))
    sq = np.random.default_rng(15).uniform(0.0, 2.0e5, size=100_000)     # g h and M^2 + N^2 ranges
    assert np.array_equal(probe(rti.RTI_PROBE_SQRT, sq), np.sqrt(sq))
    assert np.array_equal(probe(rti.RTI_PROBE_SQRT, np.zeros(64)), np.zeros(64))
