"""HIP path against the CPU oracle, through the C ABI, on the same seeded inputs.

Bar (FP64): every operation of the step is correctly rounded on both sides
(IEEE +, -, *, /, sqrt; a correctly rounded cube root on each side), the
formulas are evaluated operation by operation in the same order with no fused
multiply-add, so from the same state the two give the same bits: eta, M, N and
the maxima are compared for bitwise equality on every cell and face of every
level (which implies the required max |d eta| <= 1e-9 m, checked first).
The initial condition is the one part that is not exact: both sides evaluate
the source with their own exp, sin and cos (not correctly rounded), so a run
that starts from each side's own rti_set_source is held to the 1e-9 m bar
only, and the bitwise runs start the GPU from the oracle's initial level.
"""
import numpy as np
import pytest

import oracle
import scenarios

pytestmark = pytest.mark.gpu

TOL = 1e-9


def gpu_domain(sc, flags=0):
    from paper_2408_07609_amd import Domain
    return Domain(sc.levels, sc.dx0, sc.dt, g=sc.g, manning_n=sc.manning_n, dry_eps=sc.dry_eps, bc=sc.bc,
                  x0=sc.x0, y0=sc.y0, flags=flags)


def ora_domain(sc, **kw):
    return oracle.OracleDomain(**sc.oracle_kwargs(), **kw)


def diffs(d, o, nlev):
    out = []
    for k in range(nlev):
        e, M, N = d.get_state(k)
        eo, Mo, No = o.get_state(k)
        z, zo = d.max_inundation(k), o.max_inundation(k)
        assert np.all(np.isfinite(e)) and np.all(np.isfinite(M)) and np.all(np.isfinite(N))
        fs = max(1.0, np.abs(Mo).max(), np.abs(No).max())
        out.append(dict(eta=float(np.abs(e - eo).max()), M=float(np.abs(M - Mo).max() / fs),
                        N=float(np.abs(N - No).max() / fs), zmax=float(np.abs(z - zo).max()),
                        eta_equal=float(np.mean(e == eo))))
    return out


def assert_close(ds, tol=TOL, what=""):
    for k, d in enumerate(ds):
        print(f"{what} level {k}: {d}")
        assert d["eta"] <= tol and d["zmax"] <= tol, f"{what} level {k}: {d}"
        assert d["M"] <= tol and d["N"] <= tol, f"{what} level {k}: {d}"


def assert_bitwise(d, o, nlev, what=""):
    for k in range(nlev):
        for name, x, y in zip(("eta", "M", "N", "max"), d.get_state(k) + (d.max_inundation(k),),
                              o.get_state(k) + (o.max_inundation(k),)):
            assert np.array_equal(x, y), f"{what} level {k}: {name} not bitwise equal (max {np.abs(x - y).max():.3e})"


def start_from_oracle_source(d, o, sc):
    """The oracle's rti_set_source counterpart, copied to the GPU as a raw
    initial level (fluxes zero, maxima start there, like rti_set_source)."""
    o.set_source(*sc.source.astuple())
    for k in range(len(sc.levels)):
        d.set_eta(k, o.get_state(k)[0])


def set_random(d, o, sc, seed, flux=5.0):
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed, flux=flux)):
        h = sc.levels[k]["h"]
        z = np.where(h > 0, e, h + e)
        d.set_state(k, e, M, N)
        d.set_max(k, z)
        o.set_state(k, eta=e, M=M, N=N, zmax=z)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nlev", [1, 2, 3])
def test_one_step_random_state(nlev):
    """Every branch of one step (wet/dry faces, both flux signs, thin films,
    ring and edge exchanges, open sides) on a random state."""
    sc = scenarios.small_nested(seed=31 + nlev, nlev=nlev)
    d, o = gpu_domain(sc), ora_domain(sc)
    set_random(d, o, sc, seed=5)
    d.step(1)
    o.step(1)
    assert_close(diffs(d, o, nlev), what=f"one step nlev={nlev}")
    assert_bitwise(d, o, nlev, what=f"one step nlev={nlev}")


def test_steps_random_state_graph_and_eager_agree():
    sc = scenarios.small_nested(seed=40, nlev=3)
    from paper_2408_07609_amd import RTI_FLAG_NO_GRAPH
    a, b, o = gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_GRAPH), ora_domain(sc)
    set_random(a, o, sc, seed=6, flux=0.5)
    set_random(b, ora_domain(sc), sc, seed=6, flux=0.5)
    a.step(45)
    b.step(45)
    o.step(45)
    for k in range(3):
        ea, Ma, Na = a.get_state(k)
        eb, Mb, Nb = b.get_state(k)
        assert np.array_equal(ea, eb) and np.array_equal(Ma, Mb) and np.array_equal(Na, Nb)
    assert_close(diffs(a, o, 3), what="45 steps from a random state")
    assert_bitwise(a, o, 3, what="45 steps from a random state")


def test_set_source_matches_oracle():
    """rti_set_source against the oracle's source on every level: land cells
    and cells outside the uplift exactly, the displacement within a few ulp
    of its amplitude (each side's own exp, sin and cos)."""
    for sc in (scenarios.c1(), scenarios.small_nested(seed=7, nlev=3), scenarios.c2(scale=10)):
        d, o = gpu_domain(sc), ora_domain(sc)
        d.set_source(*sc.source.astuple())
        o.set_source(*sc.source.astuple())
        amp = abs(sc.source.amp)
        for k in range(len(sc.levels)):
            e, M, N = d.get_state(k)
            eo = o.get_state(k)[0]
            h = sc.levels[k]["h"]
            assert np.array_equal(e[h <= 0], eo[h <= 0]) and np.array_equal(e[eo == 0.0], eo[eo == 0.0])
            assert np.abs(e - eo).max() <= 8e-16 * amp, f"{sc.name} level {k}: {np.abs(e - eo).max()}"
            assert np.abs(d.max_inundation(k) - o.max_inundation(k)).max() <= 8e-16 * amp
            assert not M.any() and not N.any()


def test_c1_full_run():
    """Configuration 1: 256x256 at 810 m, shelf and shoals, 2 m hump, open
    sides, 1000 steps of 1 s.  From each side's own source: within 1e-9 m;
    from the oracle's initial level: bitwise."""
    sc = scenarios.c1()
    d, o = gpu_domain(sc), ora_domain(sc)
    d.set_source(*sc.source.astuple())
    o.set_source(*sc.source.astuple())
    d.run(sc.steps * sc.dt)
    o.run(sc.steps * sc.dt)
    assert d.steps == sc.steps == o.steps
    ds = diffs(d, o, 1)
    assert_close(ds, what="c1 full run")
    z = o.max_inundation(0)
    assert z.max() > 0.5
    d2 = gpu_domain(sc)
    start_from_oracle_source(d2, o2 := ora_domain(sc), sc)
    d2.run(sc.steps * sc.dt)
    o2.run(sc.steps * sc.dt)
    assert_bitwise(d2, o2, 1, what="c1 full run from the oracle's initial level")


def test_small_nested_source_run():
    sc = scenarios.small_nested(seed=7, nlev=3)
    d, o = gpu_domain(sc), ora_domain(sc)
    start_from_oracle_source(d, o, sc)
    d.step(3000)
    o.step(3000)
    ds = diffs(d, o, 3)
    assert_close(ds, what="small nested 3000 steps")
    assert_bitwise(d, o, 3, what="small nested 3000 steps")
    land = sc.levels[2]["h"] <= 0
    assert (o.max_inundation(2)[land] > 0.01).any(), "no inundation in the finest level"


@pytest.mark.timeout(900)
def test_c2_reduced_run():
    """Configuration 2 with every cell count divided by 10 (four levels at
    810/270/90/30 m over the same kind of coast), 4000 steps of 0.2 s."""
    sc = scenarios.c2(scale=10)
    d, o = gpu_domain(sc), ora_domain(sc)
    start_from_oracle_source(d, o, sc)
    d.step(4000)
    o.step(4000)
    assert_close(diffs(d, o, 4), what="c2/10 4000 steps")
    assert_bitwise(d, o, 4, what="c2/10 4000 steps")


def test_lake_at_rest_bitwise():
    sc = scenarios.small_nested(seed=11, nlev=3)
    d = gpu_domain(sc)
    before = [d.get_state(k)[0] for k in range(3)]
    d.step(1000)
    for k in range(3):
        e, M, N = d.get_state(k)
        assert np.array_equal(e, before[k])
        assert np.all(M == 0) and np.all(N == 0)


def test_mirror_symmetry_bitwise():
    n, dx = 41, 810.0
    X = (np.arange(n) + 0.5) * dx
    XX, YY = np.meshgrid(X, X)
    L = n * dx
    rng = np.random.default_rng(3)
    bump = rng.uniform(-30, 30, size=(n, n))
    h = 300.0 - 320.0 * np.exp(-(np.hypot(XX - L / 2, YY - L / 2) / (0.25 * L)) ** 2) + (bump + bump[:, ::-1])
    src = 1.5 * np.exp(-((XX - 0.3 * L) ** 2 + (YY - 0.4 * L) ** 2) / (2 * (3 * dx) ** 2))
    src = src + src[:, ::-1]
    sc = scenarios.Scenario("mirror", [dict(nx=n, ny=n, parent=-1, off_i=0, off_j=0, h=h)], dx0=dx, dt=1.0, steps=0)
    d = gpu_domain(sc)
    d.set_eta(0, src)
    d.step(300)
    e, M, N = d.get_state(0)
    assert np.abs(M).max() > 0
    assert np.array_equal(e, e[:, ::-1]) and np.array_equal(M, -M[:, ::-1]) and np.array_equal(N, N[:, ::-1])


def test_checkpoint_resume_bitwise():
    sc = scenarios.small_nested(seed=7, nlev=3)
    a = gpu_domain(sc)
    a.set_source(*sc.source.astuple())
    a.step(100)
    saved = [(a.get_state(k), a.max_inundation(k)) for k in range(3)]
    a.step(100)
    b = gpu_domain(sc)
    for k, ((e, M, N), z) in enumerate(saved):
        b.set_state(k, e, M, N)
        b.set_max(k, z)
    b.step(100)
    for k in range(3):
        for x, y in zip(a.get_state(k), b.get_state(k)):
            assert np.array_equal(x, y)
        assert np.array_equal(a.max_inundation(k), b.max_inundation(k))


def test_errors_on_gpu():
    from paper_2408_07609_amd import RtiError, RTI_ESTATE, RTI_EDIVERGED
    sc = scenarios.small_nested(seed=7, nlev=2)
    d = gpu_domain(sc)
    d.set_source(*sc.source.astuple())
    d.step(2)
    with pytest.raises(RtiError) as ei:
        d.set_source(*sc.source.astuple())
    assert ei.value.code == RTI_ESTATE
    e, M, N = d.get_state(1)
    e[5, 5] = np.nan
    d.set_state(1, e, M, N)
    with pytest.raises(RtiError) as ei:
        d.run(10 * sc.dt)
    assert ei.value.code == RTI_EDIVERGED


def test_divergence_watchdog_in_the_step():
    """The fused kernel checks every value it writes: a non-finite level set
    from the host is caught by rti_sync after plain rti_step calls (graphs of
    20 steps), the flag is sticky, further steps are refused, and a batch
    reports its diverged member at rti_batch_sync."""
    from paper_2408_07609_amd import RTI_EDIVERGED, RTI_STATUS_DIVERGED, Batch, RtiError
    sc = scenarios.small_nested(seed=7, nlev=3)
    d = gpu_domain(sc)
    d.set_source(*sc.source.astuple())
    d.step(40)
    d.sync()
    assert d.device_status() == 0
    e, M, N = d.get_state(2)
    e[4, 7] = np.inf
    d.set_state(2, e, M, N)
    d.step(40)
    with pytest.raises(RtiError) as ei:
        d.sync()
    assert ei.value.code == RTI_EDIVERGED
    assert d.device_status() & RTI_STATUS_DIVERGED
    with pytest.raises(RtiError) as ei:
        d.step(1)
    assert ei.value.code == RTI_EDIVERGED
    a, b = gpu_domain(sc), gpu_domain(scenarios.small_nested(seed=5, nlev=1, base=(150, 40)))
    a.set_source(*sc.source.astuple())
    e, M, N = a.get_state(0)
    M[3, 9] = np.nan
    a.set_state(0, e, M, N)
    with Batch([a, b]) as bt:
        bt.step(20)
        with pytest.raises(RtiError) as ei:
            bt.sync()
        assert ei.value.code == RTI_EDIVERGED
    assert b.device_status() == 0


def test_fused_phased_and_unskipped_agree_bitwise():
    """The fused tile kernel, the per-phase kernels and the fused kernel with
    tile skipping off produce identical bits."""
    from paper_2408_07609_amd import RTI_FLAG_NO_ACTIVE, RTI_FLAG_PHASED
    sc = scenarios.small_nested(seed=7, nlev=3)
    doms = [gpu_domain(sc), gpu_domain(sc, flags=RTI_FLAG_NO_ACTIVE), gpu_domain(sc, flags=RTI_FLAG_PHASED)]
    for d in doms:
        d.set_source(*sc.source.astuple())
        d.step(777)
    for k in range(3):
        ref = doms[2].get_state(k) + (doms[2].max_inundation(k),)
        for d in doms[:2]:
            got = d.get_state(k) + (d.max_inundation(k),)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y)
