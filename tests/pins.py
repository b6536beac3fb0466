"""Pins of the CPU oracle to what the paper and mathematics fix.

Every pin runs the oracle (optionally a rebuilt copy of it, ``lib=``) on a
seeded input and checks a property that does not come from the oracle's own
formulas: an analytic solution, a conservation law, a symmetry, a truncation
error derived from the paper's differential equations, a brute-force maximum.
Each raises AssertionError on failure.  ``quick=True`` shrinks the sizes so a
battery of pins can run against many planted mistakes.

Equations referred to: continuity Eq. (1), momentum Eqs. (2)-(3), CFL Eq. (4),
all in Sec. II-A of arXiv 2408.07609; nesting rules in Sec. II-A; the
child->parent 3x3 mean in Sec. IV-C.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import scenarios

G = 9.81


def lvl(h, parent=-1, off_i=0, off_j=0):
    h = np.ascontiguousarray(h, dtype=np.float64)
    ny, nx = h.shape
    return dict(nx=nx, ny=ny, parent=parent, off_i=off_i, off_j=off_j, h=h)


def dom(levels, dx0, dt, lib=None, **kw):
    return oracle.OracleDomain(levels, dx0, dt, lib=lib, **kw)


# ---------------------------------------------------------------------------
def pin_lake_at_rest(lib=None, quick=False):
    """Still water over arbitrary bathymetry stays still, bitwise: nested
    levels whose shorelines cross the exchange strips, friction on, open
    sides, and sea cells shallower than the dry threshold."""
    sc = scenarios.small_nested(seed=11, nlev=3)
    rng = np.random.default_rng(12)
    for lv in sc.levels:
        h = lv["h"]
        near = np.abs(h) < 2.0
        lv["h"] = np.where(near, rng.uniform(-0.02, 0.02, size=h.shape), h)
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
    d.set_lake_at_rest()
    before = [d.get_state(k)[0] for k in range(d.nlev)]
    d.step(200 if quick else 3000)
    for k in range(d.nlev):
        e, M, N = d.get_state(k)
        assert np.array_equal(e, before[k]), f"lake at rest: level {k} eta moved by {np.abs(e - before[k]).max()}"
        assert np.all(M == 0.0) and np.all(N == 0.0), f"lake at rest: level {k} max |flux| {max(np.abs(M).max(), np.abs(N).max())}"


def _volume(d, counted_masks, clip=True):
    terms = []
    for k in range(d.nlev):
        e = d.level(k)["eta"]
        c = d.level(k)["clip"] if clip else None
        w = d.dx[k] ** 2
        m = counted_masks[k]
        terms.extend((e[m] * w).ravel().tolist())
        if c is not None:
            terms.extend((-c[m] * w).ravel().tolist())
    return math.fsum(terms)


def pin_closed_mass(lib=None, quick=False):
    """Continuity Eq. (1) conserves volume in a closed basin: with walls on
    every side, sum(eta dx^2) minus the clipped volume is constant to
    rounding (coastal basin with wetting and drying, friction on).  The
    water depth h + eta is never negative."""
    sc = scenarios.small_nested(seed=5, nlev=1, bc=(1, 1, 1, 1))
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc, track_clip=True)
    (e, M, N), = scenarios.random_state(sc, seed=6, flux=0.5)
    d.set_state(0, eta=e, M=M, N=N)
    d.bc_root()                 # the walls carry no flux from the start
    mask = [np.ones_like(sc.levels[0]["h"], dtype=bool)]
    v0 = _volume(d, mask)
    scale = math.fsum(np.abs(d.level(0)["eta"]).ravel().tolist()) * d.dx[0] ** 2
    d.step(100 if quick else 2000)
    v1 = _volume(d, mask)
    assert np.abs(d.level(0)["M"]).max() > 0.0
    assert np.all(sc.levels[0]["h"] + d.level(0)["eta"] >= 0.0), "negative water depth"
    assert d.clipped_depth(0).max() > 0.0, "no cell dried below the ground (clip path not exercised)"
    assert abs(v1 - v0) <= 1e-12 * scale, f"closed mass drift {abs(v1 - v0) / scale:.3e} (relative)"


def footprint_masks(sc_levels):
    """Cells counted once in a nested volume: every cell inside its level
    and not covered by a child."""
    masks = [oracle.level_mask(lv).copy() for lv in sc_levels]
    for lv in sc_levels[1:]:
        p = lv["parent"]
        masks[p][lv["off_j"]:lv["off_j"] + lv["ny"] // 3, lv["off_i"]:lv["off_i"] + lv["nx"] // 3] &= \
            ~oracle.coverage(lv)
    return masks


def pin_nested_mass(lib=None, quick=False):
    """Volume is conserved across levels: with a closed root, the volume of
    the cells not covered by a child (the finest level whole) minus the
    clipped volume stays constant.  It holds only if the fluxes injected on a
    child's edge carry exactly the discharge of the parent faces there, at the
    same time level.  Random fluxes everywhere make every edge carry flow from
    the first step."""
    sc = scenarios.small_nested(seed=21, nlev=3, bc=(1, 1, 1, 1))
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc, track_clip=True)
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed=22, flux=0.5)):
        d.set_state(k, eta=e, M=M, N=N)
    d.bc_root()         # the walls carry no flux from the start
    for k in range(1, d.nlev):
        d.jnq(k)        # child edges start consistent with their parents
    masks = footprint_masks(sc.levels)
    v0 = _volume(d, masks)
    scale = sum(math.fsum(np.abs(d.level(k)["eta"][masks[k]]).ravel().tolist()) * d.dx[k] ** 2
                for k in range(d.nlev))
    d.step(100 if quick else 2000)
    v1 = _volume(d, masks)
    assert max(np.abs(d.level(k)["M"]).max() for k in range(1, d.nlev)) > 0.0
    assert abs(v1 - v0) <= 1e-12 * scale, f"nested mass drift {abs(v1 - v0) / scale:.3e} (relative)"


# ---------------------------------------------------------------------------
def dispersion_theta(h, dt, dx, kx, ky):
    """Angle per step of the linearised staggered leap-frog scheme:
    sin^2(theta/2) = (sqrt(g h) dt/dx)^2 (sin^2(kx dx/2) + sin^2(ky dx/2))."""
    s2 = (math.sqrt(G * h) * dt / dx) ** 2 * (math.sin(kx * dx / 2) ** 2 + math.sin(ky * dx / 2) ** 2)
    return 2.0 * math.asin(math.sqrt(s2))


def _mode_run(amp, lib, nsteps, nx=24, ny=18, h0=100.0, dx=810.0, dt=4.0, modes=((2, 1), (1, 3))):
    h = np.full((ny, nx), h0)
    d = dom([lvl(h)], dx, dt, lib=lib, manning_n=0.0, bc=(1, 1, 1, 1))
    X = (np.arange(nx) + 0.5) * dx
    Y = (np.arange(ny) + 0.5) * dx
    XX, YY = np.meshgrid(X, Y)
    shapes, thetas = [], []
    for (p, q) in modes:
        kx, ky = math.pi * p / (nx * dx), math.pi * q / (ny * dx)
        shapes.append(np.cos(kx * XX) * np.cos(ky * YY))
        thetas.append(dispersion_theta(h0, dt, dx, kx, ky))
    d.set_eta(0, amp * sum(shapes))
    d.step(nsteps)
    exact = sum(amp * s * math.cos((nsteps - 0.5) * th) / math.cos(th / 2) for s, th in zip(shapes, thetas))
    return np.abs(d.level(0)["eta"] - exact).max() / amp


def pin_dispersion(lib=None, quick=False):
    """Flat bottom, closed basin, no friction: a sum of two cosine modes
    evolves as eta^n = sum a cos(kx x) cos(ky y) cos((n-1/2) theta)/cos(theta/2),
    the exact solution of the linearised scheme (theta from the discrete
    dispersion relation).  The nonlinear model departs from it only at order
    a/h, so the relative error must shrink in proportion to the amplitude."""
    n = 150 if quick else 600
    e2 = _mode_run(1e-2, lib, n)
    e3 = _mode_run(1e-3, lib, n)
    e4 = _mode_run(1e-4, lib, n)
    assert e4 < 2e-3, f"dispersion: relative error {e4:.3e} at a = 1e-4 m"
    assert 5.0 < e3 / e4 < 20.0 and 5.0 < e2 / e3 < 20.0, f"dispersion: error not linear in a ({e2:.2e}, {e3:.2e}, {e4:.2e})"


def pin_standing_period(lib=None, quick=False):
    """The (1,0) standing mode of a closed flat channel has period
    2 pi dt / theta in steps (discrete) and 2 L / sqrt(g h) in time
    (continuous); the measured period agrees with both."""
    nx, ny, h0, dx, dt = 64, 3, 100.0, 810.0, 1.0
    d = dom([lvl(np.full((ny, nx), h0))], dx, dt, lib=lib, manning_n=0.0, bc=(1, 1, 1, 1))
    X = (np.arange(nx) + 0.5) * dx
    k = math.pi / (nx * dx)
    d.set_eta(0, np.tile(1e-3 * np.cos(k * X), (ny, 1)))
    steps = 3600 if quick else 7000
    series = np.empty(steps)
    for s in range(steps):
        d.step(1)
        series[s] = d.level(0)["eta"][1, 0]
    sgn = np.sign(series)
    idx = np.nonzero(sgn[1:] != sgn[:-1])[0]
    t = [(i + 1) + series[i] / (series[i] - series[i + 1]) for i in idx]   # step count at zero crossings
    period = 2.0 * float(np.mean(np.diff(t)))
    th = dispersion_theta(h0, dt, dx, k, 0.0)
    p_disc = 2 * math.pi / th
    p_cont = 2 * nx * dx / math.sqrt(G * h0) / dt
    assert abs(period - p_disc) / p_disc < 2e-3, f"period {period:.2f} vs discrete {p_disc:.2f}"
    assert abs(period - p_cont) / p_cont < 5e-3, f"period {period:.2f} vs continuous {p_cont:.2f}"


def pin_wave_speed(lib=None, quick=False):
    """A long wave travels at sqrt(g h): the crest of a y-uniform pulse in a
    flat channel arrives at the time distance / sqrt(g h)."""
    nx, ny, h0, dx, dt = 400, 3, 50.0, 200.0, 2.0
    d = dom([lvl(np.full((ny, nx), h0))], dx, dt, lib=lib, manning_n=0.0, bc=(1, 1, 1, 1))
    X = (np.arange(nx) + 0.5) * dx
    x0 = 100 * dx
    d.set_eta(0, np.tile(1e-3 * np.exp(-((X - x0) / (8 * dx)) ** 2), (ny, 1)))
    c = math.sqrt(G * h0)
    probe = 300
    t_exp = (X[probe] - x0) / c
    steps = int(1.3 * t_exp / dt)
    series = np.empty(steps)
    for s in range(steps):
        d.step(1)
        series[s] = d.level(0)["eta"][1, probe]
    i = int(np.argmax(series))
    a, b, cc = series[i - 1], series[i], series[i + 1]
    t_peak = (i + 1 + 0.5 * (a - cc) / (a - 2 * b + cc)) * dt
    assert abs(t_peak - t_exp) / t_exp < 0.01, f"arrival {t_peak:.1f} s vs {t_exp:.1f} s"


# ---------------------------------------------------------------------------
def pin_mirror_symmetry(lib=None, quick=False):
    """Bitwise mirror and transpose symmetry on one level: x-symmetric depth
    and source give an x-symmetric level (M odd, N even); a transposed input
    gives the transposed output.  Wetting and drying, friction and open
    sides are all on."""
    n = 41
    dx, dt = 810.0, 1.0
    X = (np.arange(n) + 0.5) * dx
    XX, YY = np.meshgrid(X, X)
    L = n * dx
    rng = np.random.default_rng(3)
    r = np.hypot(XX - L / 2, YY - L / 2)
    hsym = 300.0 - 320.0 * np.exp(-(r / (0.25 * L)) ** 2)          # an island in the middle
    bump = rng.uniform(-30, 30, size=(n, n))
    hx = hsym + (bump + bump[:, ::-1])                                 # symmetric in x only
    steps = 80 if quick else 400

    def run(h, src):
        d = dom([lvl(h)], dx, dt, lib=lib)
        d.set_eta(0, src)
        d.step(steps)
        return d.get_state(0)

    srcx = 1.5 * np.exp(-((XX - 0.3 * L) ** 2 + (YY - 0.4 * L) ** 2) / (2 * (3 * dx) ** 2))
    srcx = srcx + srcx[:, ::-1]
    e, M, N = run(hx, srcx)
    assert np.abs(M).max() > 0 and np.any((hx + e <= 0.01) & (hx > -1e9))
    assert np.array_equal(e, e[:, ::-1]), "x-mirror: eta not symmetric"
    assert np.array_equal(M, -M[:, ::-1]), "x-mirror: M not odd"
    assert np.array_equal(N, N[:, ::-1]), "x-mirror: N not even"

    ha = hsym + bump
    srca = 1.5 * np.exp(-((XX - 0.3 * L) ** 2 + (YY - 0.6 * L) ** 2) / (2 * (3 * dx) ** 2))
    e1, M1, N1 = run(ha, srca)
    e2, M2, N2 = run(np.ascontiguousarray(ha.T), np.ascontiguousarray(srca.T))
    assert np.array_equal(e1, e2.T), "transpose: eta"
    assert np.array_equal(M1, N2.T) and np.array_equal(N1, M2.T), "transpose: fluxes"


def pin_nested_symmetry(lib=None, quick=False):
    """Mirror symmetry with a centred nest: symmetric to rounding (the 3x3
    sums of the child->parent exchange run in a fixed order, so the mirror
    image adds the same numbers in another order)."""
    dx, dt = 810.0, 1.0
    npx, npy = 45, 33
    Xp = (np.arange(npx) + 0.5) * dx
    Yp = (np.arange(npy) + 0.5) * dx
    Lx = npx * dx

    def depth(XX, YY):
        return 120.0 - 140.0 * np.exp(-((XX - Lx / 2) / (0.12 * Lx)) ** 2) + 5.0 * np.cos(YY / 3000.0)

    XX, YY = np.meshgrid(Xp, Yp)
    parent = lvl(depth(XX, YY))
    cnx, cny, oi, oj = 27, 27, 18, 12
    Xc = oi * dx + (np.arange(cnx) + 0.5) * dx / 3
    Yc = oj * dx + (np.arange(cny) + 0.5) * dx / 3
    XC, YC = np.meshgrid(Xc, Yc)
    child = lvl(depth(XC, YC), parent=0, off_i=oi, off_j=oj)
    d = dom([parent, child], dx, dt, lib=lib)
    src = lambda XX, YY: 1.0 * (np.exp(-((XX - 0.3 * Lx) ** 2 + (YY - 0.5 * npy * dx) ** 2) / (2 * (4 * dx) ** 2))
                                + np.exp(-((XX - 0.7 * Lx) ** 2 + (YY - 0.5 * npy * dx) ** 2) / (2 * (4 * dx) ** 2)))
    d.set_eta(0, src(XX, YY))
    d.set_eta(1, src(XC, YC))
    d.step(60 if quick else 300)
    for k in range(2):
        e, M, N = d.get_state(k)
        assert np.abs(M).max() > 1e-3
        assert np.abs(e - e[:, ::-1]).max() <= 1e-9 * max(1.0, np.abs(e).max()), f"nested mirror: level {k} eta"
        assert np.abs(M + M[:, ::-1]).max() <= 1e-9 * np.abs(M).max(), f"nested mirror: level {k} M"


# ---------------------------------------------------------------------------
def pin_friction_ode(lib=None, quick=False):
    """Uniform flow on a flat bed feels friction only: far from the walls the
    flux follows the Manning ODE dM/dt = -g n^2 M|M| / D^(7/3) of
    Eqs. (2)-(3), whose solution is M(t) = M0 / (1 + k M0 t),
    k = g n^2 / D^(7/3).  The scheme converges to it as dt shrinks."""
    n, h0, dx, M0, nman, T = 96, 2.0, 100.0, 1.5, 0.05, 8.0
    k = G * nman ** 2 / h0 ** (7.0 / 3.0)
    exact = M0 / (1.0 + k * M0 * T)
    errs = []
    for dt in (1.0, 0.5, 0.25):
        d = dom([lvl(np.full((n, n), h0))], dx, dt, lib=lib, manning_n=nman, bc=(1, 1, 1, 1))
        d.set_lake_at_rest()
        M = np.full((n, n + 1), M0)
        M[:, 0] = 0.0
        M[:, n] = 0.0
        d.set_state(0, M=M)
        steps = int(round(T / dt))
        d.step(steps)
        assert steps < n // 2 - 2
        errs.append(abs(d.level(0)["M"][n // 2, n // 2] - exact))
    assert errs[-1] / exact < 2e-3, f"friction: relative error {errs[-1] / exact:.2e}"
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8, f"friction: no convergence {errs}"


# ---------------------------------------------------------------------------
def _smooth_fields():
    import sympy as sp
    x, y = sp.symbols("x y", real=True)
    Lp = 100e3
    k = 2 * sp.pi / Lp
    h = 50 + 10 * sp.sin(k * x) * sp.cos(k * y)
    eta = sp.Rational(1, 2) * sp.cos(k * x + 0.3) * sp.sin(k * y + 0.7)
    M = 15 * sp.sin(k * x + 1.0) * sp.cos(k * y - 0.4) + 4
    N = 12 * sp.cos(k * x - 0.2) * sp.sin(k * y + 0.9) - 3
    D = h + eta
    return sp, x, y, Lp, h, eta, M, N, D


def _consistency(n, lib, nman=0.025, dt=1e-3):
    """One momentum update (and one mass update) of smooth fields on an
    n x n grid; returns the discrete tendencies and the analytic right-hand
    sides of Eqs. (1)-(3) at the same points, plus the leading truncation
    term predicted for first-order upwind advection."""
    sp, x, y, Lp, h, eta, M, N, D = _smooth_fields()
    g = G
    S = sp.sqrt(M ** 2 + N ** 2)
    rhs_M = -(sp.diff(M ** 2 / D, x) + sp.diff(M * N / D, y) + g * D * sp.diff(eta, x)
              + g * nman ** 2 * M * S / D ** sp.Rational(7, 3))
    rhs_N = -(sp.diff(M * N / D, x) + sp.diff(N ** 2 / D, y) + g * D * sp.diff(eta, y)
              + g * nman ** 2 * N * S / D ** sp.Rational(7, 3))
    rhs_e = -(sp.diff(M, x) + sp.diff(N, y))
    f = {nm: sp.lambdify((x, y), ex, "numpy") for nm, ex in dict(
        h=h, eta=eta, M=M, N=N, rhs_M=rhs_M, rhs_N=rhs_N, rhs_e=rhs_e,
        qxx=sp.diff(M ** 2 / D, x, 2), pyy=sp.diff(M * N / D, y, 2),
        rxx=sp.diff(M * N / D, x, 2), qyy=sp.diff(N ** 2 / D, y, 2)).items()}
    dx = Lp / n
    xc = (np.arange(n) + 0.5) * dx
    xf = np.arange(n + 1) * dx
    ev = lambda name, X, Y: np.broadcast_to(f[name](*np.meshgrid(X, Y)), (len(Y), len(X))).astype(np.float64)
    hc = ev("h", xc, xc)
    d = dom([lvl(hc)], dx, dt, lib=lib, manning_n=nman, bc=(1, 1, 1, 1))
    e0, M0, N0 = ev("eta", xc, xc), ev("M", xf, xc), ev("N", xc, xf)
    d.set_state(0, eta=e0, M=M0, N=N0)
    d.momentum(0)
    _, M1, N1 = d.get_state(0)
    d.set_state(0, eta=e0, M=M0, N=N0)
    d.mass(0)
    e1 = d.get_state(0)[0]
    nb = 0.25 * ((N0[:-1, :-1] + N0[1:, :-1]) + (N0[:-1, 1:] + N0[1:, 1:]))        # N at interior x-faces
    mb = 0.25 * ((M0[:-1, :-1] + M0[:-1, 1:]) + (M0[1:, :-1] + M0[1:, 1:]))        # M at interior y-faces
    out = dict(dx=dx)
    out["M"] = ((M1 - M0) / dt)[:, 1:-1], ev("rhs_M", xf, xc)[:, 1:-1]
    out["N"] = ((N1 - N0) / dt)[1:-1, :], ev("rhs_N", xc, xf)[1:-1, :]
    out["e"] = (e1 - e0) / dt, ev("rhs_e", xc, xc)
    sM, sNb = np.sign(M0[:, 1:-1]), np.sign(nb)
    out["lead_M"] = 0.5 * sM * ev("qxx", xf, xc)[:, 1:-1] + 0.5 * sNb * ev("pyy", xf, xc)[:, 1:-1]
    out["mask_M"] = (np.abs(M0[:, 1:-1]) > 1.0) & (np.abs(nb) > 1.0)
    sN, sMb = np.sign(N0[1:-1, :]), np.sign(mb)
    out["lead_N"] = 0.5 * sN * ev("qyy", xc, xf)[1:-1, :] + 0.5 * sMb * ev("rxx", xc, xf)[1:-1, :]
    out["mask_N"] = (np.abs(N0[1:-1, :]) > 1.0) & (np.abs(mb) > 1.0)
    return out


def _interior(a, m=3):
    return a[m:-m, m:-m]


def pin_consistency(lib=None, quick=False):
    """The discrete operators approximate Eqs. (1)-(3): for smooth fields the
    one-step tendencies match the analytic right-hand sides (advection,
    pressure and Manning friction together); the momentum error is first
    order in dx and its leading term is the one first-order upwinding
    predicts (which pins the upwind direction and the stencil indices); the
    continuity error is second order."""
    ns = (32, 64) if quick else (32, 64, 128)
    res = [_consistency(n, lib) for n in ns]
    for comp in ("M", "N"):
        errs = [np.abs(_interior(r[comp][0] - r[comp][1])).max() for r in res]
        scale = np.abs(_interior(res[-1][comp][1])).max()
        assert errs[-1] / scale < 0.05, f"{comp}: tendency error {errs[-1] / scale:.3f} of the rhs"
        for a, b in zip(errs, errs[1:]):
            assert 1.6 < a / b < 2.6, f"{comp}: error ratio {a / b:.2f} on halving dx (first order expected)"
        r = res[-1]
        m = _interior(r["mask_" + comp])
        lead = _interior(r["lead_" + comp])[m] * r["dx"]
        err = _interior(r[comp][0] - r[comp][1])[m]
        mis = np.abs(err - lead).max() / np.abs(lead).max()
        assert mis < (0.35 if quick else 0.2), f"{comp}: leading truncation term mismatch {mis:.2f}"
    errs = [np.abs(r["e"][0] - r["e"][1]).max() for r in res]
    for a, b in zip(errs, errs[1:]):
        assert 3.3 < a / b < 4.7, f"continuity: error ratio {a / b:.2f} (second order expected)"


# ---------------------------------------------------------------------------
def pin_dam_break(lib=None, quick=False):
    """Moving shoreline against Ritter's analytic dam break on a dry flat bed
    (no friction): the depth at the dam is (4/9) h0 and the rarefaction fan
    D = (2 c0 - (x - x0)/t)^2 / (9 g), c0 = sqrt(g h0), is reproduced with an
    error that shrinks with dx.  The wet front (D > eps) trails the exact
    eps-contour x0 + (2 c0 - 3 sqrt(g eps)) t by a bounded amount: the dry
    threshold holds back the thinnest part of the tongue (approximate pin;
    the wet/dry details are the model's own)."""
    h0, Lx, T, eps = 1.0, 400.0, 20.0, 0.01
    c0 = math.sqrt(G * h0)
    errs = []
    for n in ((100, 200, 400) if quick else (100, 200, 400, 800)):
        dx = Lx / n
        dt = 0.2 * dx / c0
        steps = int(round(T / dt))
        d = dom([lvl(np.zeros((3, n)))], dx, dt, lib=lib, manning_n=0.0, dry_eps=eps, bc=(1, 1, 1, 1))
        X = (np.arange(n) + 0.5) * dx
        x0 = Lx / 4
        d.set_eta(0, np.tile(np.where(X < x0, h0, 0.0), (3, 1)))
        d.step(steps)
        t = steps * dt
        D = d.level(0)["eta"][1]
        assert np.all(np.isfinite(D)) and np.all(D >= 0.0)
        xi = (X - x0) / t
        fan = (xi > -c0) & (xi < 0.8 * c0)
        exact = (2 * c0 - xi) ** 2 / (9 * G)
        errs.append(np.abs(D - exact)[fan].mean() / h0)
        wet = np.nonzero(D > eps)[0]
        front = X[wet[-1]] + dx / 2
        front_exp = x0 + (2 * c0 - 3 * math.sqrt(G * eps)) * t
        assert 0.7 < (front - x0) / (front_exp - x0) <= 1.02, f"front at {front:.1f} m, eps-contour at {front_exp:.1f} m"
        i0 = int(round(x0 / dx))
        assert abs(0.5 * (D[i0 - 1] + D[i0]) - 4 * h0 / 9) < 0.02, f"dam depth {0.5 * (D[i0 - 1] + D[i0]):.3f}"
    assert errs[-1] < 0.01, f"dam break fan error {errs[-1]:.3e}"
    for a, b in zip(errs, errs[1:]):
        assert a / b > 1.3, f"dam break: fan error does not shrink {errs}"


# ---------------------------------------------------------------------------
def pin_max_tracking(lib=None, quick=False):
    """The maxima equal a brute-force maximum over every stored time level,
    t = 0 included: water level on sea cells, depth h + eta on land."""
    sc = scenarios.small_nested(seed=8, nlev=2)
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
    hs = [lv["h"] for lv in sc.levels]
    best = []
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed=9, flux=0.5)):
        z = np.where(hs[k] > 0, e, hs[k] + e)
        d.set_state(k, eta=e, M=M, N=N, zmax=z)
        best.append(z)
    for _ in range(60 if quick else 400):
        d.step(1)
        for k, h in enumerate(hs):
            e = d.level(k)["eta"]
            best[k] = np.maximum(best[k], np.where(h > 0, e, h + e))
    for k in range(d.nlev):
        assert np.array_equal(d.max_inundation(k), best[k]), f"max tracking, level {k}"
    assert np.any((hs[-1] <= 0) & (best[-1] > 0.01)), "no land was inundated"


def pin_jnz_linear(lib=None, quick=False):
    """Sec. IV-C averages 3x3 child cells onto the parent: for a water level
    linear in x and y the average is the value at the parent cell's centre,
    so after the exchange the parent's ring cells carry exactly that value
    (to rounding) and no other parent cell changes."""
    dx = 900.0
    parent = lvl(np.full((17, 19), 100.0))
    cnx, cny, oi, oj = 21, 24, 4, 5
    child = lvl(np.full((cny, cnx), 100.0), parent=0, off_i=oi, off_j=oj)
    d = dom([parent, child], dx, 1.0, lib=lib)
    a, bx, by = 0.3, 2e-4, -3e-4
    lin = lambda XX, YY: a + bx * XX + by * YY
    Xc = oi * dx + (np.arange(cnx) + 0.5) * dx / 3
    Yc = oj * dx + (np.arange(cny) + 0.5) * dx / 3
    Xp = (np.arange(19) + 0.5) * dx
    Yp = (np.arange(17) + 0.5) * dx
    d.set_state(1, eta=lin(*np.meshgrid(Xc, Yc)))
    ep0 = np.full((17, 19), -0.25)
    d.set_state(0, eta=ep0)
    d.jnz(1)
    ep = d.level(0)["eta"]
    ring = np.zeros_like(ep, dtype=bool)
    fw, fh = cnx // 3, cny // 3
    ring[oj:oj + fh, oi:oi + fw] = True
    ring[oj + 1:oj + fh - 1, oi + 1:oi + fw - 1] = False
    expect = lin(*np.meshgrid(Xp, Yp))
    assert np.abs(ep[ring] - expect[ring]).max() < 1e-12, "child->parent mean is not centred on the parent cell"
    assert np.array_equal(ep[~ring], ep0[~ring]), "child->parent exchange touched cells off the ring"


def pin_open_boundary(lib=None, quick=False):
    """An open side lets a long wave leave: after a y-uniform pulse has
    crossed the open ends of a channel, less than 5 % of its amplitude is
    left; behind walls it stays."""
    nx, ny, h0, dx, dt = 200, 3, 100.0, 810.0, 5.0
    X = (np.arange(nx) + 0.5) * dx
    pulse = np.tile(1e-2 * np.exp(-((X - 100 * dx) / (6 * dx)) ** 2), (ny, 1))
    left = {}
    for name, bc in (("open", (0, 0, 1, 1)), ("wall", (1, 1, 1, 1))):
        d = dom([lvl(np.full((ny, nx), h0))], dx, dt, lib=lib, manning_n=0.0, bc=bc)
        d.set_eta(0, pulse)
        d.step(700)
        left[name] = np.abs(d.level(0)["eta"]).max() / 1e-2
    assert left["open"] < 0.05, f"open boundary reflects {left['open']:.3f}"
    assert left["wall"] > 0.3, f"walls lost the wave ({left['wall']:.3f})"


# ---------------------------------------------------------------------------
def pin_validation(lib=None, quick=False):
    """Eq. (4) and the nesting rules reject bad layouts (CFL, ratio/margin)."""
    ok = lvl(np.full((30, 30), 100.0))
    assert oracle.validate([ok], 810.0, 1.0) == oracle.OK
    deep = lvl(np.full((30, 30), 9000.0))
    assert oracle.validate([deep], 810.0, 2.0) == oracle.ECFL       # 405 < sqrt(2 g 9000) = 420
    assert oracle.validate([deep], 810.0, 1.9) == oracle.OK         # 426 >= 420
    child = lvl(np.full((27, 27), 100.0), parent=0, off_i=5, off_j=5)
    assert oracle.validate([ok, child], 810.0, 1.0) == oracle.OK
    assert oracle.validate([ok, dict(child, nx=28)], 810.0, 1.0) == oracle.ENEST
    assert oracle.validate([ok, dict(child, off_i=2)], 810.0, 1.0) == oracle.ENEST
    assert oracle.validate([ok, dict(child, off_i=19)], 810.0, 1.0) == oracle.ENEST
    deep_child = lvl(np.full((27, 27), 4000.0), parent=0, off_i=5, off_j=5)
    assert oracle.validate([ok, deep_child], 810.0, 1.0) == oracle.ECFL   # 270 < sqrt(2 g 4000) = 280


# ---------------------------------------------------------------------------
# Levels made of touching blocks (a masked level, Sec. II-A and Table 1).
OUTSIDE_DEPTH = 5000.0      # the depth given to cells outside a level: deep enough to break Eq. (4) if counted


def masked_twin(lv, pad):
    """Level lv held as a masked level: its array grown by pad parent cells
    on every side, its own cells inside, the new ones outside (with a depth
    that would change every result if the step read it)."""
    nx, ny = lv["nx"] + 6 * pad, lv["ny"] + 6 * pad
    h = np.full((ny, nx), OUTSIDE_DEPTH)
    h[3 * pad:3 * pad + lv["ny"], 3 * pad:3 * pad + lv["nx"]] = lv["h"]
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[3 * pad:3 * pad + lv["ny"], 3 * pad:3 * pad + lv["nx"]] = 1
    return dict(nx=nx, ny=ny, parent=lv["parent"], off_i=lv["off_i"] - pad, off_j=lv["off_j"] - pad, h=h, mask=mask)


def embed(a, pad3, shape, seed):
    """a placed at offset pad3 in an array of the given shape filled with noise."""
    out = np.random.default_rng(seed).uniform(-3.0, 3.0, size=shape)
    out[pad3:pad3 + a.shape[0], pad3:pad3 + a.shape[1]] = a
    return out


def pin_masked_subrect(lib=None, quick=False):
    """A masked level whose inside is a rectangle is that rectangular level:
    the middle level of a 3-level nest grown by 3 parent cells on every side
    (the new cells outside, 5000 m deep, random state on them) gives bitwise
    the plain nest's results on every level, from a source and from a random
    state, with its own child inside it; cells outside hold 0."""
    sc = scenarios.small_nested(seed=7, nlev=3)
    pad, p3 = 3, 9
    tw = masked_twin(sc.levels[1], pad)
    grand = dict(sc.levels[2], off_i=sc.levels[2]["off_i"] + p3, off_j=sc.levels[2]["off_j"] + p3)
    twin_levels = [sc.levels[0], tw, grand]
    assert oracle.validate(twin_levels, sc.dx0, sc.dt) == oracle.OK
    ox, oy = sc.level_origin(1)
    w = sc.levels[1]["nx"] * sc.level_dx(1)
    src = scenarios.Source(ox + 0.3 * w, oy + 0.4 * w, 0.3 * w, 0.2 * w, 0.4, 1.0, scenarios.GAUSS)
    for mode in ("source", "random"):
        a = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
        b = dom(twin_levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
        if mode == "source":
            a.set_source(*src.astuple())
            b.set_source(*src.astuple())
        else:
            for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed=31, flux=2.0)):
                z = np.where(sc.levels[k]["h"] > 0, e, sc.levels[k]["h"] + e)
                a.set_state(k, eta=e, M=M, N=N, zmax=z)
                if k == 1:
                    sh = (tw["ny"], tw["nx"])
                    e, z = embed(e, p3, sh, 1), embed(z, p3, sh, 2)
                    M = embed(M, p3, (sh[0], sh[1] + 1), 3)
                    N = embed(N, p3, (sh[0] + 1, sh[1]), 4)
                b.set_state(k, eta=e, M=M, N=N, zmax=z)
        n = 80 if quick else 400
        a.step(n)
        b.step(n)
        for k in range(3):
            ea, Ma, Na = a.get_state(k)
            eb, Mb, Nb = b.get_state(k)
            za, zb = a.max_inundation(k), b.max_inundation(k)
            if k == 1:
                r = slice(p3, p3 + sc.levels[1]["ny"]), slice(p3, p3 + sc.levels[1]["nx"])
                out = b.level(1)["mask"] == 0
                assert np.all(eb[out] == 0.0) and np.all(zb[out] == 0.0), f"{mode}: outside cells changed"
                eb, zb = eb[r], zb[r]
                Mb = Mb[r[0], p3:p3 + sc.levels[1]["nx"] + 1]
                Nb = Nb[p3:p3 + sc.levels[1]["ny"] + 1, r[1]]
            assert k == 2 or np.abs(Ma).max() > 1e-3, f"{mode}: level {k} at rest"
            for name, x, y in (("eta", ea, eb), ("M", Ma, Mb), ("N", Na, Nb), ("max", za, zb)):
                assert np.array_equal(x, y), \
                    f"masked rectangle, {mode}: level {k} {name} differs by {np.abs(x - y).max():.3e}"


def merge_siblings(levels, a, b):
    """Blocks a < b of one parent merged into one masked level at index a
    (their children re-parented, with offsets in the merged array)."""
    A, B = levels[a], levels[b]
    assert A["parent"] == B["parent"]
    i0, j0 = min(A["off_i"], B["off_i"]), min(A["off_j"], B["off_j"])
    i1 = max(A["off_i"] + A["nx"] // 3, B["off_i"] + B["nx"] // 3)
    j1 = max(A["off_j"] + A["ny"] // 3, B["off_j"] + B["ny"] // 3)
    nx, ny = 3 * (i1 - i0), 3 * (j1 - j0)
    h = np.full((ny, nx), OUTSIDE_DEPTH)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    shift = {}
    for q, L in ((a, A), (b, B)):
        di, dj = 3 * (L["off_i"] - i0), 3 * (L["off_j"] - j0)
        h[dj:dj + L["ny"], di:di + L["nx"]] = L["h"]
        mask[dj:dj + L["ny"], di:di + L["nx"]] = 1
        shift[q] = (di, dj)
    merged = dict(nx=nx, ny=ny, parent=A["parent"], off_i=i0, off_j=j0, h=h, mask=mask)
    out, where = [], {}
    for k, L in enumerate(levels):
        if k == b:
            continue
        where[k] = len(out)
        if k == a:
            out.append(merged)
            continue
        L = dict(L)
        if L["parent"] in (a, b):
            di, dj = shift[L["parent"]]
            L["off_i"], L["off_j"], L["parent"] = L["off_i"] + di, L["off_j"] + dj, a
        elif L["parent"] >= 0:
            L["parent"] = where[L["parent"]]
        out.append(L)
    return out, shift, where


def pin_masked_blocks(lib=None, quick=False):
    """Two blocks of one resolution held as one masked level (two covered
    rectangles apart, outside cells between them) give bitwise the results
    of the two blocks as separate levels, on every level below and above."""
    sc = scenarios.small_blocks()
    merged, shift, where = merge_siblings(sc.levels, 1, 2)
    assert oracle.validate(merged, sc.dx0, sc.dt) == oracle.OK
    a = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
    b = dom(merged, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
    a.set_source(*sc.source.astuple())
    b.set_source(*sc.source.astuple())
    n = 60 if quick else 300
    a.step(n)
    b.step(n)
    for k, L in enumerate(sc.levels):
        got = [*b.get_state(where.get(k, 1)), b.max_inundation(where.get(k, 1))]
        want = [*a.get_state(k), a.max_inundation(k)]
        if k in shift:
            di, dj = shift[k]
            ny, nx = L["ny"], L["nx"]
            got = [got[0][dj:dj + ny, di:di + nx], got[1][dj:dj + ny, di:di + nx + 1],
                   got[2][dj:dj + ny + 1, di:di + nx], got[3][dj:dj + ny, di:di + nx]]
        for name, x, y in zip(("eta", "M", "N", "max"), want, got):
            assert np.array_equal(x, y), f"merged blocks: block {k} {name} differs by {np.abs(x - y).max():.3e}"
    assert np.abs(a.get_state(6)[1]).max() > 1e-3


def pin_masked_rest(lib=None, quick=False):
    """Still water stays still bitwise on an L-shaped level of two touching
    blocks with a child across their junction, shorelines crossing the
    exchanges; cells outside hold 0."""
    sc = scenarios.small_union()
    rng = np.random.default_rng(13)
    for lv in sc.levels:
        h = lv["h"]
        lv["h"] = np.where(np.abs(h) < 2.0, rng.uniform(-0.02, 0.02, size=h.shape), h)
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc)
    before = [d.get_state(k)[0] for k in range(d.nlev)]
    d.step(200 if quick else 2000)
    for k in range(d.nlev):
        e, M, N = d.get_state(k)
        assert np.array_equal(e, before[k]) and np.all(M == 0.0) and np.all(N == 0.0), f"L-shaped rest: level {k}"
    out = oracle.level_mask(sc.levels[1]) == 0
    assert out.any() and np.all(d.get_state(1)[0][out] == 0.0)


def pin_masked_mass(lib=None, quick=False):
    """Volume is conserved across an L-shaped level of two touching blocks
    (closed root, random fluxes everywhere): the injected fluxes follow the
    covered region's boundary, including the inner corner, and carry exactly
    the parent faces' discharge."""
    sc = scenarios.small_union()
    sc.bc = (1, 1, 1, 1)
    d = dom(sc.levels, sc.dx0, sc.dt, lib=lib, bc=sc.bc, track_clip=True)
    for k, (e, M, N) in enumerate(scenarios.random_state(sc, seed=24, flux=0.5)):
        d.set_state(k, eta=e, M=M, N=N)
    d.bc_root()
    for k in range(1, d.nlev):
        d.jnq(k)
    masks = footprint_masks(sc.levels)
    v0 = _volume(d, masks)
    scale = sum(math.fsum(np.abs(d.level(k)["eta"][masks[k]]).ravel().tolist()) * d.dx[k] ** 2
                for k in range(d.nlev))
    d.step(100 if quick else 1500)
    v1 = _volume(d, masks)
    assert np.abs(d.level(1)["M"]).max() > 0.0
    assert abs(v1 - v0) <= 1e-12 * scale, f"L-shaped mass drift {abs(v1 - v0) / scale:.3e} (relative)"


def pin_masked_symmetry(lib=None, quick=False):
    """Mirror symmetry across a U-shaped level of three touching blocks:
    symmetric depth and source give results mirrored to rounding."""
    dx, dt = 810.0, 1.0
    npx, npy = 45, 33
    Xp = (np.arange(npx) + 0.5) * dx
    Yp = (np.arange(npy) + 0.5) * dx
    Lx = npx * dx

    def depth(XX, YY):
        return 90.0 - 110.0 * np.exp(-((XX - Lx / 2) / (0.15 * Lx)) ** 2) + 4.0 * np.cos(YY / 2500.0)

    XX, YY = np.meshgrid(Xp, Yp)
    child = scenarios.union_level(0, [(12, 9, 21, 4), (12, 13, 6, 8), (27, 13, 6, 8)])
    Xc = child["off_i"] * dx + (np.arange(child["nx"]) + 0.5) * dx / 3
    Yc = child["off_j"] * dx + (np.arange(child["ny"]) + 0.5) * dx / 3
    XC, YC = np.meshgrid(Xc, Yc)
    child["h"] = np.ascontiguousarray(depth(XC, YC))
    d = dom([lvl(depth(XX, YY)), child], dx, dt, lib=lib)

    def src(XX, YY):
        return 1.0 * np.exp(-((XX - Lx / 2) ** 2 + (YY - 0.75 * npy * dx) ** 2) / (2 * (5 * dx) ** 2))

    d.set_eta(0, src(XX, YY))
    d.set_eta(1, src(XC, YC))
    d.step(60 if quick else 300)
    for k in range(2):
        e, M, N = d.get_state(k)
        assert np.abs(M).max() > 1e-3
        assert np.abs(e - e[:, ::-1]).max() <= 1e-9 * max(1.0, np.abs(e).max()), f"U-shaped mirror: level {k} eta"
        assert np.abs(M + M[:, ::-1]).max() <= 1e-9 * np.abs(M).max(), f"U-shaped mirror: level {k} M"
        assert np.abs(N - N[:, ::-1]).max() <= 1e-9 * np.abs(N).max(), f"U-shaped mirror: level {k} N"


def pin_nest_locality(lib=None, quick=False):
    """The exchanges touch only the child's edge and ring: a bump in the
    middle of a child, over a parent at rest, evolves for the first steps
    (before its stencil reaches the ring blocks) bitwise like the child's
    grid alone with walls, and the parent stays bitwise at rest.  Run for a
    rectangular child and for an L-shaped level of touching blocks."""
    for shaped in (False, True):
        dx0, dt = 810.0, 0.5
        root = lvl(np.full((36, 36), 60.0))
        if shaped:
            child = scenarios.union_level(0, [(9, 9, 15, 9), (9, 18, 8, 9)])
            ci, cj = 18, 13                       # the bump's centre, child cells (in the 15x9 block)
        else:
            child = dict(nx=45, ny=45, parent=0, off_i=10, off_j=11, h=None)
            ci, cj = 22, 22
        ny, nx = child["ny"], child["nx"]
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        child["h"] = np.ascontiguousarray(40.0 + 10.0 * np.sin(ii / 5.0) * np.cos(jj / 7.0))
        rho = np.hypot(ii - ci, jj - cj) / 4.0
        bump = np.where(rho < 1.0, np.cos(0.5 * np.pi * rho) ** 2, 0.0)
        alone_lv = dict(lvl(child["h"]))
        d = dom([root, child], dx0, dt, lib=lib)
        a = dom([alone_lv], dx0 / 3.0, dt, lib=lib, bc=(1, 1, 1, 1))
        d.set_eta(1, bump)
        a.set_eta(0, np.where(oracle.level_mask(child), bump, 0.0))
        before = d.get_state(0)
        for n in range(1, 6):
            d.step(1)
            a.step(1)
            e, M, N = d.get_state(1)
            ea, Ma, Na = a.get_state(0)
            inside = oracle.level_mask(child)
            assert np.array_equal(e[inside], ea[inside]), f"locality ({'L' if shaped else 'rect'}): eta, step {n}"
            assert np.array_equal(M, Ma) and np.array_equal(N, Na), f"locality ({'L' if shaped else 'rect'}): flux, step {n}"
            for x, y in zip(d.get_state(0), before):
                assert np.array_equal(x, y), f"locality: parent moved at step {n}"
        assert np.abs(M).max() > 1e-3


def pin_masked_validation(lib=None, quick=False):
    """Masks: 0/1, constant over each 3x3 child block, covering something,
    not on the root; a child keeps 3 cells inside a masked parent; Eq. (4)
    counts only inside cells."""
    sc = scenarios.small_union()
    L = sc.levels
    assert oracle.validate(L, sc.dx0, sc.dt) == oracle.OK
    child = dict(L[1], mask=L[1]["mask"].copy())
    child["mask"][0, 0] = 1 - child["mask"][0, 0]
    assert oracle.validate([L[0], child, L[2]], sc.dx0, sc.dt) == oracle.ENEST      # not constant over a block
    child = dict(L[1], mask=np.zeros_like(L[1]["mask"]))
    assert oracle.validate([L[0], child], sc.dx0, sc.dt) == oracle.ENEST            # covers nothing
    root = dict(L[0], mask=np.ones((L[0]["ny"], L[0]["nx"]), dtype=np.uint8))
    assert oracle.validate([root] + L[1:], sc.dx0, sc.dt) == oracle.ENEST          # mask on the root
    assert oracle.validate([L[0], L[1], dict(L[2], off_i=15)], sc.dx0, sc.dt) == oracle.OK      # 3 cells of margin
    assert oracle.validate([L[0], L[1], dict(L[2], off_i=16)], sc.dx0, sc.dt) == oracle.ENEST   # 2 cells of margin
    deep = dict(L[1], h=np.where(L[1]["mask"] != 0, L[1]["h"], OUTSIDE_DEPTH))
    assert oracle.validate([L[0], deep, L[2]], sc.dx0, sc.dt) == oracle.OK


# ---------------------------------------------------------------------------
def cbrt_hard_cases(n, seed):
    """Inputs whose cube root lies within about 2^-106 of a midpoint between
    two adjacent doubles, with the correctly rounded roots: for y < y' adjacent
    (y in [0.5, 4), plus the binade edges around 1 and 2), x is the double
    nearest to m^3, m = (y + y')/2, and the nearest double to x^(1/3) is y' when
    x > m^3 and y when x < m^3 (never equal), decided on exact rationals."""
    from fractions import Fraction
    rng = np.random.default_rng(seed)
    ys = [float(v) for v in rng.uniform(0.5, 4.0, size=max(n - 4, 0))]
    ys += [1.0, 2.0, float(np.nextafter(1.0, 0.0)), float(np.nextafter(2.0, 0.0))]
    xs, want = [], []
    for y in ys[:n]:
        yu = float(np.nextafter(y, np.inf))
        m = (Fraction(y) + Fraction(yu)) / 2
        x = float(m ** 3)                              # Fraction -> nearest double
        xs.append(x)
        want.append(yu if Fraction(x) > m ** 3 else y)
    return np.array(xs), np.array(want)


def pin_cbrt_rn(lib=None, quick=False):
    """The friction term's cube root is the double nearest to the real cube
    root (correct rounding is a plain definition, so it is checked against
    arithmetic that does not come from the oracle):
    - exact cubes k^3 2^(3e) give k 2^e exactly;
    - the hardest inputs, x = the double nearest to a midpoint m^3 between two
      adjacent doubles y < y': the root then lies within about 2^-106 of m, and
      whether it is above m (answer y') or below (answer y) is read off the
      exact rational x - m^3;
    - random depths' reciprocals and log-uniform values against mpmath at 200
      bits (10^6 values, 10^5 with quick)."""
    import mpmath
    rng = np.random.default_rng(97)
    # exact cubes
    k = rng.integers(1, 1 << 17, size=2000).astype(np.float64)
    e = rng.integers(-60, 60, size=2000)
    x = np.ldexp(k ** 3, 3 * e)
    got = oracle.cbrt_rn(x, lib=lib)
    assert np.array_equal(got, np.ldexp(k, e)), "cube root of an exact cube is not exact"
    # near-midpoint inputs
    xs, want = cbrt_hard_cases(4000 if quick else 20000, seed=98)
    got = oracle.cbrt_rn(xs, lib=lib)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"near-midpoint cube roots wrong at {bad.size} of {xs.size} inputs, e.g. x={xs[bad[0]]!r}"
    # random values against mpmath
    mpmath.mp.prec = 200
    n = 100_000 if quick else 1_000_000
    depth = rng.uniform(0.01, 6000.0, size=n // 2)
    xr = np.concatenate([1.0 / depth, np.exp2(rng.uniform(-1000.0, 1000.0, size=n - n // 2))])
    got = oracle.cbrt_rn(xr, lib=lib)
    ref = np.array([float(mpmath.cbrt(mpmath.mpf(float(v)))) for v in xr])
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"cube root differs from mpmath at {bad.size} of {n} values, e.g. x={xr[bad[0]]!r}"


# ---------------------------------------------------------------------------
def _source_at(lib, x, y, src, h=1000.0):
    """The initial level that set_source gives a cell centred at (x, y), and
    its starting maximum (a 3 x 3 level whose middle cell sits there)."""
    dx = 100.0
    hh = np.full((3, 3), h)
    d = dom([lvl(hh)], dx, 0.1, lib=lib, x0=x - 1.5 * dx, y0=y - 1.5 * dx)
    d.set_source(*src)
    return d.level(0)["eta"][1, 1], d.level(0)["zmax"][1, 1]


def pin_source(lib=None, quick=False):
    """The initial sea-surface displacement follows its definition (Sec. II-A
    gives the fault model no form; the reading: a Gaussian amp exp(-rho^2/2),
    or an elliptic uplift amp cos^2(pi rho / 2) inside rho < 1, with
    rho^2 = (x'/a)^2 + (y'/b)^2 and (x', y') the offset from the centre
    rotated by theta, so a and b are the semi-axes along theta and
    theta + 90 degrees).  Checked at points placed by hand: the centre, the
    ends of both semi-axes, half-way along an axis, just inside and outside
    the ellipse; the field is unchanged when theta grows by pi; land cells
    hold eta = -h (no water) and a displacement below the ground is clipped."""
    xc, yc, a, b, th, amp = 3.0e5, 2.0e5, 5.0e4, 2.0e4, 0.4, 3.0
    ca, sa = math.cos(th), math.sin(th)
    along = lambda t: (xc + t * a * ca, yc + t * a * sa)        # t semi-axes along theta
    across = lambda t: (xc - t * b * sa, yc + t * b * ca)       # t semi-axes along theta + 90 deg
    gauss = (xc, yc, a, b, th, amp, 0)
    ell = (xc, yc, a, b, th, amp, 1)
    close = lambda v, w, tol=1e-13: abs(v - w) <= tol * abs(amp)
    for src in (gauss, ell):
        e, z = _source_at(lib, xc, yc, src)
        assert e == amp and z == amp, f"shape {src[6]}: centre {e}"
    for pt in (along(1.0), along(-1.0), across(1.0), across(-1.0)):
        e, _ = _source_at(lib, *pt, gauss)
        assert close(e, amp * math.exp(-0.5)), f"Gaussian at a semi-axis end: {e} vs {amp * math.exp(-0.5)}"
    for pt in (along(0.5), across(-0.5)):
        e, _ = _source_at(lib, *pt, ell)
        assert close(e, 0.5 * amp), f"uplift half-way along an axis: {e} vs {0.5 * amp}"
    for pt in (along(1.001), across(1.001), along(-1.001)):
        e, _ = _source_at(lib, *pt, ell)
        assert e == 0.0, f"uplift outside the ellipse: {e}"
    for pt in (along(0.999), across(0.999)):
        e, _ = _source_at(lib, *pt, ell)
        want = amp * math.cos(0.5 * math.pi * 0.999) ** 2
        assert close(e, want, 1e-9), f"uplift just inside the ellipse: {e} vs {want}"
    # off-axis point: (0.6, 0.5) semi-axes gives rho^2 = 0.61
    px, py = xc + 0.6 * a * ca - 0.5 * b * sa, yc + 0.6 * a * sa + 0.5 * b * ca
    e, _ = _source_at(lib, px, py, gauss)
    assert close(e, amp * math.exp(-0.5 * 0.61)), f"Gaussian off the axes: {e}"
    # theta + pi describes the same ellipse
    rng = np.random.default_rng(5)
    n = 24
    h = np.full((n, n), 2000.0)
    for shape in (0, 1):
        f = []
        for t in (th, th + math.pi):
            d = dom([lvl(h)], 4000.0, 1.0, lib=lib)
            d.set_source(n * 2000.0 + 1234.5, n * 2000.0 - 777.0, 3.0e4, 1.5e4, t, amp, shape)
            f.append(d.level(0)["eta"].copy())
        assert np.abs(f[0] - f[1]).max() <= 1e-12 * amp, f"shape {shape}: theta and theta + pi differ"
        assert np.abs(f[0]).max() > 0.5 * amp
    # land keeps -h even under an uplift higher than the land (amp 30 m over
    # land up to 20 m); a trough deeper than a shallow sea cell is clipped to
    # its ground
    h = rng.uniform(-20.0, 3000.0, size=(n, n))
    h[::5, ::3] = 0.5                                  # shallow sea cells
    h[n // 2 - 2:n // 2 + 2, ::2] = -5.0               # land under the middle of the source
    land = h <= 0
    for amp_k in (30.0, -2.0):
        d = dom([lvl(h)], 4000.0, 1.0, lib=lib)
        d.set_source(n * 2000.0, n * 2000.0, 4.0e4, 3.0e4, 0.0, amp_k, 1)
        e, z = d.level(0)["eta"], d.level(0)["zmax"]
        assert np.array_equal(e[land], -h[land]) and np.array_equal(z[land], np.zeros(land.sum())), "land cells"
        assert np.array_equal(z[~land], e[~land]), "sea maxima start at eta"
        assert np.all(h + e >= 0.0)
    assert np.any((h > 0) & (h + e == 0.0)), "shallow cells under the trough not clipped"


ALL = [pin_cbrt_rn, pin_source, pin_lake_at_rest, pin_closed_mass, pin_nested_mass, pin_dispersion, pin_standing_period,
       pin_wave_speed, pin_mirror_symmetry, pin_nested_symmetry, pin_friction_ode, pin_consistency,
       pin_dam_break, pin_max_tracking, pin_jnz_linear, pin_open_boundary, pin_validation, pin_masked_subrect,
       pin_masked_blocks, pin_masked_rest, pin_masked_mass, pin_masked_symmetry, pin_masked_validation,
       pin_nest_locality]
