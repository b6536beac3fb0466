"""Seeded synthetic inputs for the nested long-wave model.

This module only *describes* inputs: grid layouts, bathymetry, source
parameters and random states.  It contains none of the time-step arithmetic;
both the HIP library (through its binding) and the CPU oracle consume what it
returns.  The Kochi model of the paper (Sec. V-A, Table 1) is not available,
so its shapes are reproduced with synthetic coastlines:

* ``c1()``: one 256x256 level at 810 m, a shelf from 6000 m depth to 50 m of
  land along x plus eight seeded 200 m shoals (sigma 10 km), a 2 m Gaussian
  hump (sigma 20 km) in the centre, open sides, dt = 1 s, 1000 steps.
* ``c2(scale)``: four levels at 810/270/90/30 m, 1200x1000, 900^2, 1500^2,
  2400^2 cells (about 10 M), a seeded wavy coastline with land up to 30 m,
  dt = 0.2 s, 3600 s (18,000 steps), a 3 m elliptic uplift of 100x50 km about
  150 km offshore.  ``scale`` divides every cell count (and the length scales
  of the coast) for test-sized versions.
* ``c3(scale)``: five levels at 810/270/90/30/10 m with the cell counts of the
  paper's Table 1 (1266x1590, 1305^2, 1494^2, 3141^2, 5604^2; 47.2 M cells),
  the three finest about 40 % land, finest-level sea no deeper than 100 m,
  dt = 0.2 s, 6 h (108,000 steps).
* ``random_state``: per-level random water levels and fluxes with a wet/dry
  mix (dry land, thin films below and above the dry threshold, both flux
  signs), used to exercise every branch of one step.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

G = 9.81
GAUSS, COS2_ELLIPSE = 0, 1
BC_OPEN, BC_WALL = 0, 1


@dataclasses.dataclass
class Source:
    xc: float
    yc: float
    a: float
    b: float
    theta: float
    amp: float
    shape: int

    def astuple(self):
        return (self.xc, self.yc, self.a, self.b, self.theta, self.amp, self.shape)


@dataclasses.dataclass
class Scenario:
    name: str
    levels: list          # dicts: nx, ny, parent, off_i, off_j, h (ny, nx) float64
    dx0: float
    dt: float
    steps: int
    bc: tuple = (BC_OPEN,) * 4
    g: float = G
    manning_n: float = 0.025
    dry_eps: float = 0.01
    x0: float = 0.0
    y0: float = 0.0
    source: Source | None = None

    @property
    def cells(self) -> int:
        """Cells of all levels (inside cells only, on a masked level)."""
        return int(sum(lv["nx"] * lv["ny"] if lv.get("mask") is None else int(np.count_nonzero(lv["mask"]))
                       for lv in self.levels))

    def level_dx(self, k: int) -> float:
        dx = self.dx0
        depth = 0
        p = self.levels[k]["parent"]
        while p != -1:
            depth += 1
            p = self.levels[p]["parent"]
        for _ in range(depth):
            dx = dx / 3.0
        return dx

    def level_origin(self, k: int):
        """South-west corner of level k in metres (root origin + offsets)."""
        chain = []
        q = k
        while q != -1:
            chain.append(q)
            q = self.levels[q]["parent"]
        chain.reverse()
        ox, oy, dx = self.x0, self.y0, self.dx0
        for q in chain[1:]:
            ox = ox + self.levels[q]["off_i"] * dx
            oy = oy + self.levels[q]["off_j"] * dx
            dx = dx / 3.0
        return ox, oy

    def cell_centres(self, k: int):
        lv = self.levels[k]
        dx = self.level_dx(k)
        ox, oy = self.level_origin(k)
        x = ox + (np.arange(lv["nx"], dtype=np.float64) + 0.5) * dx
        y = oy + (np.arange(lv["ny"], dtype=np.float64) + 0.5) * dx
        return np.meshgrid(x, y)

    def oracle_kwargs(self):
        return dict(levels=self.levels, dx0=self.dx0, dt=self.dt, g=self.g, manning_n=self.manning_n,
                    dry_eps=self.dry_eps, bc=self.bc, x0=self.x0, y0=self.y0)

    def check_cfl(self):
        """Eq. (4) of the paper per level: dx/dt >= sqrt(2 g h_max)."""
        for k, lv in enumerate(self.levels):
            h = lv["h"] if lv.get("mask") is None else lv["h"][np.asarray(lv["mask"]) != 0]
            hmax = float(np.max(h))
            lim = (self.level_dx(k) / self.dt) ** 2 / (2.0 * self.g)
            assert hmax <= lim, f"{self.name}: level {k} depth {hmax:.1f} m exceeds CFL limit {lim:.1f} m"


def _level(nx, ny, parent=-1, off_i=0, off_j=0, h=None):
    return dict(nx=int(nx), ny=int(ny), parent=int(parent), off_i=int(off_i), off_j=int(off_j), h=h)


# ---------------------------------------------------------------------------
def c1(seed: int = 1) -> Scenario:
    rng = np.random.default_rng(seed)
    nx = ny = 256
    dx = 810.0
    L = nx * dx
    sc = Scenario("c1-single-256", [_level(nx, ny)], dx0=dx, dt=1.0, steps=1000)
    X, Y = sc.cell_centres(0)
    h = 6000.0 - 6050.0 * X / L
    for _ in range(8):
        cx, cy = rng.uniform(0, L, size=2)
        h = h - 200.0 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * 10e3 ** 2))
    sc.levels[0]["h"] = np.ascontiguousarray(h)
    sc.source = Source(L / 2, L / 2, 20e3, 20e3, 0.0, 2.0, GAUSS)
    sc.check_cfl()
    return sc


# ---------------------------------------------------------------------------
class _Coast:
    """A wavy north-south coastline with land to the east.

    x_c(y) = X0 + sum_k a_k sin(2 pi k y / Ly + phi_k); offshore distance
    s = x_c(y) - x; sea depth a piecewise-linear profile in s through the
    knots, plus 200 m / 10 km shoals in deep water; land rises with a slope
    up to zmax."""

    def __init__(self, rng, X0, Ly, wiggle, knots, zmax, slope, Lx, nbumps, scale):
        self.X0, self.Ly = X0, Ly
        self.a = [rng.uniform(0.0, wiggle / k) for k in range(1, 7)]
        self.phi = [rng.uniform(0.0, 2 * math.pi) for _ in range(6)]
        self.knots = knots
        self.zmax, self.slope = zmax, slope
        self.bumps = [(rng.uniform(0, max(1.0, X0 - knots[-2][0] / 2)), rng.uniform(0, Ly)) for _ in range(nbumps)]
        self.bump_sigma = 10e3 / scale

    def xc(self, y):
        out = np.full_like(y, self.X0)
        for k in range(6):
            out = out + self.a[k] * np.sin(2 * math.pi * (k + 1) * y / self.Ly + self.phi[k])
        return out

    def depth(self, X, Y):
        s = self.xc(Y) - X
        ks = np.array([k[0] for k in self.knots])
        hs = np.array([k[1] for k in self.knots])
        sea = np.interp(s, ks, hs)
        deep = sea > 500.0
        if self.bumps and deep.any():
            Xd, Yd = X[deep], Y[deep]
            bump = np.zeros_like(Xd)
            for (bx, by) in self.bumps:
                bump = bump + 200.0 * np.exp(-((Xd - bx) ** 2 + (Yd - by) ** 2) / (2.0 * self.bump_sigma ** 2))
            sd = sea[deep]
            sea = sea.copy()
            sea[deep] = sd - np.minimum(bump, sd - 500.0)
        land = -np.minimum(self.zmax, self.slope * (-s))
        return np.where(s > 0.0, sea, land)


def _nest_chain(sc: Scenario, sizes, centre_xy, land_shift):
    """Append levels of the given (nx, ny) sizes, each the child of the
    previous one, centred on centre_xy shifted landward (east) by
    land_shift[k] times the level's width."""
    for k, (nx, ny) in enumerate(sizes, start=1):
        p = k - 1
        pdx = sc.level_dx(p)
        pox, poy = sc.level_origin(p)
        fw, fh = nx // 3, ny // 3
        width = fw * pdx
        cx = centre_xy[0] + land_shift[k] * width
        cy = centre_xy[1]
        off_i = int(round((cx - pox) / pdx - fw / 2))
        off_j = int(round((cy - poy) / pdx - fh / 2))
        pn = sc.levels[p]
        off_i = max(3, min(off_i, pn["nx"] - 3 - fw))
        off_j = max(3, min(off_j, pn["ny"] - 3 - fh))
        sc.levels.append(_level(nx, ny, p, off_i, off_j))


def _fill_depths(sc: Scenario, coast: _Coast):
    for k, lv in enumerate(sc.levels):
        X, Y = sc.cell_centres(k)
        lv["h"] = np.ascontiguousarray(coast.depth(X, Y))


def c2(scale: int = 1, seed: int = 2) -> Scenario:
    s = int(scale)
    assert 1200 % s == 0 and 1000 % s == 0 and (900 // s) % 3 == 0 and (1500 // s) % 3 == 0 \
        and (2400 // s) % 3 == 0, "scale must keep every child size divisible by 3"
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 1200 // s, 1000 // s
    Lx, Ly = nx0 * dx0, ny0 * dx0
    X0 = 0.75 * Lx
    f = 1.0 / s
    coast = _Coast(rng, X0, Ly, wiggle=8e3 * f,
                   knots=[(0.0, 0.0), (20e3 * f, 100.0), (60e3 * f, 1000.0), (200e3 * f, 5000.0), (1e9, 5000.0)],
                   zmax=30.0, slope=30.0 / (6e3 * f), Lx=Lx, nbumps=6, scale=s)
    sc = Scenario(f"c2-nested4{'' if s == 1 else f'-s{s}'}", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=18000)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    _nest_chain(sc, [(900 // s, 900 // s), (1500 // s, 1500 // s), (2400 // s, 2400 // s)], (cx, cy),
                land_shift=[0.0, 0.0, 0.0, 0.0])
    _fill_depths(sc, coast)
    # 3 m elliptic uplift, 100 x 50 km, about 150 km offshore, long axis along the coast
    sc.source = Source(cx - 150e3 * f, cy, 50e3 * f, 25e3 * f, 0.5 * math.pi, 3.0, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def c3(scale: int = 1, seed: int = 3) -> Scenario:
    s = int(scale)
    sizes = [(1305, 1305), (1494, 1494), (3141, 3141), (5604, 5604)]
    assert all((n // s) % 3 == 0 and n % s == 0 for n, _ in sizes) or s == 1, \
        "scale must keep every child size divisible by 3"
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 1266 // s, 1590 // s
    Lx, Ly = nx0 * dx0, ny0 * dx0
    X0 = 0.72 * Lx
    f = 1.0 / s
    coast = _Coast(rng, X0, Ly, wiggle=5e3 * f,
                   knots=[(0.0, 0.0), (45e3 * f, 100.0), (90e3 * f, 1000.0), (250e3 * f, 5000.0), (1e9, 5000.0)],
                   zmax=30.0, slope=1.0 / 1000.0 * s, Lx=Lx, nbumps=6, scale=s)
    sc = Scenario(f"c3-nested5{'' if s == 1 else f'-s{s}'}", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=108000)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    _nest_chain(sc, [(n // s, m // s) for n, m in sizes], (cx, cy), land_shift=[0.0, 0.0, -0.1, -0.1, -0.1])
    _fill_depths(sc, coast)
    sc.source = Source(cx - 150e3 * f, cy, 50e3 * f, 25e3 * f, 0.5 * math.pi, 3.0, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def c3_nearshore(seed: int = 3) -> Scenario:
    """Configuration 3's five levels and bathymetry with the 3 m, 100 x 50 km
    uplift moved to 10 km offshore (its seaward half over the shelf, its
    landward half over the coastal plain, where it raises no water), so that
    the 30 m and 10 m levels flood within the first 600 s: a full-size
    wet/dry workload short enough for the oracle to run as a parity
    reference."""
    sc = c3(seed=seed)
    src = sc.source
    sc.name = "c3-nested5-nearshore"
    sc.source = Source(src.xc + 140e3, src.yc, src.a, src.b, src.theta, src.amp, src.shape)
    return sc


def union_level(parent, rects):
    """A level made of touching blocks of one resolution (Sec. II-A, Table 1),
    held as one array over their bounding box with an inside mask.  rects:
    (i0, j0, w, h) per block, in cells of the parent level."""
    i0 = min(r[0] for r in rects)
    j0 = min(r[1] for r in rects)
    i1 = max(r[0] + r[2] for r in rects)
    j1 = max(r[1] + r[3] for r in rects)
    mask = np.zeros((3 * (j1 - j0), 3 * (i1 - i0)), dtype=np.uint8)
    for (a, b, w, h) in rects:
        mask[3 * (b - j0):3 * (b - j0 + h), 3 * (a - i0):3 * (a - i0 + w)] = 1
    lv = _level(3 * (i1 - i0), 3 * (j1 - j0), parent, i0, j0)
    lv["mask"] = mask
    return lv


def small_union(seed: int = 23, grandchild: bool = True) -> Scenario:
    """An L-shaped level of two touching blocks over the shoreline of a small
    coast: a 54x48 root at 810 m; at 270 m an 18x9 block (parent cells) with a
    9x9 block on top of its west half, as one masked level; at 90 m a 27x27
    block that spans both 270 m blocks."""
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 54, 48
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.6 * Lx, Ly, wiggle=0.04 * Ly,
                   knots=[(0.0, 0.0), (0.1 * Lx, 20.0), (0.4 * Lx, 200.0), (1e12, 200.0)],
                   zmax=5.0, slope=5.0 / (0.05 * Lx), Lx=Lx, nbumps=0, scale=1)
    sc = Scenario("small-union", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=0)
    cx = int(round(float(coast.xc(np.array([Ly / 2]))[0]) / dx0))
    cy = ny0 // 2
    sc.levels.append(union_level(0, [(cx - 9, cy - 9, 18, 9), (cx - 9, cy, 9, 9)]))
    if grandchild:
        sc.levels.append(_level(27, 27, 1, 6, 22))     # child cells [6, 15) x [22, 31): across the junction
    _fill_depths(sc, coast)
    sc.source = Source((cx - 0.03 * nx0) * dx0, Ly / 2, 0.08 * Lx, 0.3 * Ly, 0.0, 1.5, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


# ---------------------------------------------------------------------------
def _block_tree(sc: Scenario, coast, tree):
    """Append blocks level by level.  tree: one list per finer resolution of
    (nx, ny, parent block index) entries; the children of each parent are
    stacked along y with equal gaps (at least 3 parent cells) and centred on
    the coastline in x at their own mid-height, inside the parent with at
    least 3 cells of margin."""
    for blocks in tree:
        by_parent = {}
        for (nx, ny, par) in blocks:
            by_parent.setdefault(par, []).append((nx, ny))
        for par, kids in by_parent.items():
            pn = sc.levels[par]
            pdx = sc.level_dx(par)
            pox, poy = sc.level_origin(par)
            total = sum(ny // 3 for _, ny in kids)
            gap = (pn["ny"] - total) // (len(kids) + 1)
            assert gap >= 3, f"parent block {par} too short for its children"
            y = gap
            for (nx, ny) in kids:
                fw, fh = nx // 3, ny // 3
                ymid = poy + (y + fh / 2) * pdx
                cx = float(coast.xc(np.array([ymid]))[0])
                off_i = int(round((cx - pox) / pdx - fw / 2))
                off_i = max(3, min(off_i, pn["nx"] - 3 - fw))
                sc.levels.append(_level(nx, ny, par, off_i, y))
                y += fh + gap


def c3_blocks(seed: int = 3) -> Scenario:
    """C3 with the block structure of the paper's Table 1: one root block of
    1266x1590 at 810 m; 3 blocks at 270 m, 9 at 90 m, 11 at 30 m and 60 at
    10 m (84 blocks, 47,227,698 cells; the paper: 47,211,444), every block
    inside one parent block, stacked along the seeded coast of C3."""
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 1266, 1590
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.72 * Lx, Ly, wiggle=5e3,
                   knots=[(0.0, 0.0), (45e3, 100.0), (90e3, 1000.0), (250e3, 5000.0), (1e9, 5000.0)],
                   zmax=30.0, slope=1.0 / 1000.0, Lx=Lx, nbumps=6, scale=1)
    sc = Scenario("c3-blocks84", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=108000)
    l2 = [(501, 1140, 0), (750, 756, 0), (750, 756, 0)]                         # blocks 1..3
    l3 = [(186, 1344, 1), (186, 1344, 1), (360, 690, 1)] + [(360, 690, 2)] * 3 + [(360, 690, 3)] * 3   # 4..12
    l4 = [(450, 1995, 4), (450, 1995, 4), (450, 1995, 5), (450, 1995, 5)] + [(450, 1995, p) for p in range(6, 13)]
    l5 = []
    for k, p in enumerate(range(13, 24)):                                       # 11 blocks at 30 m: 13..23
        l5 += [(540, 969, p)] * (6 if k < 5 else 5)
    _block_tree(sc, coast, [l2, l3, l4, l5])
    assert len(sc.levels) == 84
    _fill_depths(sc, coast)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    sc.source = Source(cx - 150e3, cy, 50e3, 25e3, 0.5 * math.pi, 3.0, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def _touching_chain(sc: Scenario, coast, specs):
    """Append one masked level per resolution, each the child of the last.
    specs: (rows, cols, w, h) per resolution: a grid of rows x cols touching
    blocks of w x h parent cells (3w x 3h cells of their own); each row of
    blocks is centred on the coast at its mid-height, the rows stacked along
    y without gaps, and kept 3 parent cells inside the parent's own cells."""
    for (nr, ncol, w, h) in specs:
        p = len(sc.levels) - 1
        P = sc.levels[p]
        inside = np.ones((P["ny"], P["nx"]), dtype=bool) if P.get("mask") is None else P["mask"] != 0
        if P.get("mask") is None:                       # the rectangle rule: 3 cells from the parent's edge
            inside[:3, :] = inside[-3:, :] = False
            inside[:, :3] = inside[:, -3:] = False
        pdx = sc.level_dx(p)
        pox, poy = sc.level_origin(p)
        rows_in = np.flatnonzero(inside.any(axis=1))
        span = rows_in[-1] - rows_in[0] + 1
        assert nr * h <= span - 6, f"{nr} rows of {h} parent cells do not fit in {span} rows"
        y0 = int(rows_in[0] + (span - nr * h) // 2)
        rects = []
        for r in range(nr):
            y = y0 + r * h
            band = inside[y - 3:y + h + 3]
            lo = max(int(np.flatnonzero(row)[0]) for row in band) + 3
            hi = min(int(np.flatnonzero(row)[-1]) + 1 for row in band) - 3 - ncol * w
            assert lo <= hi, f"a row of {ncol} blocks of {w} cells does not fit at rows {y}..{y + h}"
            cx = float(coast.xc(np.array([poy + (y + h / 2) * pdx]))[0])
            x = int(round((cx - pox) / pdx - ncol * w / 2))
            x = min(max(x, lo), hi)
            rects += [(x + c * w, y, w, h) for c in range(ncol)]
        sc.levels.append(union_level(p, rects))


def c3_touching_nearshore(seed: int = 3) -> Scenario:
    """The touching-block C3 layout with its uplift moved 10 km offshore, as
    in c3_nearshore, so that the 30 m and 10 m bands flood within the first
    600 s: the full-size wet/dry reference window of levels of touching
    blocks."""
    sc = c3_touching(seed=seed)
    src = sc.source
    sc.name = "c3-touching-nearshore"
    sc.source = Source(src.xc + 140e3, src.yc, src.a, src.b, src.theta, src.amp, src.shape)
    return sc


def small_touching(seed: int = 29) -> Scenario:
    """A small chain of levels of touching blocks over a seeded coast: a
    90x72 root at 810 m; at 270 m two blocks of 12x8 root cells, one above
    the other; at 90 m a 3 x 2 grid of blocks of 9x7 cells at 270 m (each a
    masked level whose rows of blocks step along the coast)."""
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 90, 72
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.6 * Lx, Ly, wiggle=0.06 * Ly,
                   knots=[(0.0, 0.0), (0.1 * Lx, 20.0), (0.4 * Lx, 200.0), (1e12, 200.0)],
                   zmax=5.0, slope=5.0 / (0.05 * Lx), Lx=Lx, nbumps=0, scale=1)
    sc = Scenario("small-touching", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=0)
    _touching_chain(sc, coast, [(2, 1, 12, 8), (3, 2, 9, 7)])
    _fill_depths(sc, coast)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    sc.source = Source(cx - 0.03 * Lx, cy, 0.08 * Lx, 0.3 * Ly, 0.0, 1.5, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def c3_touching(seed: int = 3) -> Scenario:
    """C3 with the paper's block counts (Table 1: 3, 9, 11 and 60 blocks at
    270, 90, 30 and 10 m) as touching rectangles: every resolution is one
    band of blocks that share edges, stepping along the seeded coast of C3
    (one masked level per resolution).  The root and the coast are C3's; the
    levels hold 46,983,789 cells in all (the paper: 47,211,444)."""
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 1266, 1590
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.72 * Lx, Ly, wiggle=5e3,
                   knots=[(0.0, 0.0), (45e3, 100.0), (90e3, 1000.0), (250e3, 5000.0), (1e9, 5000.0)],
                   zmax=30.0, slope=1.0 / 1000.0, Lx=Lx, nbumps=6, scale=1)
    sc = Scenario("c3-touching", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=108000)
    _touching_chain(sc, coast, [(3, 1, 67, 77),        # 270 m: 3 blocks of 201 x 231
                                (9, 1, 140, 76),       # 90 m: 9 blocks of 420 x 228
                                (11, 1, 294, 186),     # 30 m: 11 blocks of 882 x 558
                                (12, 5, 140, 510)])    # 10 m: 60 blocks of 420 x 1530
    _fill_depths(sc, coast)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    sc.source = Source(cx - 150e3, cy, 50e3, 25e3, 0.5 * math.pi, 3.0, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def small_blocks(seed: int = 21) -> Scenario:
    """A small multi-block nest for step-level tests: a 90x96 root at 810 m,
    2 blocks at 270 m, 3 at 90 m (two in one parent) and 2 at 30 m, with a
    1.5 m uplift across the shoreline."""
    rng = np.random.default_rng(seed)
    dx0 = 810.0
    nx0, ny0 = 90, 96
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.6 * Lx, Ly, wiggle=0.03 * Ly,
                   knots=[(0.0, 0.0), (0.1 * Lx, 20.0), (0.4 * Lx, 200.0), (1e12, 200.0)],
                   zmax=5.0, slope=5.0 / (0.05 * Lx), Lx=Lx, nbumps=0, scale=1)
    sc = Scenario("small-blocks", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=0)
    _block_tree(sc, coast, [[(45, 108, 0), (45, 90, 0)],
                            [(27, 36, 1), (27, 45, 1), (36, 27, 2)],
                            [(27, 27, 3), (18, 27, 5)]])
    _fill_depths(sc, coast)
    # a near-field uplift across the shoreline, so the finest blocks flood within a few hundred steps
    cx = float(coast.xc(np.array([Ly / 2]))[0])
    sc.source = Source(cx - 0.02 * Lx, Ly / 2, 0.08 * Lx, 0.45 * Ly, 0.0, 1.5, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


# ---------------------------------------------------------------------------
def _single(seed: int, n: int, amp: float) -> Scenario:
    """One level of n x n cells at 810 m over a C1-style shelf (6000 m deep in
    the west, 50 m of land in the east, 8 shoals), dt = 1 s, with an elliptic
    uplift of amplitude amp in the deep half."""
    rng = np.random.default_rng(seed)
    dx = 810.0
    L = n * dx
    sc = Scenario(f"single-{n}", [_level(n, n)], dx0=dx, dt=1.0, steps=0)
    X, Y = sc.cell_centres(0)
    h = 6000.0 - 6050.0 * X / L
    for _ in range(8):
        cx, cy = rng.uniform(0, L, size=2)
        h = h - 200.0 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * 10e3 ** 2))
    sc.levels[0]["h"] = np.ascontiguousarray(h)
    xc, yc = rng.uniform(0.15 * L, 0.55 * L), rng.uniform(0.2 * L, 0.8 * L)
    sc.source = Source(xc, yc, 50e3, 25e3, rng.uniform(0, math.pi), amp, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def _nest3(seed: int, cells: float, amp: float) -> Scenario:
    """Three nested levels (810/270/90 m) in the proportions of the first
    three C2 levels (1200x1000, 900^2, 1500^2), scaled to about `cells`
    cells, over a seeded wavy coast, dt = 0.2 s, elliptic uplift of amplitude
    amp about 150 km (scaled) offshore."""
    rng = np.random.default_rng(seed)
    f = math.sqrt(cells / (1200 * 1000 + 900 ** 2 + 1500 ** 2))
    dx0 = 810.0
    nx0, ny0 = int(round(1200 * f)), int(round(1000 * f))
    n2 = 3 * int(round(300 * f))
    n3 = 3 * int(round(500 * f))
    Lx, Ly = nx0 * dx0, ny0 * dx0
    X0 = 0.75 * Lx
    coast = _Coast(rng, X0, Ly, wiggle=8e3 * f,
                   knots=[(0.0, 0.0), (20e3 * f, 100.0), (60e3 * f, 1000.0), (200e3 * f, 5000.0), (1e9, 5000.0)],
                   zmax=30.0, slope=30.0 / (6e3 * f), Lx=Lx, nbumps=6, scale=1.0 / f)
    sc = Scenario(f"nest3-{nx0 * ny0 + n2 * n2 + n3 * n3}", [_level(nx0, ny0)], dx0=dx0, dt=0.2, steps=0)
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    _nest_chain(sc, [(n2, n2), (n3, n3)], (cx, cy), land_shift=[0.0, 0.0, 0.0])
    _fill_depths(sc, coast)
    sc.source = Source(cx - 150e3 * f, cy + rng.uniform(-0.2, 0.2) * Ly, 50e3 * f, 25e3 * f,
                       0.5 * math.pi + rng.uniform(-0.3, 0.3), amp, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def c4(count: int = 48, seed: int = 4000):
    """The batched ensemble: `count` uneven scenarios, member s seeded with
    seed + s.  Even members: one level of n^2 cells, n log-uniform in
    [256, 2048]; odd members: three nested levels of 1 M to 8 M cells
    (log-uniform).  Uplift amplitudes uniform in [0.5, 5] m."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed + s)
        amp = float(rng.uniform(0.5, 5.0))
        if s % 2 == 0:
            n = int(round(256 * 2.0 ** (3.0 * rng.uniform()) / 4)) * 4
            sc = _single(seed + s, n, amp)
        else:
            sc = _nest3(seed + s, 1e6 * 8.0 ** rng.uniform(), amp)
        sc.name = f"c4-{s:02d}-{sc.name}"
        out.append(sc)
    return out


def c5_sites():
    """The forecast-serving site database: six nested domains of 1 M to 47 M
    cells (three-level nests of about 1, 2.5 and 6 M cells, C2, a 20 M
    three-level nest and C3)."""
    return [_nest3(5001, 1.0e6, 1.0), _nest3(5002, 2.5e6, 1.0), _nest3(5003, 6.0e6, 1.0), c2(),
            _nest3(5004, 2.0e7, 1.0), c3()]


def c5_requests(sites, count: int = 24, seed: int = 5000, rate_per_min: float = 2.0, time_scale: float = 30.0):
    """Poisson arrivals (mean rate_per_min requests per minute) of forecast
    requests: a site drawn uniformly, a simulated duration uniform in 1-6 h,
    an uplift of 0.5-5 m shifted around the site's source.  time_scale
    compresses both the arrival clock and the durations by the same factor
    (30: 2 requests per minute become 1 per second, 1-6 h become 2-12 min),
    so a serving run fits in a bench.  Returns (site index, source tuple,
    steps, arrival seconds) per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(60.0 / rate_per_min) / time_scale
        k = int(rng.integers(len(sites)))
        sc = sites[k]
        hours = rng.uniform(1.0, 6.0)
        steps = max(1, int(round(hours * 3600.0 / time_scale / sc.dt)))
        s0 = sc.source
        Ly = sc.levels[0]["ny"] * sc.dx0
        src = (s0.xc + rng.uniform(-0.05, 0.05) * Ly, s0.yc + rng.uniform(-0.15, 0.15) * Ly, s0.a, s0.b,
               s0.theta + rng.uniform(-0.3, 0.3), float(rng.uniform(0.5, 5.0)), s0.shape)
        out.append((k, src, steps, t))
    return out


# ---------------------------------------------------------------------------
def small_nested(seed: int = 7, nlev: int = 3, base=(36, 30), child=(27, 27), dx0=810.0, dt=0.2,
                 bc=(BC_OPEN,) * 4) -> Scenario:
    """A small chain of nests over a random coast, for step-level tests.
    base: root cells; child: cells of every child (divisible by 3)."""
    rng = np.random.default_rng(seed)
    nx0, ny0 = base
    Lx, Ly = nx0 * dx0, ny0 * dx0
    coast = _Coast(rng, 0.6 * Lx, Ly, wiggle=0.05 * Ly,
                   knots=[(0.0, 0.0), (0.1 * Lx, 20.0), (0.4 * Lx, 200.0), (1e12, 200.0)],
                   zmax=5.0, slope=5.0 / (0.05 * Lx), Lx=Lx, nbumps=0, scale=1)
    sc = Scenario(f"small-nested{nlev}", [_level(nx0, ny0)], dx0=dx0, dt=dt, steps=0, bc=tuple(bc))
    cy = Ly / 2
    cx = float(coast.xc(np.array([cy]))[0])
    _nest_chain(sc, [child] * (nlev - 1), (cx, cy), land_shift=[0.0] * nlev)
    _fill_depths(sc, coast)
    sc.source = Source(cx - 0.3 * Lx, cy, 0.1 * Lx, 0.05 * Ly, 0.5 * math.pi, 1.0, COS2_ELLIPSE)
    sc.check_cfl()
    return sc


def inland_nest(seed: int = 31) -> Scenario:
    """A nest wholly on dry land, for tests of tile skipping at nest
    boundaries: a 120x150 root of 90 m cells with a 10 m deep sea south of an
    east-west coast (row 25) and land 0.3-0.6 m high rising northwards with
    seeded 0.4 m bumps; a child of 30 m cells (footprint columns 30-89, rows
    58-87) holding a grandchild of 10 m cells, and a second child beside it
    (columns 93-113), dt = 0.1 s.  The nest
    stays dry until water crosses its edges.  `dam` holds, per level, the
    land cells that start under water (dam_state): a block of water behind
    the coast (rows 28-49 of the root), south of the child."""
    rng = np.random.default_rng(seed)
    dx0 = 90.0
    nx0, ny0 = 120, 150
    sc = Scenario("inland-nest", [_level(nx0, ny0), _level(180, 90, 0, 30, 58), _level(180, 90, 1, 60, 15),
                                  _level(63, 90, 0, 93, 58)], dx0=dx0, dt=0.1, steps=0)
    Ly = ny0 * dx0
    yc = 25 * dx0
    bumps = [(rng.uniform(0, nx0 * dx0), rng.uniform(yc, Ly)) for _ in range(8)]
    sc.dam = []
    for k, lv in enumerate(sc.levels):
        X, Y = sc.cell_centres(k)
        ground = 0.3 + 0.3 * (Y - yc) / (Ly - yc)
        for bx, by in bumps:
            ground = ground + 0.4 * np.exp(-((X - bx) ** 2 + (Y - by) ** 2) / (2.0 * 400.0 ** 2))
        lv["h"] = np.ascontiguousarray(np.where(Y < yc, 10.0, -ground))
        sc.dam.append((Y >= 28 * dx0) & (Y < 50 * dx0))
    sc.check_cfl()
    return sc


def dam_state(sc: Scenario, level: int, level_of_water: float = 5.0):
    """(eta, M, N) of a level at rest with the cells of sc.dam[level] under
    the given water level (dry land elsewhere, sea at 0)."""
    h = sc.levels[level]["h"]
    eta = np.where(h > 0, 0.0, -h)
    eta = np.where(sc.dam[level], level_of_water, eta)
    ny, nx = h.shape
    return (np.ascontiguousarray(eta), np.zeros((ny, nx + 1)), np.zeros((ny + 1, nx)))


def random_state(sc: Scenario, seed: int, flux: float = 5.0):
    """Random (eta, M, N) per level exercising every branch of one step.

    Sea cells: eta ~ U(-1, 1) (clipped to the ground); land cells: half dry
    (eta = -h), half covered by a film of depth U(0, 0.05) m (below and above
    the 0.01 m dry threshold).  Fluxes ~ U(-flux, flux) on every face,
    including faces between dry cells."""
    rng = np.random.default_rng(seed)
    out = []
    for lv in sc.levels:
        h = lv["h"]
        ny, nx = h.shape
        eta = rng.uniform(-1.0, 1.0, size=(ny, nx))
        film = rng.uniform(0.0, 0.05, size=(ny, nx))
        dry = rng.uniform(size=(ny, nx)) < 0.5
        eta = np.where(h > 0, eta, np.where(dry, -h, -h + film))
        eta = np.where(h + eta < 0, -h, eta)
        M = rng.uniform(-flux, flux, size=(ny, nx + 1))
        N = rng.uniform(-flux, flux, size=(ny + 1, nx))
        out.append((np.ascontiguousarray(eta), np.ascontiguousarray(M), np.ascontiguousarray(N)))
    return out
