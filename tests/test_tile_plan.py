"""The fused kernel's tile plan on the host: static tile bits and the coupled
tiles that decide when a tile near a nest boundary may be skipped.

A tile is skipped only when every input of its step stayed unchanged over
the last two steps.  Its 3x3 neighbourhood on its own level covers the
inputs written on that level; inputs written on another level (the edge
fluxes a parent injects into a child, the child blocks a parent's ring means
read, Sec. IV-C) must come from its coupled tiles.  These tests derive, by
brute force over every cell and face a tile's step reads, the set of tiles
that write those inputs, and check that the plan's lists hold all of them,
at several tile heights, on nests with one and several children per level.
"""
import ctypes

import numpy as np
import pytest

import scenarios

TW = 60
TI_PINNED, TI_CHILD, TI_EDGE, TI_DEPS = 0x1, 0x2, 0x4, 0x8


def plan(sc, th):
    from paper_2408_07609_amd import rti
    fn = rti.LIB.rti_plan_tiles_for_test
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(rti.rti_domain_desc), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                   ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p]
    desc, keep = rti.make_desc(sc.levels, sc.dx0, sc.dt)
    nt, nd = ctypes.c_int32(), ctypes.c_int32()
    assert fn(ctypes.byref(desc), th, ctypes.byref(nt), ctypes.byref(nd), None, None, None, None, None) == 0
    tinfo = np.zeros(nt.value, np.uint8)
    tlev = np.zeros(nt.value, np.uint8)
    off = np.zeros(nt.value + 1, np.int32)
    dep = np.zeros(max(nd.value, 1), np.int32)
    cmask = np.zeros(nt.value, np.uint32)
    assert fn(ctypes.byref(desc), th, ctypes.byref(nt), ctypes.byref(nd), tinfo.ctypes.data, tlev.ctypes.data,
              off.ctypes.data, dep.ctypes.data, cmask.ctypes.data) == 0
    plan.cmask = cmask
    return tinfo, tlev, off, dep[:nd.value]


class Grid:
    """Tile numbering of the plan: levels in order, row-major tiles of 60
    columns by th rows; a tile owns the cells and the left / bottom faces of
    its columns and rows.  The root's last tile column / row also owns the
    faces nx, ny (open sides); a child's faces nx, ny are the parent's to
    write, so its grid covers only its cells."""

    def __init__(self, sc, th):
        self.th, self.lv, self.base = th, [], []
        n = 0
        for k, L in enumerate(sc.levels):
            ny, nx = L["h"].shape
            f = 1 if k == 0 else 0
            tx, ty = (nx + f + TW - 1) // TW, (ny + f + th - 1) // th
            cov = None if L.get("mask") is None else np.asarray(L["mask"]).reshape(ny, nx)[::3, ::3] != 0
            self.lv.append(dict(nx=nx, ny=ny, tx=tx, ty=ty, parent=L["parent"], oi=L["off_i"], oj=L["off_j"], cov=cov))
            self.base.append(n)
            n += tx * ty
        self.ntiles = n

    def tile(self, k, i, j):
        """The tile that writes cell / left face / bottom face (i, j) of level k."""
        L = self.lv[k]
        top = 0 if k > 0 else 1          # a child's faces nx, ny are not its own to write
        assert 0 <= i <= L["nx"] - 1 + top and 0 <= j <= L["ny"] - 1 + top, (k, i, j)
        return self.base[k] + (j // self.th) * L["tx"] + i // TW

    def children(self, l):
        return [k for k, L in enumerate(self.lv) if L["parent"] == l]

    def covers(self, k, I, J):
        """Does level k cover parent cell (I, J) of its footprint?"""
        C = self.lv[k]
        if not (0 <= I < C["nx"] // 3 and 0 <= J < C["ny"] // 3):
            return False
        return C["cov"] is None or bool(C["cov"][J, I])

    def ring(self, k, I, J):
        """Ring cell of child k (Sec. IV-C): covered, with an uncovered 8-neighbour."""
        return self.covers(k, I, J) and not all(self.covers(k, I + a, J + b) for a in (-1, 0, 1) for b in (-1, 0, 1))

    def xface_injected(self, k, fi, jj):
        """Is child x-face (fi, jj) of level k injected by its parent?"""
        return fi % 3 == 0 and self.covers(k, fi // 3 - 1, jj // 3) != self.covers(k, fi // 3, jj // 3)

    def yface_injected(self, k, ii, fj):
        return fj % 3 == 0 and self.covers(k, ii // 3, fj // 3 - 1) != self.covers(k, ii // 3, fj // 3)


def required(G, l, tx, ty):
    """(own-level writers, other-level writers, reads ring, reads injected
    faces) of the inputs of tile (tx, ty) of level l, from the fused kernel's
    access pattern: lanes c = x0-2 .. x0+61, rows t = y0-2 .. min(y0+th, ny)
    of new water levels (each with the ring mean of its child blocks where it
    is a ring cell), x-faces of columns up to x0+62 and y-faces of rows up to
    min(y0+th, ny)+1."""
    L, th = G.lv[l], G.th
    nx, ny = L["nx"], L["ny"]
    x0, y0 = tx * TW, ty * th
    t1 = min(y0 + th, ny + 1)
    own, other = set(), set()
    ring = inj = False
    cols = range(max(x0 - 2, 0), min(x0 + 61, nx - 1) + 1)
    rows = range(max(y0 - 2, 0), min(t1, ny - 1) + 1)
    top = 1 if l == 0 else 0             # a child's faces nx, ny come from the parent (below)
    for i in range(max(x0 - 2, 0), min(x0 + 62, nx - 1 + top) + 1):
        for j in range(max(y0 - 2, 0), min(t1 + 1, ny - 1 + top) + 1):
            own.add(G.tile(l, i, j))
    for k in G.children(l):
        C = G.lv[k]
        fw, fh = C["nx"] // 3, C["ny"] // 3
        for c in cols:
            I = c - C["oi"]
            if not 0 <= I < fw:
                continue
            for t in rows:
                J = t - C["oj"]
                if not 0 <= J < fh or not G.ring(k, I, J):
                    continue
                ring = True
                for jj in range(3 * J, 3 * J + 3):
                    for ii in range(3 * I, 3 * I + 3):
                        other.add(G.tile(k, ii, jj))                 # eta, h of the child cell
                        for fi in (ii, ii + 1):                      # its x-faces
                            if G.xface_injected(k, fi, jj):
                                own.add(G.tile(l, C["oi"] + fi // 3, C["oj"] + jj // 3))   # injected by this level
                            else:
                                other.add(G.tile(k, fi, jj))
                        for fj in (jj, jj + 1):                      # its y-faces
                            if G.yface_injected(k, ii, fj):
                                own.add(G.tile(l, C["oi"] + ii // 3, C["oj"] + fj // 3))
                            else:
                                other.add(G.tile(k, ii, fj))
    if l > 0:
        p = L["parent"]
        for i in range(max(x0 - 2, 0), min(x0 + 62, nx) + 1):
            for j in range(max(y0 - 2, 0), min(t1, ny - 1) + 1):
                if G.xface_injected(l, i, j):
                    inj = True
                    other.add(G.tile(p, L["oi"] + i // 3, L["oj"] + j // 3))
        for j in range(max(y0 - 2, 0), min(t1 + 1, ny) + 1):
            for i in range(max(x0 - 2, 0), min(x0 + 61, nx - 1) + 1):
                if G.yface_injected(l, i, j):
                    inj = True
                    other.add(G.tile(p, L["oi"] + i // 3, L["oj"] + j // 3))
    return own, other, ring, inj


def nest_cases():
    smallest = scenarios.Scenario("smallest-nest", [dict(nx=15, ny=15, parent=-1, off_i=0, off_j=0, h=None),
                                                    dict(nx=9, ny=9, parent=0, off_i=6, off_j=6, h=None)],
                                  dx0=810.0, dt=0.2, steps=0)
    for k in range(2):
        smallest.levels[k]["h"] = np.ones((smallest.levels[k]["ny"], smallest.levels[k]["nx"]))
    return {
        "small_nested3": scenarios.small_nested(seed=7, nlev=3),
        "wide_child": scenarios.small_nested(seed=11, nlev=2, base=(150, 72), child=(240, 54)),
        "small_blocks": scenarios.small_blocks(),
        "inland_nest": scenarios.inland_nest(),
        "smallest": smallest,
    }


def random_nest(seed):
    """A random layout obeying the nesting rules: a root of 30-200 by 20-120
    cells, 1-3 children side by side (3 cells apart, 3 from the parent's
    edge), sometimes a grandchild; depths do not matter to the plan."""
    rng = np.random.default_rng(seed)
    nx0, ny0 = int(rng.integers(30, 201)), int(rng.integers(20, 121))
    levels = [dict(nx=nx0, ny=ny0, parent=-1, off_i=0, off_j=0)]

    def place(p, n):
        P = levels[p]
        x = 3
        for _ in range(n):
            fw = int(rng.integers(3, max(4, (P["nx"] - 6) // n)))
            fh = int(rng.integers(3, P["ny"] - 5))
            if x + fw > P["nx"] - 3:
                break
            oj = int(rng.integers(3, P["ny"] - 3 - fh + 1))
            levels.append(dict(nx=3 * fw, ny=3 * fh, parent=p, off_i=x, off_j=oj))
            x += fw + 3 + int(rng.integers(0, 4))
    place(0, int(rng.integers(1, 4)))
    if rng.uniform() < 0.6 and levels[1]["nx"] >= 15 and levels[1]["ny"] >= 15:
        place(1, int(rng.integers(1, 3)))
    for L in levels:
        L["h"] = np.ones((L["ny"], L["nx"]))
    return scenarios.Scenario(f"random-{seed}", levels, dx0=810.0, dt=0.2, steps=0)


def aligned_nest(d):
    """Footprint edges placed at d cells from a tile boundary of the parent
    (column 60, rows that are multiples of 4 to 7): child A ends at column
    60 + d and starts at row 12 + d, child B starts at column 64 + d + 3 and
    ends at row 36 + d; A holds a grandchild whose edges sit at d from A's own
    tile boundaries."""
    levels = [dict(nx=150, ny=66, parent=-1, off_i=0, off_j=0)]
    a0, a1 = 24, 60 + d                       # A: columns a0 .. a1, rows 12 + d .. 40
    levels.append(dict(nx=3 * (a1 - a0 + 1), ny=3 * (40 - 12 - d + 1), parent=0, off_i=a0, off_j=12 + d))
    b0 = a1 + 4 + 3
    levels.append(dict(nx=3 * (140 - b0 + 1), ny=3 * (36 + d - 6 + 1), parent=0, off_i=b0, off_j=6))
    A = levels[1]
    g0 = max(3, 20 + d)
    levels.append(dict(nx=3 * min(60 + d - g0, A["nx"] - 3 - g0), ny=3 * 12, parent=1, off_i=g0, off_j=4 + (d % 4)))
    for L in levels:
        L["h"] = np.ones((L["ny"], L["nx"]))
    return scenarios.Scenario(f"aligned{d:+d}", levels, dx0=810.0, dt=0.2, steps=0)


@pytest.mark.parametrize("d", range(-5, 6))
def test_coupled_tiles_at_tile_boundaries(d):
    sc = aligned_nest(d)
    for th in (4, 5, 6, 7):
        check_plan(sc, th, sc.name)


def test_coupled_tiles_with_more_than_32_children():
    from test_gpu_blocks import many_children
    sc = many_children()
    for th in (4, 6, 12):
        check_plan(sc, th, sc.name)


@pytest.mark.parametrize("name", ["small_nested3", "wide_child", "small_blocks", "inland_nest", "smallest"])
@pytest.mark.parametrize("th", [4, 6, 13, 64])
def test_coupled_tiles_cover_every_writer(name, th):
    check_plan(nest_cases()[name], th, name)


@pytest.mark.parametrize("seed", range(24))
def test_coupled_tiles_random_layouts(seed):
    sc = random_nest(seed)
    for th in (4, 5, 7, 9):
        check_plan(sc, th, sc.name)


def check_plan(sc, th, name):
    tinfo, tlev, off, dep = plan(sc, th)
    G = Grid(sc, th)
    assert len(tinfo) == G.ntiles
    assert not (tinfo & TI_PINNED).any(), "a coupled-tile list did not fit its reservation"
    assert (np.diff(off) >= 0).all() and off[0] == 0 and off[-1] == len(dep)
    # the kernels index the flag array with these entries directly
    assert ((dep >= 0) & (dep < G.ntiles)).all(), "a coupled-tile entry lies outside the tile table"
    n_dep_tiles = 0
    for l, L in enumerate(G.lv):
        for ty in range(L["ty"]):
            for tx in range(L["tx"]):
                g = G.base[l] + ty * L["tx"] + tx
                assert tlev[g] == l
                lst = dep[off[g]:off[g + 1]]
                assert (np.diff(lst) > 0).all() and all(tlev[d] != l for d in lst)
                assert bool(tinfo[g] & TI_DEPS) == (len(lst) > 0)
                n_dep_tiles += len(lst) > 0
                own, other, ring, inj = required(G, l, tx, ty)
                if ring:
                    assert tinfo[g] & TI_CHILD, f"tile {g} reads ring means but is not marked"
                if inj:
                    assert tinfo[g] & TI_EDGE, f"tile {g} reads injected faces but is not marked"
                nb = {G.base[l] + y * L["tx"] + x for y in range(ty - 1, ty + 2) for x in range(tx - 1, tx + 2)
                      if 0 <= x < L["tx"] and 0 <= y < L["ty"]}
                assert own <= nb, f"tile {g}: own-level inputs outside the 3x3 neighbourhood: {sorted(own - nb)}"
                if tinfo[g] & TI_CHILD:
                    # the child mask holds every child whose edge faces lie in the tile's output
                    for q, k in enumerate(G.children(l)[:32]):
                        C = G.lv[k]
                        if C["cov"] is not None:
                            assert not plan.cmask[g] >> q & 1, f"tile {g}: masked child {k} in the mask"
                            continue              # its boundary is injected after the launch, from a list
                        fw, fh = C["nx"] // 3, C["ny"] // 3
                        ox = range(tx * TW, tx * TW + TW)
                        oy = range(ty * th, ty * th + th)
                        hit = any(c in ox for c in (C["oi"], C["oi"] + fw)) and any(C["oj"] <= r < C["oj"] + fh for r in oy) \
                            or any(r in oy for r in (C["oj"], C["oj"] + fh)) and any(C["oi"] <= c < C["oi"] + fw for c in ox)
                        if hit:
                            assert plan.cmask[g] >> q & 1, f"tile {g}: child {k} injects here but is not in the mask"
                missing = other - set(lst.tolist())
                assert not missing, f"{name} th={th} tile {g} (level {l}, {tx},{ty}): writers {sorted(missing)} not coupled"
    assert n_dep_tiles > 0


def masked_cases():
    import pins
    merged, _, _ = pins.merge_siblings(scenarios.small_blocks().levels, 1, 2)
    u = scenarios.Scenario("u-shape", [dict(nx=45, ny=33, parent=-1, off_i=0, off_j=0, h=np.ones((33, 45)))],
                           dx0=810.0, dt=0.2, steps=0)
    u.levels.append(scenarios.union_level(0, [(12, 9, 21, 4), (12, 13, 6, 8), (27, 13, 6, 8)]))
    u.levels[1]["h"] = np.ones((u.levels[1]["ny"], u.levels[1]["nx"]))
    return {
        "small_union": scenarios.small_union(),
        "merged_blocks": scenarios.Scenario("merged", merged, dx0=810.0, dt=0.2, steps=0),
        "u_shape": u,
    }


def random_union(seed):
    """A random level of 2-4 touching blocks (a staircase of rectangles, each
    row of blocks shifted in x from the one below, still sharing an edge with
    it) in a random root, sometimes with a child inside one block; depths do
    not matter to the plan."""
    rng = np.random.default_rng(seed)
    nx0, ny0 = int(rng.integers(80, 221)), int(rng.integers(60, 161))
    root = dict(nx=nx0, ny=ny0, parent=-1, off_i=0, off_j=0, h=np.ones((ny0, nx0)))
    rects, y, x = [], 3, int(rng.integers(3, nx0 // 3))
    for _ in range(int(rng.integers(2, 5))):
        w, hgt = int(rng.integers(8, 31)), int(rng.integers(4, 16))
        if y + hgt > ny0 - 3 or x + w > nx0 - 3:
            break
        rects.append((x, y, w, hgt))
        y += hgt
        x = max(3, min(nx0 - 3 - w, x + int(rng.integers(-w + 1, w))))
    if len(rects) < 2:
        rects = [(3, 3, 8, 4), (5, 7, 8, 4)]
    lv = scenarios.union_level(0, rects)
    lv["h"] = np.ones((lv["ny"], lv["nx"]))
    levels = [root, lv]
    big = max(rects, key=lambda r: r[2] * r[3])
    if big[2] >= 9 and big[3] >= 9 and rng.uniform() < 0.7:
        ci, cj = 3 * (big[0] - lv["off_i"]) + 3, 3 * (big[1] - lv["off_j"]) + 3
        levels.append(dict(nx=9 * ((big[2] - 2) // 3), ny=9 * ((big[3] - 2) // 3), parent=1, off_i=ci, off_j=cj,
                           h=None))
        levels[-1]["h"] = np.ones((levels[-1]["ny"], levels[-1]["nx"]))
    return scenarios.Scenario(f"random-union-{seed}", levels, dx0=810.0, dt=0.2, steps=0)


@pytest.mark.parametrize("seed", range(16))
def test_coupled_tiles_random_masked_levels(seed):
    import oracle
    sc = random_union(seed)
    if oracle.validate(sc.levels, sc.dx0, sc.dt) != oracle.OK:      # a child too near the outside: drop it
        sc.levels = sc.levels[:2]
    assert oracle.validate(sc.levels, sc.dx0, sc.dt) == oracle.OK
    for th in (4, 5, 9):
        check_plan(sc, th, sc.name)


@pytest.mark.parametrize("name", ["small_union", "merged_blocks", "u_shape"])
@pytest.mark.parametrize("th", [4, 5, 7, 12])
def test_coupled_tiles_masked_levels(name, th):
    """Levels of touching blocks (masks): ring means at inner corners, and
    boundary faces inside the rectangle injected from the parent."""
    check_plan(masked_cases()[name], th, name)


def test_root_only_has_no_coupled_tiles():
    sc = scenarios.small_nested(seed=5, nlev=1, base=(150, 40))
    tinfo, tlev, off, dep = plan(sc, 6)
    assert len(dep) == 0 and not (tinfo & (TI_DEPS | TI_PINNED | TI_CHILD)).any()
