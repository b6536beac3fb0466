"""CPU FP64 oracle for the nested long-wave time step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
binding) never does, and this package imports nothing from the product.

The arithmetic lives in ``rti_oracle.c`` (plain C, binary64, no fused
multiply-add); this module only builds it with gcc, marshals numpy arrays and
runs the steps in the paper's order (arXiv 2408.07609, Sec. IV-A: mass,
child->parent level, momentum, parent->child flux, output maxima).
The validation rules follow Sec. II-A: the CFL bound of Eq. (4) per level and
the 3:1 inclusive nesting.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rti_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "librti_oracle.so")
_LOCK = threading.Lock()
_LIB = None

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
          "-D_DEFAULT_SOURCE"]


def build(force: bool = False) -> str:
    """Compile rti_oracle.c with gcc into oracle/_build/librti_oracle.so."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Level(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("parent", ctypes.c_int32),
                ("off_i", ctypes.c_int32), ("off_j", ctypes.c_int32),
                ("dx", ctypes.c_double), ("ox", ctypes.c_double), ("oy", ctypes.c_double),
                ("h", ctypes.c_void_p), ("eta", ctypes.c_void_p), ("M", ctypes.c_void_p),
                ("N", ctypes.c_void_p), ("zmax", ctypes.c_void_p), ("M2", ctypes.c_void_p),
                ("N2", ctypes.c_void_p), ("clip", ctypes.c_void_p), ("mask", ctypes.c_void_p)]


class _Domain(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int32), ("bc", ctypes.c_int32 * 4), ("lv", ctypes.POINTER(_Level)),
                ("dt", ctypes.c_double), ("g", ctypes.c_double), ("manning", ctypes.c_double),
                ("eps", ctypes.c_double), ("steps", ctypes.c_int64)]


def _bind(L):
    P = ctypes.POINTER(_Domain)
    for name in ("ora_mass", "ora_jnz", "ora_momentum", "ora_max"):
        getattr(L, name).argtypes = [P, ctypes.c_int]
        getattr(L, name).restype = None
    L.ora_bc_root.argtypes = [P]
    L.ora_bc_root.restype = None
    L.ora_jnq.argtypes = [P, ctypes.c_int]
    L.ora_jnq.restype = None
    L.ora_step.argtypes = [P, ctypes.c_int64]
    L.ora_step.restype = None
    L.ora_set_source.argtypes = [P] + [ctypes.c_double] * 6 + [ctypes.c_int]
    L.ora_set_source.restype = None
    L.ora_threads.argtypes = []
    L.ora_threads.restype = ctypes.c_int
    L.ora_cbrt_rn.argtypes = [ctypes.c_double]
    L.ora_cbrt_rn.restype = ctypes.c_double
    L.ora_cbrt_rn_array.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    L.ora_cbrt_rn_array.restype = None
    return L


def load_variant(src_path: str, out_path: str):
    """Build and load another copy of the oracle source (used by the tests
    that plant a mistake in a copy of the oracle and check that a pin fails)."""
    subprocess.run(["gcc", *CFLAGS, src_path, "-o", out_path, "-lm"], check=True)
    return _bind(ctypes.CDLL(out_path))


def lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            _LIB = _bind(L)
    return _LIB


def cbrt_rn(x, lib=None):
    """The oracle's correctly rounded cube root, element by element (x > 0)."""
    L = lib if lib is not None else globals()["lib"]()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y = np.empty_like(x)
    L.ora_cbrt_rn_array(x.ctypes.data, y.ctypes.data, x.size)
    return y


def threads() -> int:
    """OpenMP threads the oracle's loops use (OMP_NUM_THREADS or all cores)."""
    return int(lib().ora_threads())


# Error codes of validate(): same meaning as the library's, kept independent.
OK, EINVAL, ECFL, ENEST = 0, -1, -4, -5


def level_mask(lv):
    """Cells inside level lv (ny x nx bool): its mask, or every cell."""
    m = lv.get("mask")
    if m is None:
        return np.ones((lv["ny"], lv["nx"]), dtype=bool)
    return np.asarray(m).reshape(lv["ny"], lv["nx"]) != 0


def coverage(lv):
    """Parent cells covered by child lv, over its footprint (ny/3 x nx/3 bool):
    those whose 3x3 child cells are inside it."""
    return level_mask(lv)[::3, ::3]


def _dilate(a, r):
    """Cells within Chebyshev distance r of a True cell of a."""
    ny, nx = a.shape
    p = np.pad(a, r)
    out = np.zeros_like(a)
    for dj in range(2 * r + 1):
        for di in range(2 * r + 1):
            out |= p[dj:dj + ny, di:di + nx]
    return out


def validate(levels, dx0, dt, g=9.81):
    """Check a nested layout against the paper's rules; returns an error code.

    levels: list of dicts with nx, ny, parent, off_i, off_j, h (ny x nx array)
    and, on a child, an optional mask (ny x nx, 1 = cell inside the level).
    - Eq. (4): dx_l / dt >= sqrt(2 g h_max,l) on every level (h_max over sea
      cells inside the level).
    - 3:1 inclusive nesting (Sec. II-A): child nx, ny divisible by 3, the child
      footprint inside its parent; reading: at least 3 parent cells of margin on
      every side, a footprint of at least 3x3 parent cells, siblings apart by
      at least 3 parent cells, parents listed before children.
    - A mask (the union of touching blocks of one resolution, Sec. II-A and
      Table 1) is 0 or 1 and constant over every 3x3 child block, covers at
      least one parent cell, and the root has none; every parent cell within 3
      cells of a covered one lies inside the parent.
    """
    if not levels or dt <= 0 or dx0 <= 0:
        return EINVAL
    for k, lv in enumerate(levels):
        m = lv.get("mask")
        if m is None:
            continue
        m = np.asarray(m)
        if k == 0 or m.size != lv["nx"] * lv["ny"] or not np.isin(m, (0, 1)).all():
            return ENEST
        if lv["nx"] % 3 or lv["ny"] % 3:
            return ENEST
        m = m.reshape(lv["ny"], lv["nx"])
        cov = m[::3, ::3]
        if not cov.any() or not np.array_equal(np.repeat(np.repeat(cov, 3, axis=0), 3, axis=1), m):
            return ENEST
    dxs = []
    for k, lv in enumerate(levels):
        nx, ny, p = lv["nx"], lv["ny"], lv["parent"]
        if nx < 3 or ny < 3:
            return EINVAL
        if k == 0:
            if p != -1:
                return ENEST
            dxs.append(dx0)
        else:
            if not (0 <= p < k):
                return ENEST
            if nx % 3 or ny % 3 or nx < 9 or ny < 9:
                return ENEST
            P = levels[p]
            fw, fh = nx // 3, ny // 3
            if lv["off_i"] < 3 or lv["off_j"] < 3:
                return ENEST
            if lv["off_i"] + fw > P["nx"] - 3 or lv["off_j"] + fh > P["ny"] - 3:
                return ENEST
            if P.get("mask") is not None:     # 3 cells of margin inside the parent's own cells
                near = np.zeros((P["ny"], P["nx"]), dtype=bool)
                near[lv["off_j"]:lv["off_j"] + fh, lv["off_i"]:lv["off_i"] + fw] = coverage(lv)
                if (_dilate(near, 3) & ~level_mask(P)).any():
                    return ENEST
            dxs.append(dxs[p] / 3.0)
    for k, lv in enumerate(levels):
        for q in range(k + 1, len(levels)):
            a, b = levels[k], levels[q]
            if k == 0 or a["parent"] != b["parent"]:
                continue
            ax0, ax1 = a["off_i"] - 3, a["off_i"] + a["nx"] // 3 + 3
            ay0, ay1 = a["off_j"] - 3, a["off_j"] + a["ny"] // 3 + 3
            bx0, bx1 = b["off_i"], b["off_i"] + b["nx"] // 3
            by0, by1 = b["off_j"], b["off_j"] + b["ny"] // 3
            if ax0 < bx1 and bx0 < ax1 and ay0 < by1 and by0 < ay1:
                return ENEST
    for k, lv in enumerate(levels):
        hmax = float(np.max(np.asarray(lv["h"]).reshape(lv["ny"], lv["nx"])[level_mask(lv)]))
        if hmax > 0 and dxs[k] / dt < np.sqrt(2.0 * g * hmax):
            return ECFL
    return OK


class OracleDomain:
    """A nested domain held in numpy arrays and stepped by the C oracle.

    Arrays per level (row-major, j slowest): h, eta, zmax (ny, nx);
    M (ny, nx+1) on x-faces; N (ny+1, nx) on y-faces.  Cells outside a
    masked level hold eta = 0 and zmax = 0 whatever is set there (the step
    never changes them).
    """

    def __init__(self, levels, dx0, dt, g=9.81, manning_n=0.025, dry_eps=0.01, bc=(0, 0, 0, 0),
                 x0=0.0, y0=0.0, track_clip=False, check=True, lib=None):
        if check:
            err = validate(levels, dx0, dt, g)
            if err != OK:
                raise ValueError(f"invalid nested layout (code {err})")
        self._lib = lib if lib is not None else globals()["lib"]()
        self.nlev = len(levels)
        self.dt, self.g, self.manning_n, self.dry_eps = float(dt), float(g), float(manning_n), float(dry_eps)
        self.arrays = []
        self._lv = (_Level * self.nlev)()
        dxs, oxs, oys = [], [], []
        for k, lv in enumerate(levels):
            nx, ny, p = int(lv["nx"]), int(lv["ny"]), int(lv["parent"])
            if k == 0:
                dx, ox, oy = float(dx0), float(x0), float(y0)
            else:
                dx = dxs[p] / 3.0
                ox = oxs[p] + lv["off_i"] * dxs[p]
                oy = oys[p] + lv["off_j"] * dxs[p]
            dxs.append(dx), oxs.append(ox), oys.append(oy)
            a = {
                "h": np.ascontiguousarray(np.asarray(lv["h"], dtype=np.float64).reshape(ny, nx)),
                "eta": np.zeros((ny, nx)), "zmax": np.zeros((ny, nx)),
                "M": np.zeros((ny, nx + 1)), "N": np.zeros((ny + 1, nx)),
                "M2": np.zeros((ny, nx + 1)), "N2": np.zeros((ny + 1, nx)),
                "clip": np.zeros((ny, nx)) if track_clip else None,
                "mask": (np.ascontiguousarray(level_mask(lv), dtype=np.uint8) if lv.get("mask") is not None
                         else None),
            }
            self.arrays.append(a)
            s = self._lv[k]
            s.nx, s.ny, s.parent = nx, ny, p
            s.off_i, s.off_j = int(lv.get("off_i", 0)), int(lv.get("off_j", 0))
            s.dx, s.ox, s.oy = dx, ox, oy
            for f in ("h", "eta", "M", "N", "zmax", "M2", "N2", "clip", "mask"):
                setattr(s, f, a[f].ctypes.data if a[f] is not None else None)
        self.dx = dxs
        self.origin = list(zip(oxs, oys))
        self._d = _Domain()
        self._d.nlev = self.nlev
        for q in range(4):
            self._d.bc[q] = int(bc[q])
        self._d.lv = ctypes.cast(self._lv, ctypes.POINTER(_Level))
        self._d.dt, self._d.g, self._d.manning, self._d.eps = self.dt, self.g, self.manning_n, self.dry_eps
        self._d.steps = 0
        self.set_lake_at_rest()

    # -- state -------------------------------------------------------------
    @property
    def steps(self) -> int:
        return int(self._d.steps)

    def level(self, k):
        return self.arrays[k]

    def set_lake_at_rest(self):
        """eta = 0 on sea cells, -h on land; zero fluxes; maxima at t = 0."""
        for a in self.arrays:
            h = a["h"]
            a["eta"][...] = np.where(h > 0, 0.0, -h)
            a["M"][...] = 0.0
            a["N"][...] = 0.0
            a["zmax"][...] = np.where(h > 0, a["eta"], h + a["eta"])
        for k in range(self.nlev):
            self._outside_zero(k)
        self._d.steps = 0

    def _outside_zero(self, k):
        a = self.arrays[k]
        if a["mask"] is not None:
            out = a["mask"] == 0
            a["eta"][out] = 0.0
            a["zmax"][out] = 0.0

    def set_source(self, xc, yc, a, b, theta, amp, shape):
        self._lib.ora_set_source(ctypes.byref(self._d), xc, yc, a, b, theta, amp, int(shape))
        for k in range(self.nlev):
            self._outside_zero(k)

    def set_eta(self, k, eta0):
        """Raw initial level on level k (clipped to the ground); zero fluxes; maxima reset."""
        a = self.arrays[k]
        h = a["h"]
        e = np.array(eta0, dtype=np.float64).reshape(h.shape)
        e = np.where(h + e < 0.0, -h, e)
        a["eta"][...] = e
        a["M"][...] = 0.0
        a["N"][...] = 0.0
        a["zmax"][...] = np.where(h > 0, e, h + e)
        self._outside_zero(k)
        self._d.steps = 0

    def set_state(self, k, eta=None, M=None, N=None, zmax=None):
        a = self.arrays[k]
        for name, v in (("eta", eta), ("M", M), ("N", N), ("zmax", zmax)):
            if v is not None:
                a[name][...] = np.asarray(v, dtype=np.float64).reshape(a[name].shape)
        self._outside_zero(k)

    def get_state(self, k):
        a = self.arrays[k]
        return a["eta"].copy(), a["M"].copy(), a["N"].copy()

    def max_inundation(self, k):
        return self.arrays[k]["zmax"].copy()

    def clipped_depth(self, k):
        c = self.arrays[k]["clip"]
        return None if c is None else c.copy()

    # -- stepping ----------------------------------------------------------
    def step(self, n=1):
        self._lib.ora_step(ctypes.byref(self._d), int(n))

    def run(self, t_end):
        target = int(round(t_end / self.dt))
        if target > self.steps:
            self.step(target - self.steps)

    # single phases, for the pins
    def mass(self, k):
        self._lib.ora_mass(ctypes.byref(self._d), int(k))

    def jnz(self, child):
        self._lib.ora_jnz(ctypes.byref(self._d), int(child))

    def momentum(self, k):
        self._lib.ora_momentum(ctypes.byref(self._d), int(k))

    def bc_root(self):
        self._lib.ora_bc_root(ctypes.byref(self._d))

    def jnq(self, child):
        self._lib.ora_jnq(ctypes.byref(self._d), int(child))

    def update_max(self, k):
        self._lib.ora_max(ctypes.byref(self._d), int(k))
