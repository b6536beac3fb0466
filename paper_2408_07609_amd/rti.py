"""Python binding of librti (include/rti.h): argument marshalling only.

Every function named ``rti_*`` here calls the C function of the same name and
raises RtiError on a negative return code.  ``Domain`` wraps one nested domain
whose device memory is a torch uint8 tensor (the arena) and whose kernels run
on torch's current HIP stream; torch supplies memory and streams, every step
of the computation runs in the library's HIP kernels.  There is no fallback:
without the built library, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "librti.so")

RTI_OK, RTI_EINVAL, RTI_ENOMEM, RTI_EHIP, RTI_ECFL, RTI_ENEST, RTI_ESTATE, RTI_EDIVERGED = 0, -1, -2, -3, -4, -5, -6, -7
RTI_EINTERNAL = -8
RTI_STATUS_DIVERGED, RTI_STATUS_LIST_OVERFLOW = 0x1, 0x2
RTI_FP64, RTI_FP32_BULK = 0, 1
RTI_BC_OPEN, RTI_BC_WALL = 0, 1
RTI_GAUSS, RTI_COS2_ELLIPSE = 0, 1
RTI_FLAG_NO_GRAPH, RTI_FLAG_NO_ACTIVE, RTI_FLAG_PHASED, RTI_FLAG_PERSISTENT = 0x1, 0x2, 0x4, 0x8
RTI_MAX_LEVELS = 128
RTI_TILE_ROWS_MIN, RTI_TILE_ROWS_MAX, RTI_TILE_ROWS_DEFAULT = 4, 64, 12
RTI_PROBE_CBRT, RTI_PROBE_RECIP, RTI_PROBE_SQRT = 0, 1, 2
RTI_AUTOTUNE_NOALLOC_MAX_BYTES = 128 << 20

_dptr = ctypes.POINTER(ctypes.c_double)


class rti_level_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("parent", ctypes.c_int32),
                ("off_i", ctypes.c_int32), ("off_j", ctypes.c_int32), ("h", _dptr),
                ("mask", ctypes.POINTER(ctypes.c_uint8))]


class rti_domain_desc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("levels", ctypes.POINTER(rti_level_desc)),
                ("dx0", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dt", ctypes.c_double), ("g", ctypes.c_double), ("manning_n", ctypes.c_double),
                ("dry_eps", ctypes.c_double), ("bc", ctypes.c_int32 * 4), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class rti_source(ctypes.Structure):
    _fields_ = [("xc", ctypes.c_double), ("yc", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("theta", ctypes.c_double), ("amp", ctypes.c_double), ("shape", ctypes.c_int32)]


class RtiError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{message} (code {code})")
        self.code = code


FUNCTIONS = {
    "rti_domain_footprint": (ctypes.c_int, [ctypes.POINTER(rti_domain_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "rti_domain_create": (ctypes.c_int, [ctypes.POINTER(rti_domain_desc), ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rti_set_source": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rti_source)]),
    "rti_set_eta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dptr]),
    "rti_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "rti_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "rti_max_inundation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dptr]),
    "rti_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dptr, _dptr, _dptr]),
    "rti_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dptr, _dptr, _dptr]),
    "rti_set_max": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dptr]),
    "rti_steps_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rti_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "rti_device_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "rti_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dptr, ctypes.POINTER(ctypes.c_char_p),
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dptr]),
    "rti_active_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "rti_cell_updates": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "rti_batch_cell_updates": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "rti_domain_set_tile_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rti_domain_tile_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "rti_graph_launches": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rti_domain_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dptr]),
    "rti_domain_autotune_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                   _dptr]),
    "rti_domain_destroy": (None, [ctypes.c_void_p]),
    "rti_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "rti_batch_add": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rti_batch_remove": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rti_batch_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "rti_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "rti_batch_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "rti_batch_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dptr, _dptr, _dptr]),
    "rti_batch_destroy": (None, [ctypes.c_void_p]),
    "rti_math_probe": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]),
    "rti_stream_probe": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]),
    "rti_last_error": (ctypes.c_char_p, []),
    "rti_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}


def _load():
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
    # first makes librti bind to that same runtime instead of a second copy
    # from /opt/rocm, so both share one device context, one allocator view
    # and the same streams.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"librti.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          f"python paper_2408_07609_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in FUNCTIONS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(code):
    if code < 0:
        raise RtiError(code, LIB.rti_last_error().decode())
    return code


def _as_dptr(a):
    return a.ctypes.data_as(_dptr) if a is not None else None


# ---------------------------------------------------------------------------
# Same-name wrappers of the C ABI.
def rti_domain_footprint(desc: rti_domain_desc) -> int:
    n = ctypes.c_size_t(0)
    _check(LIB.rti_domain_footprint(ctypes.byref(desc), ctypes.byref(n)))
    return int(n.value)


def rti_domain_create(desc: rti_domain_desc, arena_ptr: int | None, arena_bytes: int, stream_ptr: int | None) -> int:
    out = ctypes.c_void_p(0)
    _check(LIB.rti_domain_create(ctypes.byref(desc), arena_ptr, arena_bytes, stream_ptr, ctypes.byref(out)))
    return out.value


def rti_math_probe(op: int, x_ptr: int, y_ptr: int, n: int, stream_ptr: int | None):
    _check(LIB.rti_math_probe(op, x_ptr, y_ptr, n, stream_ptr))


def stream_probe(inputs, outputs):
    """rti_stream_probe over float64 device tensors of equal size, on torch's
    current stream."""
    import torch
    n = inputs[0].numel()
    for t in list(inputs) + list(outputs):
        if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
            raise ValueError("stream_probe takes contiguous float64 device tensors of one size")
    ins = (ctypes.c_void_p * len(inputs))(*[t.data_ptr() for t in inputs])
    outs = (ctypes.c_void_p * max(1, len(outputs)))(*[t.data_ptr() for t in outputs])
    _check(LIB.rti_stream_probe(ins, len(inputs), outs, len(outputs), n, torch.cuda.current_stream().cuda_stream))


def math_probe(op: int, x):
    """The library's FP64 operation `op` (RTI_PROBE_*) applied to a float64
    device tensor x on torch's current stream; returns a new tensor."""
    import torch
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("x must be a float64 device tensor")
    x = x.contiguous()
    y = torch.empty_like(x)
    rti_math_probe(op, x.data_ptr(), y.data_ptr(), x.numel(), torch.cuda.current_stream().cuda_stream)
    return y


def rti_set_source(dom: int, src: rti_source):
    _check(LIB.rti_set_source(dom, ctypes.byref(src)))


def rti_set_eta(dom: int, level: int, eta0: np.ndarray):
    _check(LIB.rti_set_eta(dom, level, _as_dptr(np.ascontiguousarray(eta0, dtype=np.float64))))


def rti_step(dom: int, nsteps: int):
    _check(LIB.rti_step(dom, int(nsteps)))


def rti_run(dom: int, t_end: float):
    _check(LIB.rti_run(dom, float(t_end)))


def rti_max_inundation(dom: int, level: int, out: np.ndarray):
    _check(LIB.rti_max_inundation(dom, level, _as_dptr(out)))


def rti_get_state(dom: int, level: int, eta, M, N):
    _check(LIB.rti_get_state(dom, level, _as_dptr(eta), _as_dptr(M), _as_dptr(N)))


def rti_set_state(dom: int, level: int, eta, M, N):
    _check(LIB.rti_set_state(dom, level, _as_dptr(eta), _as_dptr(M), _as_dptr(N)))


def rti_set_max(dom: int, level: int, zmax):
    _check(LIB.rti_set_max(dom, level, _as_dptr(zmax)))


def rti_steps_done(dom: int) -> int:
    n = ctypes.c_int64(0)
    _check(LIB.rti_steps_done(dom, ctypes.byref(n)))
    return int(n.value)


def rti_sync(dom: int):
    _check(LIB.rti_sync(dom))


def rti_profile(dom: int, nsteps: int):
    """Returns ({kernel name: average ms per launch}, average cells computed per step)."""
    cap = 16
    ms = (ctypes.c_double * cap)()
    names = (ctypes.c_char_p * cap)()
    n = ctypes.c_int32(0)
    cells = ctypes.c_double(0.0)
    _check(LIB.rti_profile(dom, int(nsteps), ms, names, cap, ctypes.byref(n), ctypes.byref(cells)))
    return {names[k].decode(): float(ms[k]) for k in range(n.value)}, float(cells.value)


def rti_active_tiles(dom: int):
    """Returns (computed tiles, all tiles, cells in the computed tiles) of the last step."""
    a, t, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(LIB.rti_active_tiles(dom, ctypes.byref(a), ctypes.byref(t), ctypes.byref(c)))
    return int(a.value), int(t.value), int(c.value)


def rti_cell_updates(dom: int):
    """Returns (all cell-updates, computed cell-updates) of the domain's own steps."""
    a, c = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(LIB.rti_cell_updates(dom, ctypes.byref(a), ctypes.byref(c)))
    return int(a.value), int(c.value)


def rti_batch_cell_updates(batch: int):
    """Returns (all cell-updates, computed cell-updates) of the batch's steps."""
    a, c = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(LIB.rti_batch_cell_updates(batch, ctypes.byref(a), ctypes.byref(c)))
    return int(a.value), int(c.value)


def rti_domain_set_tile_rows(dom: int, rows: int):
    _check(LIB.rti_domain_set_tile_rows(dom, int(rows)))


def rti_domain_tile_rows(dom: int) -> int:
    n = ctypes.c_int32(0)
    _check(LIB.rti_domain_tile_rows(dom, ctypes.byref(n)))
    return int(n.value)


def rti_graph_launches(dom: int):
    """Step graphs launched per kind: (default, dense)."""
    c = (ctypes.c_int64 * 2)()
    _check(LIB.rti_graph_launches(dom, c))
    return tuple(int(v) for v in c)


def rti_domain_autotune(dom: int, nsteps: int):
    """Returns (tile rows chosen, ms per step at that height)."""
    rows, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(LIB.rti_domain_autotune(dom, int(nsteps), ctypes.byref(rows), ctypes.byref(ms)))
    return int(rows.value), float(ms.value)


def rti_device_status(dom: int) -> int:
    bits = ctypes.c_uint32(0)
    _check(LIB.rti_device_status(dom, ctypes.byref(bits)))
    return int(bits.value)


def rti_domain_autotune_noalloc(dom: int, nsteps: int):
    """rti_domain_autotune staged in the library's static device array (no
    allocation).  Returns (tile rows chosen, ms per step at that height)."""
    rows, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(LIB.rti_domain_autotune_noalloc(dom, int(nsteps), ctypes.byref(rows), ctypes.byref(ms)))
    return int(rows.value), float(ms.value)


def rti_domain_destroy(dom: int | None):
    LIB.rti_domain_destroy(dom)


def rti_batch_create(members, stream_ptr: int | None, flags: int = 0) -> int:
    arr = (ctypes.c_void_p * max(1, len(members)))(*members)
    out = ctypes.c_void_p(0)
    _check(LIB.rti_batch_create(arr, len(members), stream_ptr, int(flags), ctypes.byref(out)))
    return out.value


def rti_batch_add(batch: int, dom: int):
    _check(LIB.rti_batch_add(batch, dom))


def rti_batch_remove(batch: int, dom: int):
    _check(LIB.rti_batch_remove(batch, dom))


def rti_batch_size(batch: int) -> int:
    n = ctypes.c_int32(0)
    _check(LIB.rti_batch_size(batch, ctypes.byref(n)))
    return int(n.value)


def rti_batch_step(batch: int, nsteps: int):
    _check(LIB.rti_batch_step(batch, int(nsteps)))


def rti_batch_sync(batch: int):
    _check(LIB.rti_batch_sync(batch))


def rti_batch_profile(batch: int, nsteps: int):
    """Returns (fused ms per launch, active-list ms per launch, cells computed per step)."""
    f, a, c = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(LIB.rti_batch_profile(batch, int(nsteps), ctypes.byref(f), ctypes.byref(a), ctypes.byref(c)))
    return float(f.value), float(a.value), float(c.value)


def rti_batch_destroy(batch: int | None):
    LIB.rti_batch_destroy(batch)


def rti_last_error() -> str:
    return LIB.rti_last_error().decode()


def rti_strerror(code: int) -> str:
    return LIB.rti_strerror(code).decode()


# ---------------------------------------------------------------------------
def make_desc(levels, dx0, dt, g=9.81, manning_n=0.025, dry_eps=0.01, bc=(0, 0, 0, 0), x0=0.0, y0=0.0,
              precision=RTI_FP64, flags=0):
    """Build an rti_domain_desc from level dicts (nx, ny, parent, off_i, off_j,
    h as an (ny, nx) array, optionally mask as an (ny, nx) 0/1 array: the
    cells inside a level of touching blocks).  Returns (desc, keepalive)."""
    hs = [np.ascontiguousarray(lv["h"], dtype=np.float64) for lv in levels]
    masks = [None if lv.get("mask") is None else np.ascontiguousarray(lv["mask"], dtype=np.uint8) for lv in levels]
    arr = (rti_level_desc * len(levels))()
    for k, lv in enumerate(levels):
        arr[k].nx, arr[k].ny = int(lv["nx"]), int(lv["ny"])
        arr[k].parent = int(lv["parent"])
        arr[k].off_i, arr[k].off_j = int(lv.get("off_i", 0)), int(lv.get("off_j", 0))
        arr[k].h = hs[k].ctypes.data_as(_dptr)
        if masks[k] is not None:
            arr[k].mask = masks[k].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    d = rti_domain_desc()
    d.n_levels = len(levels)
    d.levels = ctypes.cast(arr, ctypes.POINTER(rti_level_desc))
    d.dx0, d.x0, d.y0, d.dt = float(dx0), float(x0), float(y0), float(dt)
    d.g, d.manning_n, d.dry_eps = float(g), float(manning_n), float(dry_eps)
    for q in range(4):
        d.bc[q] = int(bc[q])
    d.precision, d.flags = int(precision), int(flags)
    return d, (arr, hs, masks)


class Domain:
    """One nested domain on the current GPU.  Device memory: a torch uint8
    tensor; stream: torch's current stream (or the one given)."""

    def __init__(self, levels, dx0, dt, g=9.81, manning_n=0.025, dry_eps=0.01, bc=(0, 0, 0, 0), x0=0.0, y0=0.0,
                 flags=0, device="cuda:0", stream=None, precision=RTI_FP64):
        import torch
        self.levels = [dict(nx=int(lv["nx"]), ny=int(lv["ny"])) for lv in levels]
        self.dt = float(dt)
        self.precision = int(precision)
        desc, keep = make_desc(levels, dx0, dt, g, manning_n, dry_eps, bc, x0, y0, precision, flags)
        self.footprint = rti_domain_footprint(desc)
        dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        with torch.cuda.device(dev):
            self.arena = torch.empty(self.footprint + 256, dtype=torch.uint8, device=dev)
            base = self.arena.data_ptr()
            aligned = (base + 255) // 256 * 256
            self._h = rti_domain_create(desc, aligned, self.footprint, self.stream.cuda_stream)
        del keep

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            rti_domain_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- setup
    def set_source(self, xc, yc, a, b, theta, amp, shape):
        rti_set_source(self._h, rti_source(xc, yc, a, b, theta, amp, int(shape)))

    def set_eta(self, level, eta0):
        rti_set_eta(self._h, level, np.asarray(eta0, dtype=np.float64))

    def set_state(self, level, eta=None, M=None, N=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        rti_set_state(self._h, level, c(eta), c(M), c(N))

    def set_max(self, level, zmax):
        rti_set_max(self._h, level, np.ascontiguousarray(zmax, dtype=np.float64))

    # -- stepping
    def step(self, n=1):
        rti_step(self._h, n)

    def run(self, t_end):
        rti_run(self._h, t_end)

    def sync(self):
        rti_sync(self._h)

    @property
    def steps(self):
        return rti_steps_done(self._h)

    def device_status(self):
        """The sticky device checks (RTI_STATUS_* bits); synchronises."""
        return rti_device_status(self._h)

    def _no_overflow(self):
        # an overflowed active-tile list breaks an invariant of the library:
        # every read of results checks for it
        if self.device_status() & RTI_STATUS_LIST_OVERFLOW:
            raise RtiError(RTI_EINTERNAL, "an active-tile list overflowed on the device")

    # -- results
    def get_state(self, level):
        nx, ny = self.levels[level]["nx"], self.levels[level]["ny"]
        e, M, N = np.empty((ny, nx)), np.empty((ny, nx + 1)), np.empty((ny + 1, nx))
        rti_get_state(self._h, level, e, M, N)
        self._no_overflow()
        return e, M, N

    def max_inundation(self, level):
        nx, ny = self.levels[level]["nx"], self.levels[level]["ny"]
        out = np.empty((ny, nx))
        rti_max_inundation(self._h, level, out)
        return out

    def profile(self, nsteps):
        """({kernel: ms per launch}, cells computed per step) over nsteps eager steps."""
        return rti_profile(self._h, nsteps)

    def active_tiles(self):
        return rti_active_tiles(self._h)

    def cell_updates(self):
        """(all, computed) cell-updates of this domain's own steps."""
        return rti_cell_updates(self._h)

    def graph_launches(self):
        """Step graphs launched per kind: (default, dense)."""
        return rti_graph_launches(self._h)

    # -- tile shape
    @property
    def tile_rows(self):
        return rti_domain_tile_rows(self._h)

    def set_tile_rows(self, rows):
        rti_domain_set_tile_rows(self._h, rows)

    def autotune(self, nsteps=20):
        """Time every candidate tile height from the current state, keep the
        fastest, restore the state.  Returns (rows, ms per step)."""
        return rti_domain_autotune(self._h, nsteps)

    def autotune_noalloc(self, nsteps=20):
        """autotune without allocating device memory (the snapshot is staged
        in the library's static array of RTI_AUTOTUNE_NOALLOC_MAX_BYTES)."""
        return rti_domain_autotune_noalloc(self._h, nsteps)


class Batch:
    """Domains stepped together by one launch per step over all their tiles.
    Members share one precision; the batch runs on the stream given here
    (default: torch's current stream) and adopts members created on other
    streams while they belong to it."""

    def __init__(self, members=(), flags=0, device="cuda:0", stream=None):
        import torch
        dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.members = list(members)
        with torch.cuda.device(dev):
            self._h = rti_batch_create([m._h for m in self.members], self.stream.cuda_stream, flags)

    def add(self, dom):
        rti_batch_add(self._h, dom._h)
        self.members.append(dom)

    def remove(self, dom):
        rti_batch_remove(self._h, dom._h)
        self.members.remove(dom)

    def __len__(self):
        return rti_batch_size(self._h)

    def step(self, n=1):
        rti_batch_step(self._h, n)

    def sync(self):
        rti_batch_sync(self._h)

    def profile(self, nsteps):
        """(fused ms per launch, active-list ms per launch, cells computed per step)."""
        return rti_batch_profile(self._h, nsteps)

    def cell_updates(self):
        """(all, computed) cell-updates of the batch's steps."""
        return rti_batch_cell_updates(self._h)

    def close(self):
        if getattr(self, "_h", None):
            rti_batch_destroy(self._h)
            self._h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def autotune_batch_rows(domains, nsteps=8, candidates=(6, 8, 10, 12, 16, 24)):
    """One tile height for every member of a batch: for each candidate, set
    it on every member, step the batch twice untimed and time nsteps batch
    steps with every tile computed (rti_batch_profile), and keep the fastest.
    A member's own autotuner picks short tiles for a small domain alone (more
    wavefronts for it), but in a batch the members' tiles already fill the
    GPU, and short tiles only add recomputed warm-up rows.  Of the heights
    within 2 % of the fastest the shortest is kept: a run skips stationary
    tiles, at a finer grain with shorter tiles, which the every-tile trials
    do not see.  The trials step the domains: pass copies made for tuning
    (same shapes), not the domains to be run.  Returns (rows, fused-kernel ms
    per step at that height)."""
    times = []
    for rows in candidates:
        for d in domains:
            d.set_tile_rows(rows)
        with Batch(domains, flags=RTI_FLAG_NO_ACTIVE) as b:
            b.step(2)
            fused_ms, _, _ = b.profile(nsteps)
        times.append((rows, fused_ms))
    fastest = min(ms for _, ms in times)
    return min((r, ms) for r, ms in times if ms <= fastest * 1.02)
