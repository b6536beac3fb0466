"""Forecast serving over the batch API of librti: continuous batching.

Requests (a site, a source, a simulated duration) arrive at any time.  The
server admits a waiting request as soon as its device footprint
(rti_domain_footprint) fits in the HBM budget left by the requests already
running, creates its domain (state resident on the device from then on) and
adds it to the one running batch.  The batch advances in chunks of steps; a
chunk never runs past the end of any member, so each request stops exactly
at its own step count.  A finished request's maxima (the forecast) are read
back, its domain is removed from the batch and destroyed, and its footprint
returns to the budget.  Requests that arrive while others are on the GPU
therefore join the running launch between two chunks, and their work shares
every launch with the others'.  A new request's domain is created and its
source set on a staging stream while the current chunk runs, and the batch
adopts it for the next chunk.  All numerical work runs in librti's kernels;
this module only schedules.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    site: object                 # a scenarios.Scenario (levels, bathymetry, dx0, dt, ...)
    source: tuple                # rti_source fields (xc, yc, a, b, theta, amp, shape)
    steps: int                   # time steps to simulate
    arrival: float               # seconds after the server starts
    initial: list | None = None  # optional raw initial water level per level (instead of the source)


@dataclasses.dataclass
class Result:
    rid: int
    cells: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    maxima: list                 # per level: max water level at sea / max depth on land (host arrays)

    @property
    def time_to_forecast(self):
        return self.finished - self.arrival


_FOOTPRINTS = {}


def footprint(site, precision, flags=0) -> int:
    """Device bytes of a request's domain (validated like create), cached per site."""
    from .rti import make_desc, rti_domain_footprint
    key = (id(site), precision, flags)
    if key not in _FOOTPRINTS:
        desc, keep = make_desc(site.levels, site.dx0, site.dt, site.g, site.manning_n, site.dry_eps, site.bc,
                               site.x0, site.y0, precision, flags)
        _FOOTPRINTS[key] = rti_domain_footprint(desc) + 256
        del keep
    return _FOOTPRINTS[key]


class ForecastServer:
    """One batch on one GPU; requests are admitted by footprint against
    hbm_budget bytes.  chunk_steps bounds how long a new arrival waits for
    the next admission point.  keep_state: also keep each request's final
    (eta, M, N) per level in its result (for tests)."""

    def __init__(self, hbm_budget: int, precision: int, chunk_steps: int = 200, flags: int = 0,
                 keep_state: bool = False, device: str = "cuda:0"):
        import torch

        from .rti import Batch
        self.budget = int(hbm_budget)
        self.precision = int(precision)
        self.chunk = int(chunk_steps)
        self.flags = int(flags)
        self.keep_state = keep_state
        self.device = device
        self.stream = torch.cuda.current_stream(torch.device(device))
        self.stage = torch.cuda.Stream(torch.device(device))   # new requests are prepared here
        self.batch = Batch([], device=device, stream=self.stream)
        self.used = 0
        self.peak_members = 0
        self.peak_bytes = 0
        self.cell_updates = 0
        self.chunks = []        # (steps, seconds, cells of the members, cells computed) per chunk

    def _admit(self, req: Request, now: float):
        from .rti import Domain
        s = req.site
        d = Domain(s.levels, s.dx0, s.dt, g=s.g, manning_n=s.manning_n, dry_eps=s.dry_eps, bc=s.bc, x0=s.x0, y0=s.y0,
                   flags=self.flags, device=self.device, stream=self.stage, precision=self.precision)
        if req.initial is not None:
            for k, eta0 in enumerate(req.initial):
                d.set_eta(k, eta0)
        else:
            d.set_source(*req.source)
        self.batch.add(d)       # waits for the staging stream only; the running chunk goes on
        return d

    def run(self, requests, clock=time.perf_counter, log=None):
        """Serve the requests (arrival times relative to the start) and return
        their results in completion order."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            need = footprint(r.site, self.precision, self.flags)
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs {need} bytes, more than the whole budget {self.budget}")
        waiting = deque()
        active = {}            # rid -> [request, domain, remaining steps, footprint, admitted]
        results = []
        t0 = clock()
        while pending or waiting or active:
            # 1. enqueue the next chunk for the running requests (asynchronous)
            chunk = []
            if active:
                n = min(self.chunk, min(a[2] for a in active.values()))
                c_all0, c_comp0 = self.batch.cell_updates()
                t_chunk = clock()
                self.batch.step(n)
                chunk = list(active)
                cells = sum(a[0].site.cells for a in active.values())
                self.cell_updates += n * cells
            # 2. while it runs: take in arrivals, admit in arrival order while the head fits
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                need = footprint(r.site, self.precision, self.flags)
                if self.used + need > self.budget:
                    break
                waiting.popleft()
                d = self._admit(r, now)
                self.used += need
                active[r.rid] = [r, d, r.steps, need, clock() - t0]
                if log:
                    log(f"t={clock() - t0:7.2f}s admit request {r.rid} ({r.site.cells} cells, {r.steps} steps); "
                        f"{len(active)} running, {self.used / 2**30:.2f} GiB")
            self.peak_members = max(self.peak_members, len(active))
            self.peak_bytes = max(self.peak_bytes, self.used)
            if not chunk:
                if not active and pending:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - (clock() - t0))))
                continue
            # 3. the chunk is done: retire the requests that reached their step count
            self.batch.sync()
            c_all1, c_comp1 = self.batch.cell_updates()
            self.chunks.append((n, clock() - t_chunk, cells, c_comp1 - c_comp0))
            for rid in chunk:
                active[rid][2] -= n
            for rid in [rid for rid in chunk if active[rid][2] == 0]:
                r, d, _, need, admitted = active.pop(rid)
                maxima = [d.max_inundation(k) for k in range(len(d.levels))]
                res = Result(rid, r.site.cells, r.steps, r.arrival, admitted, clock() - t0, maxima)
                if self.keep_state:
                    res.state = [d.get_state(k) for k in range(len(d.levels))]
                self.batch.remove(d)
                d.close()
                self.used -= need
                results.append(res)
                if log:
                    log(f"t={res.finished:7.2f}s done request {rid}: time to forecast {res.time_to_forecast:.2f} s")
        self.makespan = clock() - t0
        return results

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None


def fit_cost_model(chunks):
    """The time of one batch step as a * (cells computed in the step) + b
    (least squares over the chunks of a serving run; the per-launch term b
    holds the launch and listing overhead).  The analogue of the paper's
    per-block cost model (Sec. IV-D, Eq. 5: a cost per cell plus a cost per
    block), with the batch's one launch per step in place of a block."""
    A = np.array([[c[3] / c[0], 1.0] for c in chunks if c[0] > 0])
    y = np.array([c[1] / c[0] for c in chunks if c[0] > 0])
    w = np.sqrt(np.array([c[0] for c in chunks if c[0] > 0], dtype=np.float64))   # long chunks count more
    Aw, yw = A * w[:, None], y * w
    (a, b), *_ = np.linalg.lstsq(Aw, yw, rcond=None)
    # both costs are non-negative: on the boundary, fit the other one alone
    if a < 0:
        a, b = 0.0, float(np.dot(Aw[:, 1], yw) / np.dot(Aw[:, 1], Aw[:, 1]))
    elif b < 0:
        a, b = float(np.dot(Aw[:, 0], yw) / np.dot(Aw[:, 0], Aw[:, 0])), 0.0
    return float(a), float(b)


def predict(requests, a, b, computed_fraction, hbm_budget, precision, chunk_steps, flags=0):
    """Times to forecast that the cost model predicts for a request stream
    under the server's policy (admission in arrival order while the head's
    footprint fits, chunks that stop at the first member's end), with each
    step costing a * computed_fraction * (cells of the members) + b.
    Returns {rid: predicted seconds from arrival to forecast}."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    active = {}
    now, used, out = 0.0, 0, {}
    while pending or active:
        while pending and (pending[0].arrival <= now or not active):
            r = pending[0]
            need = footprint(r.site, precision, flags)
            if used + need > hbm_budget:
                break
            pending.popleft()
            now = max(now, r.arrival)
            active[r.rid] = [r, r.steps, need]
            used += need
        if not active:
            now = pending[0].arrival
            continue
        n = min(chunk_steps, min(v[1] for v in active.values()))
        cells = sum(v[0].site.cells for v in active.values())
        now += n * (a * computed_fraction * cells + b)
        for rid in list(active):
            active[rid][1] -= n
            if active[rid][1] == 0:
                r, _, need = active.pop(rid)
                used -= need
                out[rid] = now - r.arrival
    return out


def percentiles(results, qs=(50, 99)):
    t = np.array([r.time_to_forecast for r in results])
    return {f"p{q}": float(np.percentile(t, q)) for q in qs}
