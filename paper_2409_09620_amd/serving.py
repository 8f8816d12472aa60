"""Continuous-batching solve server over the C ABI (dg_batch_*).

Requests (a mesh, a degree, initial data, a final time) arrive over time.  The
server keeps every admitted request's state resident in HBM and advances all
of them together: each stage pass is one launch over the whole active set,
every request with its own alpha, Delta t and t_end.  A request is admitted as
soon as it has arrived and its HBM footprint fits in the budget (or the server
is empty), finished requests are read back and freed every few steps, and the
batch is rebuilt whenever its membership changes.

A member's reductions run over its own 256-cell groups in a fixed order, so its
result is the same, bit for bit, whatever else is in flight.

This module only orders calls: every step of the method runs in the HIP
library.
"""

import ctypes
import time
from dataclasses import dataclass, field
from typing import Any, Callable, List, Optional

import numpy as np

from .binding import Batch, Solver, load_library

# partial records of a batch: 17 doubles per 256-cell group
_BATCH_BYTES_PER_CELL = 17 * 8 / 256.0


def footprint_bytes(n_cell, k):
    """Device bytes one request holds while admitted: its workspace plus its share
    of the batch's partial records."""
    b = ctypes.c_size_t(0)
    if load_library().dg_workspace_bytes(int(n_cell), int(k), ctypes.byref(b)) != 0:
        raise ValueError("bad request size")
    return int(b.value + _BATCH_BYTES_PER_CELL * n_cell + 4096)


@dataclass
class Request:
    """One solve: `build()` returns (mesh, kind, params); k the degree."""
    id: int
    k: int
    n_cell: int
    t_end: float
    build: Callable[[], Any]
    arrival: float = 0.0                 # seconds after the start of the run
    precision: str = "fp64"
    # filled in by the server
    admitted: Optional[float] = None
    done: Optional[float] = None
    steps: int = 0
    t: float = 0.0
    result: Optional[np.ndarray] = None
    error: Optional[str] = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival

    @property
    def dof_stages(self):
        return self.n_cell * 4 * (self.k + 1) * (self.k + 2) // 2 * 3 * self.steps


@dataclass
class ServeStats:
    wall: float
    requests: int
    p50: float
    p99: float
    mean: float
    dof_stage_per_s: float
    peak_members: int
    rebuilds: int
    steps_launched: int
    latencies: List[float] = field(default_factory=list)


class Server:
    """hbm_budget: bytes the admitted requests may hold together; steps_per_tick:
    batched steps between polls (admission and retirement happen at polls);
    keep_results: read each finished state back to the host."""

    def __init__(self, device=0, hbm_budget=8 << 30, steps_per_tick=8, keep_results=True, autotune=False):
        self.device = int(device)
        self.budget = int(hbm_budget)
        self.steps_per_tick = int(steps_per_tick)
        self.keep_results = keep_results
        self.autotune = autotune

    def _admit(self, req, t0):
        m, kind, params = req.build()
        s = Solver(m, req.k, device=self.device)
        s.init_problem(kind, params, precision=req.precision)
        s.set_t_end(req.t_end)
        req.admitted = time.perf_counter() - t0
        return s

    def run(self, requests, clock=time.perf_counter):
        """Serves `requests` (arrival times relative to the start) to completion
        and returns ServeStats; each request gets its result, t, step count and
        completion time."""
        pending = sorted(requests, key=lambda r: r.arrival)
        active = []                      # (request, solver, footprint)
        used = 0
        batch = None
        members_changed = False
        peak = rebuilds = launched = 0
        t0 = clock()
        while pending or active:
            now = clock() - t0
            # admission: arrived requests in arrival order while they fit
            while pending and pending[0].arrival <= now:
                r = pending[0]
                fp = footprint_bytes(r.n_cell, r.k)
                if active and used + fp > self.budget:
                    break
                pending.pop(0)
                active.append((r, self._admit(r, t0), fp))
                used += fp
                members_changed = True
            if not active:
                # idle until the next arrival
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            if members_changed:
                if batch is not None:
                    batch.close()
                batch = Batch([s for _, s, _ in active])
                if self.autotune:
                    batch.autotune(reps=1)
                rebuilds += 1
                members_changed = False
                peak = max(peak, len(active))
            batch.step(self.steps_per_tick)
            launched += self.steps_per_tick
            _, status = batch.status()
            # retirement: read finished members back, then drop the batch before
            # their contexts
            keep, done = [], []
            for (r, s, fp), st in zip(active, status):
                if st[0] == 0.0:
                    r.done = clock() - t0
                    r.t, r.steps = float(st[2]), int(st[3])
                    if st[1] != 0.0:
                        r.error = "a cell average left the admissible set"
                    if self.keep_results:
                        r.result = s.readback()[0]
                    used -= fp
                    done.append(s)
                else:
                    keep.append((r, s, fp))
            if done:
                batch.close()
                batch = None
                members_changed = True
                for s in done:
                    s.close()
            active = keep
        wall = clock() - t0
        lat = np.array([r.latency for r in requests])
        return ServeStats(wall=wall, requests=len(requests), p50=float(np.percentile(lat, 50)),
                          p99=float(np.percentile(lat, 99)), mean=float(lat.mean()),
                          dof_stage_per_s=sum(r.dof_stages for r in requests) / wall, peak_members=peak,
                          rebuilds=rebuilds, steps_launched=launched, latencies=lat.tolist())
