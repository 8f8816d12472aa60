"""Continuous-batching solve server over the C ABI (dg_batch_*).

Requests (a mesh, a degree, initial data, a final time, a precision) arrive over
time.  The server keeps every admitted request's state resident in HBM and
advances all of them together: each stage pass is one launch over the active set
of a precision, every request with its own alpha, Delta t and t_end.

* Admission.  A request whose footprint fits in the HBM budget (or any request
  when nothing is admitted) is handed to a preparation thread as soon as it has
  arrived.  The thread builds the mesh tables on the host, uploads them and
  projects the initial data on a stream of its own, so a large request does not
  stall the requests already stepping.  A request that fails there (a bad mesh,
  no memory) is finished with its error; the others go on.
* Stepping.  A precision's requests are batched by size class (meshes below
  small_cells cells, and the rest), each class's batch on a stream of its own,
  so that a small request's steps do not wait on a large one's: the batches'
  kernels run side by side and each batch is polled when its last steps_per_tick
  steps have finished.  Prepared requests join their batch when it is idle.
* Retirement.  A request that reached its t_end is read back at the poll that
  sees it finished.  It stays in its batch, skipped by the kernels, until
  requests join that batch: the batch (and its captured step) is rebuilt only
  when members join, and the finished ones are dropped then.

A member's reductions run over its own 256-cell groups in a fixed order, so its
result is the same, bit for bit, whatever else is in flight.

This module only orders calls: every step of the method runs in the HIP
library.
"""

import ctypes
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Callable, List, Optional

import numpy as np

from .binding import PRECISION, Batch, Solver, load_library

# partial records of a batch: 26 doubles per 256-cell group
_BATCH_BYTES_PER_CELL = 26 * 8 / 256.0


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
    admitted: Optional[float] = None     # handed to a preparation thread
    joined: Optional[float] = None       # first stepped in a batch
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
    errors: int = 0
    latencies: List[float] = field(default_factory=list)


class _Group:
    """The batch of one precision and size class: its members (request, solver,
    footprint), its stream and the event of its last launched steps."""

    def __init__(self, device):
        import torch
        self.members = []
        self.batch = None
        self.stream = torch.cuda.Stream(device)
        self.event = None

    def idle(self):
        return self.event is None or self.event.query()

    def active_count(self):
        return sum(1 for m in self.members if m[0].done is None)


class Server:
    """hbm_budget: bytes the admitted requests may hold together; steps_per_tick:
    batched steps between polls; keep_results: read each finished state back to
    the host; prepare_threads: threads that build, upload and project new
    requests; small_cells: meshes below this many cells are batched apart from
    the larger ones; progress: a callable given one line of text at every admission,
    join and completion and every progress_every seconds (the members' t and step
    counts); max_wall: seconds after which the run stops and the unfinished
    requests end with an error."""

    def __init__(self, device=0, hbm_budget=8 << 30, steps_per_tick=8, keep_results=True, autotune=False,
                 prepare_threads=2, small_cells=100_000, progress=None, progress_every=5.0, max_wall=None):
        self.progress = progress
        self.progress_every = float(progress_every)
        self.max_wall = max_wall
        self.device = int(device)
        self.budget = int(hbm_budget)
        self.steps_per_tick = int(steps_per_tick)
        self.keep_results = keep_results
        self.autotune = autotune
        self.prepare_threads = max(1, int(prepare_threads))
        self.small_cells = int(small_cells)
        self._tls = threading.local()

    def _prepare(self, req):
        """Worker thread: the request's context, mesh tables, upload and initial
        state, on the thread's own stream (dg_init_problem synchronises it)."""
        import torch
        torch.cuda.set_device(self.device)
        if getattr(self._tls, "stream", None) is None:
            self._tls.stream = torch.cuda.Stream(self.device)
        with torch.cuda.stream(self._tls.stream):
            m, kind, params = req.build()
            s = Solver(m, req.k, device=self.device)
            try:
                s.init_problem(kind, params, precision=req.precision)
                s.set_t_end(req.t_end)
                s.diag()                 # synchronises the thread's stream
            except Exception:
                s.close()
                raise
        return s

    def run(self, requests, clock=time.perf_counter):
        """Serves `requests` (arrival times relative to the start) to completion
        and returns ServeStats; each request gets its result (or error), t, step
        count and completion time."""
        for r in requests:
            if r.precision not in PRECISION:
                raise ValueError(f"request {r.id}: precision must be one of {sorted(PRECISION)}")
        pending = sorted(requests, key=lambda r: r.arrival)
        preparing = []                   # (request, future, footprint)
        import torch
        groups = {(p, c): _Group(self.device) for p in PRECISION for c in (0, 1)}

        def key(r):
            return (r.precision, 0 if r.n_cell < self.small_cells else 1)
        used = 0
        peak = rebuilds = launched = 0
        pool = ThreadPoolExecutor(max_workers=self.prepare_threads)
        t0 = clock()
        last_report = 0.0
        last_status = {}

        def say(msg):
            if self.progress is not None:
                self.progress(f"[{clock() - t0:8.3f} s] {msg}")
        def compact(g, new_members=()):
            # (re)builds g's batch from its active members and the joining ones; the
            # finished members, already read back, are freed.  Returns the bytes freed.
            nonlocal rebuilds
            if g.batch is not None:
                g.batch.close()
                g.batch = None
                g.event = None
            keep, freed = [], 0
            for m in g.members:
                if m[0].done is None:
                    keep.append(m)
                else:
                    m[1].close()
                    freed += m[2]
            g.members = keep + list(new_members)
            if g.members:
                with torch.cuda.stream(g.stream):
                    g.batch = Batch([s for _, s, _ in g.members])
                if self.autotune:
                    g.batch.autotune(reps=1)
                rebuilds += 1
            return freed

        def retire(g):
            # read back the members that finished since the group's last poll (its
            # steps have finished, so the status read does not wait)
            if g.batch is None:
                return
            _, status = g.batch.status()
            for (r, s, fp), st in zip(g.members, status):
                last_status[r.id] = (float(st[2]), int(st[3]), r.t_end)
                if r.done is None and st[0] == 0.0:
                    r.done = clock() - t0
                    r.t, r.steps = float(st[2]), int(st[3])
                    if st[1] != 0.0:
                        r.error = "a cell average left the admissible set"
                    if self.keep_results:
                        r.result = s.readback()[0]
                    say(f"request {r.id} done: {r.steps} steps to t = {r.t:.4g}, latency "
                        f"{r.latency * 1e3:.1f} ms{'' if r.error is None else ', ' + r.error}")

        ready = []                       # prepared, waiting for their group to be idle
        try:
            while pending or preparing or ready or any(g.active_count() or g.event is not None
                                                       for g in groups.values()):
                now = clock() - t0
                elapsed = now
                if elapsed - last_report >= self.progress_every:
                    last_report = elapsed
                    act = [f"{i}: t {v[0]:.4g}/{v[2]:.4g} step {v[1]}" for i, v in sorted(last_status.items())
                           if any(m[0].id == i and m[0].done is None for g in groups.values() for m in g.members)]
                    say(f"{launched} batched steps launched; active {act}; {len(pending)} pending, "
                        f"{len(preparing)} preparing")
                if self.max_wall is not None and elapsed > self.max_wall:
                    for r in requests:
                        if r.done is None:
                            r.error = f"not finished within {self.max_wall} s"
                            r.done = elapsed
                    say(f"stopped after {elapsed:.1f} s: {sum(1 for r in requests if r.error)} requests unfinished")
                    break
                # admission: arrived requests in arrival order while they fit; when the
                # budget blocks one, the finished members still held are freed first
                while pending and pending[0].arrival <= now:
                    r = pending[0]
                    fp = footprint_bytes(r.n_cell, r.k)
                    held = used > 0 or preparing
                    if held and used + fp > self.budget:
                        freed = 0
                        for g in groups.values():
                            if g.idle() and any(m[0].done is not None for m in g.members):
                                freed += compact(g)
                        used -= freed
                        if freed == 0 or used + fp > self.budget:
                            break
                    pending.pop(0)
                    r.admitted = now
                    preparing.append((r, pool.submit(self._prepare, r), fp))
                    used += fp
                    say(f"admit request {r.id}: {r.n_cell} cells P{r.k} {r.precision}, t_end {r.t_end:.4g}, "
                        f"{fp / 2**20:.0f} MiB, {used / 2**20:.0f} MiB held")
                # prepared requests wait for their group; failed ones finish with their error
                still = []
                for r, fut, fp in preparing:
                    if not fut.done():
                        still.append((r, fut, fp))
                        continue
                    try:
                        ready.append((r, fut.result(), fp))
                    except Exception as e:   # noqa: BLE001 - reported per request
                        r.error = f"admission failed: {e}"
                        r.done = clock() - t0
                        used -= fp
                        say(f"request {r.id} failed in preparation: {e}")
                preparing = still
                # every group whose last steps have finished: retire the members that
                # reached their t_end, let the waiting requests join, step again
                stepped = busy = False
                for gk, g in groups.items():
                    if not g.idle():
                        busy = True
                        continue
                    if g.event is not None:
                        g.event = None
                        retire(g)
                    joining = [x for x in ready if key(x[0]) == gk]
                    if joining:
                        ready = [x for x in ready if key(x[0]) != gk]
                        used -= compact(g, joining)
                        now2 = clock() - t0
                        for r, _, _ in joining:
                            r.joined = now2
                        say(f"{gk[0]} batch {'small' if gk[1] == 0 else 'large'} rebuilt: joined "
                            f"{[r.id for r, _, _ in joining]}, members {[m[0].id for m in g.members]}")
                    elif g.members and not g.active_count():
                        used -= compact(g)   # nothing left to step: free the finished ones
                    if g.batch is not None and g.active_count():
                        with torch.cuda.stream(g.stream):
                            g.batch.step(self.steps_per_tick)
                            g.event = torch.cuda.Event()
                            g.event.record(g.stream)
                        launched += self.steps_per_tick
                        stepped = True
                peak = max(peak, sum(g.active_count() for g in groups.values()))
                if not stepped:
                    if busy or preparing or ready:
                        time.sleep(0.0002)
                    elif pending:
                        wait = pending[0].arrival - (clock() - t0)
                        if wait > 0:
                            time.sleep(min(wait, 0.01))
        finally:
            pool.shutdown(wait=True)
            for r, fut, _ in preparing:          # prepared after a stop: never joined
                if fut.exception() is None:
                    fut.result().close()
            for r, sol, _ in ready:
                sol.close()
            for g in groups.values():
                if g.batch is not None:
                    g.batch.close()
                for m in g.members:
                    m[1].close()
        wall = clock() - t0
        lat = np.array([r.latency for r in requests])
        return ServeStats(wall=wall, requests=len(requests), p50=float(np.percentile(lat, 50)),
                          p99=float(np.percentile(lat, 99)), mean=float(lat.mean()),
                          dof_stage_per_s=sum(r.dof_stages for r in requests) / wall, peak_members=peak,
                          rebuilds=rebuilds, steps_launched=launched,
                          errors=sum(1 for r in requests if r.error is not None), latencies=lat.tolist())
