"""Continuous-batching request loop for independent HDG-IMEX time-stepping jobs
on one GPU.

A job is a mesh, its parameters, an initial velocity (a callable evaluated at
the library's cell points), a time step and a step count.  Jobs are admitted
in arrival order as soon as a slot is free and their device footprint
(hdg_footprint_bytes, estimated on the host) fits the memory budget next to
the jobs already running; an admitted job gets its own context on its own
HIP stream and runs on a worker thread, so jobs that arrive while others are
on the GPU overlap with them there (the library calls release the GIL).  The
state stays on the device between steps; only the final state is copied
back.  Every job's arithmetic is that of a lone run: contexts share nothing.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hdg


@dataclass
class Job:
    coords: np.ndarray
    cells: np.ndarray
    velocity: object              # callable (x, y) -> (..., 2)
    dt: float
    steps: int
    params: dict = field(default_factory=dict)
    vertex_rep: np.ndarray | None = None
    name: str = ""


@dataclass
class Result:
    job: Job
    arrival: float
    start: float = 0.0
    end: float = 0.0
    footprint: int = 0
    state: tuple | None = None    # (Q, p, lam) as host arrays
    trace_dofs: int = 0
    stages: int = 0               # implicit stages per step
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.end - self.arrival


def implicit_stages(imex: str) -> int:
    return {"imex_euler": 1, "ars222": 2, "ars233": 2, "ssp2_332": 3, "ssp3_433": 3}[imex]


class Server:
    """Admits jobs FIFO by free slot and device-memory budget (bytes)."""

    def __init__(self, budget_bytes: int, slots: int = 8):
        import torch
        if slots < 1:
            raise ValueError("slots >= 1")
        self.budget = int(budget_bytes)
        self.slots = slots
        self._free_streams = [torch.cuda.Stream() for _ in range(slots)]
        self._cv = threading.Condition()
        self._queue: deque = deque()
        self._threads: list = []
        self.in_use = 0
        self.max_in_use = 0
        self.active = 0
        self.max_active = 0
        self.results: list[Result] = []
        self._t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, job: Job) -> Result:
        res = Result(job, arrival=self.now())
        p = dict(job.params)
        res.footprint = hdg.footprint_bytes(job.coords, job.cells, job.dt, job.vertex_rep, **p)
        with self._cv:
            self.results.append(res)
            if res.footprint > self.budget:
                res.error = f"footprint {res.footprint} B exceeds the budget {self.budget} B"
                res.start = res.end = res.arrival
            else:
                self._queue.append(res)
                self._admit()
        return res

    def _admit(self):
        # caller holds the lock; FIFO: the head waits until it fits
        while self._queue and self.active < self.slots and self.in_use + self._queue[0].footprint <= self.budget:
            res = self._queue.popleft()
            self.in_use += res.footprint
            self.active += 1
            self.max_in_use = max(self.max_in_use, self.in_use)
            self.max_active = max(self.max_active, self.active)
            stream = self._free_streams.pop()
            t = threading.Thread(target=self._run, args=(res, stream), daemon=True)
            self._threads.append(t)
            t.start()

    def _run(self, res: Result, stream):
        res.start = self.now()
        job = res.job
        ctx = None
        try:
            ctx = hdg.Context(job.coords, job.cells, stream=stream, vertex_rep=job.vertex_rep, **job.params)
            xy = ctx.cell_points()
            ctx.set_velocity_from_points(job.velocity(xy[..., 0], xy[..., 1]))
            ctx.advance(job.dt, job.steps)
            res.state = tuple(t.cpu().numpy() for t in ctx.get_state())
            res.trace_dofs = ctx.nT
            res.stages = implicit_stages(job.params.get("imex", "ars222"))
        except Exception as e:  # reported per job
            res.error = str(e)
        finally:
            if ctx is not None:
                ctx.close()
            res.end = self.now()
            with self._cv:
                self.in_use -= res.footprint
                self.active -= 1
                self._free_streams.append(stream)
                self._admit()
                self._cv.notify_all()

    def drain(self, timeout: float | None = None):
        """Wait until every submitted job has finished."""
        deadline = None if timeout is None else time.perf_counter() + timeout
        with self._cv:
            while self._queue or self.active:
                left = None if deadline is None else deadline - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("jobs still running")
                self._cv.wait(left)
        for t in self._threads:
            t.join()


def run_alone(job: Job) -> tuple[float, tuple, int]:
    """The job by itself on the current stream: (seconds, final state, trace DOFs)."""
    import torch
    t0 = time.perf_counter()
    ctx = hdg.Context(job.coords, job.cells, vertex_rep=job.vertex_rep, **job.params)
    xy = ctx.cell_points()
    ctx.set_velocity_from_points(job.velocity(xy[..., 0], xy[..., 1]))
    ctx.advance(job.dt, job.steps)
    state = tuple(t.cpu().numpy() for t in ctx.get_state())
    nT = ctx.nT
    ctx.close()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, state, nT


def percentiles(values, qs=(50, 99)):
    v = np.asarray(values, dtype=np.float64)
    return {f"p{q}": float(np.percentile(v, q)) for q in qs}
