"""Continuous-batching request loop for independent HDG-IMEX time-stepping jobs
on one GPU.

A job is a mesh, its parameters, an initial velocity (a callable evaluated at
the library's cell points), a time step and a step count.  Jobs are admitted
as their device footprint (hdg_footprint_bytes, estimated on the host) fits
the memory budget next to the admitted ones; an admitted job gets its own
context on its own HIP stream, its state stays on the device, and worker
threads run it one implicit stage at a time (hdg_advance_stages), always
picking the admitted job with the least remaining work, so a short job that
arrives while a long one runs overtakes it at the next stage boundary, and
the workers' stages overlap on the device (the library calls release the
GIL).  Only the final state is copied back.  Every job's arithmetic is that
of a lone run: contexts share nothing, and any chunking into stages gives
the same bits.  run_fifo is the one-at-a-time baseline under the same
arrivals.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hdg


@dataclass(eq=False)
class Job:
    coords: np.ndarray
    cells: np.ndarray
    velocity: object              # callable (x, y) -> (..., 2)
    dt: float
    steps: int
    params: dict = field(default_factory=dict)
    vertex_rep: np.ndarray | None = None
    name: str = ""


@dataclass(eq=False)
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


def _stage_work(job: Job, trace_dofs: int) -> float:
    """Relative cost of one implicit stage, before any stage was timed: trace
    unknowns times a slowly growing factor (the Step I iterations grow with
    the mesh), plus a fixed launch-latency floor."""
    n = max(np.sqrt(len(job.cells) / 2.0), 1.0)
    return 2e-3 + 2.5e-9 * trace_dofs * (1.0 + n / 128.0)


class Server:
    """Continuous batching at stage granularity.

    Jobs are admitted (context created, state resident on the device) as
    their device footprint fits the budget beside the admitted ones, the one
    with the least estimated work first.  `workers` host threads then run
    implicit stages (hdg_advance_stages(ctx, dt, 1)): each picks, among the
    admitted jobs no other worker is running, by its policy the one with the
    least remaining work ("srpt": shortest remaining processing time,
    re-decided after every stage, so a short arrival overtakes a long job at
    its next stage boundary) or the earliest arrival ("fifo", so that long
    jobs keep progressing).  Each job has its own HIP stream, so the workers' stages
    overlap on the device.  Remaining work = remaining stages x the job's
    measured time per stage (estimated before its first stage).  Results
    are bit for bit those of a lone run (any chunking of hdg_advance_stages
    gives the same bits, and contexts share no buffers)."""

    def __init__(self, budget_bytes: int, workers: int = 2, slots: int = 16, policies=None, on_done=None):
        import torch
        if workers < 1 or slots < workers:
            raise ValueError("workers >= 1, slots >= workers")
        # per worker: "srpt" (least remaining work first, the default) or
        # "fifo" (earliest arrival first).  On the 26-job serving sample at
        # load 0.8 two srpt workers gave p50/p99 4.31/30.94 s against one srpt
        # and one fifo worker's 5.63/31.29 s (one-at-a-time FIFO: 10.96/30.92 s)
        self.policies = list(policies) if policies else ["srpt"] * workers
        if len(self.policies) != workers or any(p not in ("srpt", "fifo") for p in self.policies):
            raise ValueError("one policy, srpt or fifo, per worker")
        self.budget = int(budget_bytes)
        self.workers = workers
        self.slots = slots  # admitted (resident) jobs at most
        self._streams = [torch.cuda.Stream() for _ in range(slots)]
        self._cv = threading.Condition()
        self._waiting: list = []    # submitted, not admitted
        self._admitted: list = []   # resident, not finished
        self._stop = False
        self.in_use = 0
        self.max_in_use = 0
        self.max_active = 0
        self.results: list[Result] = []
        self.on_done = on_done  # called with each finished Result, from its worker thread
        self._t0 = time.perf_counter()
        self._threads = [threading.Thread(target=self._worker, args=(pol,), daemon=True) for pol in self.policies]
        for t in self._threads:
            t.start()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, job: Job) -> Result:
        res = Result(job, arrival=self.now())
        p = dict(job.params)
        res.footprint = hdg.footprint_bytes(job.coords, job.cells, job.dt, job.vertex_rep, **p)
        res.stages = implicit_stages(p.get("imex", "ars222"))
        ncell = len(job.cells)
        k = int(p.get("degree", 1))
        res.trace_dofs = (3 * ncell // 2 + int(2 * np.sqrt(ncell / 2))) * (k + 1)  # split-square estimate
        res._left = job.steps * res.stages                 # stages still to run
        res._per_stage = _stage_work(job, res.trace_dofs)  # seconds per stage, refined as stages run
        res._running = False
        res._ctx = None
        res._stream = None
        with self._cv:
            self.results.append(res)
            if res.footprint > self.budget:
                res.error = f"footprint {res.footprint} B exceeds the budget {self.budget} B"
                res.start = res.end = res.arrival
            else:
                self._waiting.append(res)
                self._admit()
                self._cv.notify_all()
        return res

    @staticmethod
    def _work(res) -> float:
        return res._left * res._per_stage

    def _admit(self):
        # caller holds the lock: least estimated work first, while it fits
        self._waiting.sort(key=self._work)
        while (self._waiting and len(self._admitted) < self.slots and
               self.in_use + self._waiting[0].footprint <= self.budget):
            res = self._waiting.pop(0)
            self.in_use += res.footprint
            self.max_in_use = max(self.max_in_use, self.in_use)
            res._stream = self._streams.pop()
            self._admitted.append(res)

    def _worker(self, policy: str):
        key = self._work if policy == "srpt" else (lambda r: r.arrival)
        while True:
            with self._cv:
                while True:
                    if self._stop:
                        return
                    ready = [r for r in self._admitted if not r._running]
                    if ready:
                        res = min(ready, key=key)
                        res._running = True
                        self.max_active = max(self.max_active, sum(r._running for r in self._admitted))
                        break
                    self._cv.wait()
            done = False
            try:
                t0 = time.perf_counter()
                if res._ctx is None:
                    res.start = self.now()
                    job = res.job
                    res._ctx = hdg.Context(job.coords, job.cells, stream=res._stream, vertex_rep=job.vertex_rep,
                                           **job.params)
                    xy = res._ctx.cell_points()
                    res._ctx.set_velocity_from_points(job.velocity(xy[..., 0], xy[..., 1]))
                    res.trace_dofs = res._ctx.nT
                else:
                    res._ctx.advance_stages(res.job.dt, 1)
                    res._left -= 1
                    el = time.perf_counter() - t0
                    res._per_stage = el if res._left == res.job.steps * res.stages - 1 else \
                        0.5 * (res._per_stage + el)
                if res._left == 0:
                    res.state = tuple(t.cpu().numpy() for t in res._ctx.get_state())
                    done = True
            except Exception as e:  # reported per job
                res.error = str(e)
                done = True
            if done:
                if res._ctx is not None:
                    res._ctx.close()
                    res._ctx = None
                res.end = self.now()
            with self._cv:
                res._running = False
                if done:
                    self._admitted = [r for r in self._admitted if r is not res]
                    self.in_use -= res.footprint
                    self._streams.append(res._stream)
                    self._admit()
                self._cv.notify_all()
            if done and self.on_done is not None:
                self.on_done(res)

    def drain(self, timeout: float | None = None):
        """Wait until every submitted job has finished, then stop the workers."""
        deadline = None if timeout is None else time.perf_counter() + timeout
        with self._cv:
            while self._waiting or self._admitted:
                left = None if deadline is None else deadline - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("jobs still running")
                self._cv.wait(left)
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()


def run_fifo(jobs, arrivals, clock=time.perf_counter, progress=None) -> list:
    """The baseline: one job at a time in arrival order (FP64 contexts on the
    current stream), each started at its arrival or when the previous one has
    finished.  Returns [(arrival, start, end)] in seconds from the first
    arrival; progress(i, (arrival, start, end)) is called after each job."""
    import torch
    out = []
    t0 = clock()
    for a, job in zip(arrivals, jobs):
        wait = a - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        start = clock() - t0
        ctx = hdg.Context(job.coords, job.cells, vertex_rep=job.vertex_rep, **job.params)
        xy = ctx.cell_points()
        ctx.set_velocity_from_points(job.velocity(xy[..., 0], xy[..., 1]))
        ctx.advance(job.dt, job.steps)
        _ = ctx.get_state()[0].cpu()
        ctx.close()
        torch.cuda.synchronize()
        out.append((a, start, clock() - t0))
        if progress is not None:
            progress(len(out), out[-1])
    return out


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
