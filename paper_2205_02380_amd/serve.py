"""Continuous-batching server for advection jobs.

Requests (grid, step count, dt, seeded initial packets) arrive over time.  A request is
admitted when its arrival time has passed, a slot is free and its device memory (the
FP32 field plus the library's workspace) fits in the HBM budget; admission is FIFO, so
a request that does not fit yet blocks the ones behind it (no starvation).  Resident
jobs are grouped into shape classes (grid and kernel shape); each class has a stream of
its own and advances all its jobs by one step through one `chasm_advect_step_many`
call, in which they share launches.  Classes run concurrently: the host issues a class's
next step as soon as its previous one has completed (detected by polling an event
recorded after it, never by synchronising a stream), so a small class is not held back
by a large one.  Jobs whose steps are done retire (their FP64 diagnostics are read, a
non-finite mass marks the job failed) and free their memory for the next admissions.
Fields stay resident on the device for the whole life of a job.

The scheduling here is host logic only; all device work goes through the C ABI.  The
backend is pluggable: `ChasmBackend` runs on the GPU, `FakeBackend` simulates step
times on a virtual clock (one device executing the classes' steps in launch order) so
the scheduling invariants can be tested without a GPU.

Step latency of a job = the interval between two consecutive step completions of that
job (the first one counts from admission); the report gives p50/p99 over all jobs and
per shape class.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from .inputs import Request


@dataclasses.dataclass
class JobState:
    req: Request
    handle: object
    nbytes: int
    admitted: float
    last: float
    cls: tuple = ()
    done_steps: int = 0
    latencies: List[float] = dataclasses.field(default_factory=list)
    failed: bool = False
    mass: Optional[float] = None


@dataclasses.dataclass
class ServeReport:
    completed: int
    failed: int
    rejected: int
    point_updates: float
    makespan_s: float
    throughput: float                 # point-updates per second over the makespan
    p50_step_ms: float
    p99_step_ms: float
    max_resident_bytes: int
    max_active: int
    ticks: int                        # class steps issued (one step of every job of a class)
    mean_queue_s: float
    per_class: Dict[str, dict]        # p50/p99 step latency (ms) and steps per shape class
    results: Dict[int, dict]

    def as_dict(self) -> dict:
        d = dataclasses.asdict(self)
        d.pop("results")
        return d


class ChasmBackend:
    """GPU backend: fields are torch tensors on `device`, stepping goes through libchasm;
    one stream per shape class (default priority)."""

    def __init__(self, device: str = "cuda:0", keep: Sequence[int] = (), nan_rids: Sequence[int] = (),
                 poll_s: float = 20e-6):
        import torch

        from . import chasm
        self.torch = torch
        self.chasm = chasm
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.streams: Dict[tuple, object] = {}
        self.keep = set(keep)
        self.nan = set(nan_rids)          # fault injection: these fields start with a NaN
        self.kept: Dict[int, object] = {}
        self.poll_s = poll_s

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float) -> None:
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def class_of(self, req: Request, patch, ghost) -> tuple:
        return (tuple(req.grid.nx), tuple(req.grid.nk), patch, ghost)

    def bytes_needed(self, req: Request, patch, ghost) -> int:
        desc = self.chasm.make_desc(req.grid, patch, ghost, req.dt)
        return req.grid.points * 4 + self.chasm.chasm_advect_workspace_bytes(desc)

    def admit(self, req: Request, patch, ghost):
        from . import inputs
        cls = self.class_of(req, patch, ghost)
        st = self.streams.get(cls)
        if st is None:
            st = self.streams[cls] = self.torch.cuda.Stream(self.device)
        with self.torch.cuda.stream(st):
            f = self.torch.empty(req.grid.shape(), dtype=self.torch.float32, device=self.device)
            coef, gx, gk = inputs.packet_factors(req.grid, req.packets)
            inputs.fill_separable(f, coef, gx, gk)
            if req.rid in self.nan:
                f.view(-1)[f.numel() // 2] = float("nan")
        return self.chasm.Advect(f, req.grid, patch, ghost, req.dt, stream=st)

    def launch(self, cls: tuple, handles: List[object]):
        """Issue one step of every job of a class on the class's stream; returns the
        event that completes with it."""
        self.chasm.step_many(handles, [1] * len(handles))
        ev = self.torch.cuda.Event()
        ev.record(self.streams[cls])
        return ev

    def wait_any(self, inflight: Dict[tuple, object], deadline: Optional[float]) -> List[tuple]:
        """Poll the in-flight classes' events until at least one has completed (or the
        deadline, an absolute time, passes); returns the completed classes."""
        while True:
            done = [c for c, ev in inflight.items() if ev.query()]
            if done or (deadline is not None and time.perf_counter() >= deadline):
                return done
            time.sleep(self.poll_s)

    def retire(self, job: JobState) -> dict:
        m, l2, mom = job.handle.mass()
        if job.req.rid in self.keep:
            self.kept[job.req.rid] = job.handle.f.detach().clone()
        job.handle.close()
        return {"mass": m, "l2": l2}

    def release(self, job: JobState) -> None:
        job.handle.f = None


class FakeBackend:
    """Host-only backend: a virtual clock; one simulated device runs the classes' steps in
    launch order, each taking launch_s + points x seconds per point."""

    def __init__(self, sec_per_point: float = 2e-12, launch_s: float = 20e-6, workspace: int = 1 << 20,
                 nan_rids: Sequence[int] = ()):
        self.t = 0.0
        self.sec_per_point = sec_per_point
        self.launch_s = launch_s
        self.workspace = workspace
        self.nan = set(nan_rids)
        self.live: Dict[int, int] = {}
        self.device_free = 0.0

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float) -> None:
        self.t = max(self.t, t)

    def class_of(self, req: Request, patch, ghost) -> tuple:
        return (tuple(req.grid.nx), tuple(req.grid.nk), patch, ghost)

    def bytes_needed(self, req: Request, patch, ghost) -> int:
        return req.grid.points * 4 + self.workspace

    def admit(self, req: Request, patch, ghost):
        self.live[req.rid] = req.grid.points
        return req.rid

    def launch(self, cls: tuple, handles: List[object]) -> float:
        start = max(self.t, self.device_free)
        self.device_free = start + self.launch_s + sum(self.live[h] for h in handles) * self.sec_per_point
        return self.device_free

    def wait_any(self, inflight: Dict[tuple, float], deadline: Optional[float]) -> List[tuple]:
        first = min(inflight.values())
        if deadline is not None and deadline < first:
            self.t = max(self.t, deadline)
            return []
        self.t = max(self.t, first)
        return sorted(c for c, end in inflight.items() if end <= self.t)

    def retire(self, job: JobState) -> dict:
        del self.live[job.handle]
        return {"mass": float("nan") if job.req.rid in self.nan else 1.0, "l2": 1.0}

    def release(self, job: JobState) -> None:
        pass


class Server:
    def __init__(self, backend, budget_bytes: float = 200e9, max_active: int = 64, patch=8, ghost: int = 6):
        self.backend = backend
        self.budget = float(budget_bytes)
        self.max_active = int(max_active)
        self.patch = patch
        self.ghost = ghost

    def run(self, trace: Sequence[Request], cancel_at: Optional[Dict[int, int]] = None) -> ServeReport:
        """Serve the trace to completion.  cancel_at[rid] = k cancels job rid after k steps."""
        be = self.backend
        cancel_at = cancel_at or {}
        pending = collections.deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        t0 = be.now()
        classes: Dict[tuple, List[JobState]] = collections.OrderedDict()   # resident jobs per class
        inflight: Dict[tuple, object] = {}                                  # class -> its step's token
        stepping: Dict[tuple, List[JobState]] = {}                          # the jobs of that step
        used = 0
        max_used = 0
        max_active = 0
        rejected = 0
        completed = 0
        failed = 0
        ticks = 0
        pupd = 0.0
        lat: List[float] = []
        lat_cls: Dict[tuple, List[float]] = collections.defaultdict(list)
        queue: List[float] = []
        results: Dict[int, dict] = {}
        last_done = t0

        def n_active():
            return sum(len(v) for v in classes.values())

        while pending or n_active():
            now = be.now() - t0
            while pending and pending[0].arrival <= now and n_active() < self.max_active:
                req = pending[0]
                need = be.bytes_needed(req, self.patch, self.ghost)
                if need > self.budget:
                    pending.popleft()            # can never fit: reject
                    rejected += 1
                    results[req.rid] = {"status": "rejected", "bytes": need}
                    continue
                if used + need > self.budget:
                    break                        # FIFO: wait for memory
                pending.popleft()
                handle = be.admit(req, self.patch, self.ghost)
                t = be.now()
                cls = be.class_of(req, self.patch, self.ghost)
                classes.setdefault(cls, []).append(JobState(req, handle, need, admitted=t, last=t, cls=cls))
                used += need
                queue.append(t - t0 - req.arrival)
                max_used = max(max_used, used)
            max_active = max(max_active, n_active())
            # every class with resident jobs and no step in flight issues its next step
            for cls, jobs in classes.items():
                if jobs and cls not in inflight:
                    stepping[cls] = list(jobs)
                    inflight[cls] = be.launch(cls, [j.handle for j in jobs])
                    ticks += 1
            if not inflight:
                if pending:
                    be.wait_until(t0 + pending[0].arrival)
                continue
            # wait for a class to finish its step, or for the next arrival (a future one that
            # a free slot could take; one already waiting on memory waits for a retirement)
            deadline = None
            if pending and n_active() < self.max_active and t0 + pending[0].arrival > be.now():
                deadline = t0 + pending[0].arrival
            done = be.wait_any(inflight, deadline)
            t = be.now()
            for cls in done:
                del inflight[cls]
                still = []
                for j in stepping.pop(cls):
                    j.done_steps += 1
                    j.latencies.append(t - j.last)
                    j.last = t
                    pupd += j.req.grid.points
                    stop = cancel_at.get(j.req.rid)
                    if j.done_steps >= j.req.steps or (stop is not None and j.done_steps >= stop):
                        info = be.retire(j)
                        be.release(j)
                        used -= j.nbytes
                        lat.extend(j.latencies)
                        lat_cls[cls].extend(j.latencies)
                        ok = np.isfinite(info["mass"])
                        cancelled = stop is not None and j.done_steps < j.req.steps
                        status = "cancelled" if cancelled else ("done" if ok else "failed")
                        if status == "failed":
                            failed += 1
                        elif status == "done":
                            completed += 1
                        results[j.req.rid] = dict(status=status, steps=j.done_steps, mass=info["mass"],
                                                  admitted=j.admitted - t0, finished=t - t0)
                        last_done = t
                    else:
                        still.append(j)
                # jobs admitted while this step ran stay in the class; retired ones leave
                gone = {id(j) for j in classes[cls] if j.done_steps >= j.req.steps or
                        (cancel_at.get(j.req.rid) is not None and j.done_steps >= cancel_at[j.req.rid])}
                classes[cls] = [j for j in classes[cls] if id(j) not in gone]
        makespan = last_done - t0
        lat_ms = np.array(lat) * 1e3 if lat else np.zeros(1)
        per_class = {}
        for cls, v in lat_cls.items():
            a = np.array(v) * 1e3
            per_class["x".join(map(str, cls[0])) + "/" + "x".join(map(str, cls[1]))] = {
                "p50_step_ms": float(np.percentile(a, 50)), "p99_step_ms": float(np.percentile(a, 99)),
                "job_steps": int(a.size)}
        return ServeReport(
            completed=completed, failed=failed, rejected=rejected, point_updates=pupd,
            makespan_s=makespan, throughput=pupd / makespan if makespan > 0 else 0.0,
            p50_step_ms=float(np.percentile(lat_ms, 50)), p99_step_ms=float(np.percentile(lat_ms, 99)),
            max_resident_bytes=int(max_used), max_active=max_active, ticks=ticks,
            mean_queue_s=float(np.mean(queue)) if queue else 0.0, per_class=per_class, results=results)
