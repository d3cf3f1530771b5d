"""Continuous-batching server for spectrum-synthesis requests.

A request is one ejecta model (shells, lines, Sobolev depths) and a number
of Monte Carlo iterations (Kerzendorf & Sim 2014, section 2.8: each
iteration re-derives T_inner from the emergent luminosity).  The server
admits requests in arrival order while their device workspaces fit in a
memory budget, and advances every admitted request by one iteration per
step in ONE multi-model launch (smc_batch_run), so requests that arrive
while others are running join at the next step and their work overlaps on
the device.  Model state (inputs, tallies, T_inner) stays resident on the
device between iterations; a request's workspace is released when its last
iteration is read back.

The device work goes through a backend object; `GpuBackend` drives libsmc.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

QUEUED, RUNNING, DONE, CANCELLED, REJECTED = "queued", "running", "done", "cancelled", "rejected"


@dataclasses.dataclass(eq=False)
class Request:
    model: object                 # workloads.Model (host arrays)
    n_iterations: int
    n_packets: int
    T_inner: float
    L_requested: float = 0.0
    damping: float = 0.5
    arrival: float = 0.0          # seconds after the server's start
    rid: int = -1
    # filled in by the server
    state: str = QUEUED
    admitted_at: Optional[float] = None
    completed_at: Optional[float] = None
    iteration: int = 0
    handle: object = None
    bytes: int = 0
    result: Optional[dict] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed_at is None else self.completed_at - self.arrival


class GpuBackend:
    """libsmc on one GPU: a context, per-request device workspaces, one
    multi-model launch per step."""

    def __init__(self, device: int = 0, flags: Optional[int] = None, tune: Optional[dict] = None):
        from . import smc
        self.smc = smc
        self.ctx = smc.Context(device)
        self.flags = smc.F_JBLUE if flags is None else flags
        self.tune = tune

    def workspace_bytes(self, req: Request) -> int:
        return self.smc.workspace_bytes(req.model, req.n_packets, self.flags)

    def load(self, req: Request):
        return self.smc.Model(self.ctx, req.model, req.n_packets, flags=self.flags)

    def free(self, handle) -> None:
        handle.free()
        handle.workspace = None

    def step(self, reqs: List[Request]) -> None:
        params = [dict(n_packets=r.n_packets, T_inner=r.T_inner if r.iteration == 0 else 0.0,
                       iteration=r.iteration, flags=self.flags, L_requested=r.L_requested,
                       damping=r.damping) for r in reqs]
        handles = [r.handle for r in reqs]
        if len(handles) == 1:
            handles[0].run_iteration(**params[0])
        else:
            self.ctx.batch_run(handles, params, tune=self.tune)

    def sync(self) -> None:
        import torch
        torch.cuda.synchronize()

    def result(self, req: Request) -> dict:
        m = req.handle
        est = m.read_estimators(jblue=bool(self.flags & self.smc.F_JBLUE))
        spec = m.read_spectrum()
        return dict(J=est["J"], nubar=est["nubar"], T_R=est["T_R"], W=est["W"],
                    jblue=est["jblue"], L_nu=spec["L_nu"], L_emitted=spec["L_emitted"],
                    T_inner=spec["T_inner"], T_inner_next=spec["T_inner_next"],
                    counters=m.read_counters())


class Server:
    """Admission by device-memory budget, continuous batching, FIFO order.

    `clock` returns seconds since an arbitrary origin; `sleep(dt)` waits (a
    simulated clock may advance instead)."""

    def __init__(self, backend, memory_budget: int, max_active: int = 1024,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.backend = backend
        self.budget = int(memory_budget)
        self.max_active = int(max_active)
        self.clock = clock
        self.sleep = sleep
        self.t0 = clock()
        self.pending: List[Request] = []   # arrived or future, arrival order
        self.active: List[Request] = []
        self.requests: Dict[int, Request] = {}
        self.in_use = 0
        self.steps = 0
        self.step_sizes: List[int] = []
        self._next_id = 0

    def now(self) -> float:
        return self.clock() - self.t0

    # ---- request API
    def submit(self, req: Request) -> int:
        req.rid = self._next_id
        self._next_id += 1
        req.bytes = self.backend.workspace_bytes(req)
        self.requests[req.rid] = req
        if req.bytes > self.budget:
            req.state = REJECTED
            return req.rid
        req.state = QUEUED
        # keep pending in arrival order (stable for equal arrival times)
        i = len(self.pending)
        while i > 0 and self.pending[i - 1].arrival > req.arrival:
            i -= 1
        self.pending.insert(i, req)
        return req.rid

    def poll(self, rid: int) -> str:
        return self.requests[rid].state

    def result(self, rid: int) -> Optional[dict]:
        return self.requests[rid].result

    def wait(self, rid: int) -> Optional[dict]:
        """Serve (every admitted request advances with it) until request rid
        has finished, been cancelled or been rejected; its result, if any."""
        req = self.requests[rid]
        while req.state in (QUEUED, RUNNING):
            if not self.step():
                if not self.pending:
                    break
                self.sleep(max(0.0, self.pending[0].arrival - self.now()))
        return req.result

    def cancel(self, rid: int) -> bool:
        req = self.requests[rid]
        if req.state == QUEUED:
            self.pending.remove(req)
        elif req.state == RUNNING:
            self.active.remove(req)
            self._release(req)
        else:
            return False
        req.state = CANCELLED
        return True

    # ---- scheduling
    def _release(self, req: Request) -> None:
        if req.handle is not None:
            self.backend.free(req.handle)
            req.handle = None
        self.in_use -= req.bytes

    def _admit(self) -> None:
        now = self.now()
        while self.pending and self.pending[0].arrival <= now:
            req = self.pending[0]
            if len(self.active) >= self.max_active or self.in_use + req.bytes > self.budget:
                break  # FIFO: later arrivals wait behind the head
            self.pending.pop(0)
            req.handle = self.backend.load(req)
            self.in_use += req.bytes
            req.state = RUNNING
            req.admitted_at = now
            self.active.append(req)

    def step(self) -> bool:
        """Admit what fits, run one iteration of every admitted request, and
        complete the finished ones.  Returns False when nothing ran."""
        self._admit()
        if not self.active:
            return False
        batch = list(self.active)
        self.backend.step(batch)
        self.backend.sync()
        self.steps += 1
        self.step_sizes.append(len(batch))
        t = self.now()
        for req in batch:
            req.iteration += 1
            if req.iteration >= req.n_iterations:
                req.result = self.backend.result(req)
                req.completed_at = t
                req.state = DONE
                self.active.remove(req)
                self._release(req)
        return True

    def run(self) -> None:
        """Serve until every submitted request is finished."""
        while self.pending or self.active:
            if not self.step():
                nxt = self.pending[0].arrival if self.pending else None
                if nxt is not None:
                    self.sleep(max(0.0, nxt - self.now()))

    # ---- reporting
    def stats(self) -> dict:
        done = [r for r in self.requests.values() if r.state == DONE]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        span = (max(r.completed_at for r in done) - min(r.arrival for r in done)) if done else 0.0
        return dict(completed=len(done),
                    rejected=sum(r.state == REJECTED for r in self.requests.values()),
                    p50_s=float(np.percentile(lat, 50)) if lat.size else None,
                    p99_s=float(np.percentile(lat, 99)) if lat.size else None,
                    mean_s=float(lat.mean()) if lat.size else None,
                    models_per_s=len(done) / span if span > 0 else None,
                    steps=self.steps,
                    mean_batch=float(np.mean(self.step_sizes)) if self.step_sizes else 0.0,
                    max_batch=int(max(self.step_sizes)) if self.step_sizes else 0)


def serve_plain(backend, reqs: List[Request], clock=time.perf_counter, sleep=time.sleep) -> dict:
    """The per-request path: one request at a time in arrival order, each
    iteration a single-model launch.  Latency = completion - arrival."""
    t0 = clock()
    done = []
    for req in sorted(reqs, key=lambda r: r.arrival):
        wait = req.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        req.bytes = backend.workspace_bytes(req)
        req.handle = backend.load(req)
        req.admitted_at = clock() - t0
        for it in range(req.n_iterations):
            req.iteration = it
            backend.step([req])
        backend.sync()
        req.iteration = req.n_iterations
        req.result = backend.result(req)
        req.completed_at = clock() - t0
        req.state = DONE
        backend.free(req.handle)
        req.handle = None
        done.append(req)
    lat = np.array([r.latency for r in done])
    span = max(r.completed_at for r in done) - min(r.arrival for r in done)
    return dict(completed=len(done), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                models_per_s=len(done) / span if span > 0 else None)
