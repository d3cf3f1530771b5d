"""Continuous-batching servers for spectrum-synthesis requests.

A request is one ejecta model (shells, lines, Sobolev depths) and a number
of Monte Carlo iterations (Kerzendorf & Sim 2014, section 2.8: each
iteration re-derives T_inner from the emergent luminosity).  Both servers
admit requests in arrival order while their device workspaces fit in a
memory budget and keep model state (inputs, tallies, T_inner) resident on
the device between iterations; a request's workspace is released when its
last iteration is read back.

`Server` advances every admitted request by one iteration per step in ONE
multi-model launch (smc_batch_run) and waits for it: a request that arrives
mid-step, and every request of the step, waits for the step's slowest
history (head-of-line blocking).

`StreamServer` has no global step: several launch streams run cohorts
concurrently, an idle stream launches every ready request at once (admitted,
not in flight), and a cohort's requests advance when their own launch ends.
A new arrival waits only for a free stream, and the long tail of one launch
overlaps the bulk of the next on the device.

The device work goes through a backend object; `GpuBackend` drives libsmc.
Per request the servers record the queue wait (arrival to first launch),
the service time (first launch to completion) and the time it spent ready
between iterations without running.
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
    first_launch_at: Optional[float] = None
    ready_at: Optional[float] = None   # when its next iteration became launchable
    ready_wait: float = 0.0            # time spent launchable but not running
    in_flight: bool = False

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed_at is None else self.completed_at - self.arrival

    @property
    def queue_wait(self) -> Optional[float]:
        return None if self.first_launch_at is None else self.first_launch_at - self.arrival

    @property
    def service(self) -> Optional[float]:
        if self.completed_at is None or self.first_launch_at is None:
            return None
        return self.completed_at - self.first_launch_at

    def launched(self, t: float) -> None:
        if self.first_launch_at is None:
            self.first_launch_at = t
        elif self.ready_at is not None:
            self.ready_wait += t - self.ready_at


class GpuBackend:
    """libsmc on one GPU: a context, per-request device workspaces, one
    multi-model launch per step (or per cohort, on a launch stream).  Models
    are uploaded on a stream of their own, so that loading a request never
    waits for launches in flight.  keep_jblue=False leaves a result's J_blue
    (shells x lines) on the device instead of reading it back."""

    def __init__(self, device: int = 0, flags: Optional[int] = None, tune: Optional[dict] = None,
                 keep_jblue: bool = True):
        import torch

        from . import smc
        self.smc = smc
        self.device = device
        self.ctx = smc.Context(device)
        self.flags = smc.F_JBLUE if flags is None else flags
        self.tune = tune
        self.keep_jblue = keep_jblue
        self.upload = torch.cuda.Stream(device=device)

    def workspace_bytes(self, req: Request) -> int:
        return self.smc.workspace_bytes(req.model, req.n_packets, self.flags)

    def load(self, req: Request):
        import torch
        with torch.cuda.stream(self.upload):
            return self.smc.Model(self.ctx, req.model, req.n_packets, flags=self.flags,
                                  stream=self.upload)

    def free(self, handle) -> None:
        handle.free()
        handle.workspace = None

    def _params(self, reqs):
        return [dict(n_packets=r.n_packets, T_inner=r.T_inner if r.iteration == 0 else 0.0,
                     iteration=r.iteration, flags=self.flags, L_requested=r.L_requested,
                     damping=r.damping) for r in reqs]

    def step(self, reqs: List[Request], stream=None) -> None:
        params = self._params(reqs)
        handles = [r.handle for r in reqs]
        if len(handles) == 1:
            handles[0].run_iteration(**params[0], stream=stream)
        else:
            self.ctx.batch_run(handles, params, tune=self.tune, stream=stream)

    def sync(self) -> None:
        import torch
        torch.cuda.synchronize()

    # ---- launch streams (StreamServer)
    def stream(self, k: int):
        import torch
        return torch.cuda.Stream(device=self.device)  # default priority

    def launch(self, reqs: List[Request], stream):
        """Enqueue one iteration of reqs on `stream`; returns an event that
        completes with it."""
        import torch
        self.step(reqs, stream)
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    def query(self, ev) -> bool:
        return ev.query()

    def result(self, req: Request, stream=None) -> dict:
        m = req.handle
        jb = bool(self.flags & self.smc.F_JBLUE) and self.keep_jblue
        est = m.read_estimators(jblue=jb, stream=stream)
        spec = m.read_spectrum(stream=stream)
        out = dict(J=est["J"], nubar=est["nubar"], T_R=est["T_R"], W=est["W"],
                   jblue=est["jblue"], L_nu=spec["L_nu"], L_emitted=spec["L_emitted"],
                   T_inner=spec["T_inner"], T_inner_next=spec["T_inner_next"],
                   counters=m.read_counters(stream=stream))
        return out


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
        t0 = self.now()
        for req in batch:
            req.launched(t0)
        self.backend.step(batch)
        self.backend.sync()
        self.steps += 1
        self.step_sizes.append(len(batch))
        t = self.now()
        for req in batch:
            req.iteration += 1
            req.ready_at = t
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
        return dict(**latency_stats(done),
                    rejected=sum(r.state == REJECTED for r in self.requests.values()),
                    steps=self.steps,
                    mean_batch=float(np.mean(self.step_sizes)) if self.step_sizes else 0.0,
                    max_batch=int(max(self.step_sizes)) if self.step_sizes else 0)


def latency_stats(done: List[Request]) -> dict:
    """Completed requests: latency (arrival to completion), queue wait
    (arrival to first launch) and service time (first launch to completion)
    at p50 / p99 / mean, the time ready between iterations without running,
    and models/s over the span from the first arrival to the last
    completion."""
    def pct(x):
        x = np.asarray([v for v in x if v is not None], dtype=np.float64)
        if not x.size:
            return dict(p50=None, p99=None, mean=None)
        return dict(p50=float(np.percentile(x, 50)), p99=float(np.percentile(x, 99)),
                    mean=float(x.mean()))
    lat = pct(r.latency for r in done)
    span = (max(r.completed_at for r in done) - min(r.arrival for r in done)) if done else 0.0
    return dict(completed=len(done), p50_s=lat["p50"], p99_s=lat["p99"], mean_s=lat["mean"],
                models_per_s=len(done) / span if span > 0 else None,
                queue_wait_s=pct(r.queue_wait for r in done),
                service_s=pct(r.service for r in done),
                ready_wait_per_iteration_s=pct(r.ready_wait / max(r.n_iterations - 1, 1)
                                               for r in done))


class StreamServer(Server):
    """Continuous batching on n_streams launch streams with no global step.
    Each scheduling round completes the cohorts whose launches have ended
    (their requests advance one iteration; finished ones are read back and
    released), admits what fits, and gives every idle stream the ready
    requests (admitted and not in flight), at most max_cohort per launch in
    arrival order.  A request is in at most one launch at a time, so its
    iterations stay in order."""

    def __init__(self, backend, memory_budget: int, n_streams: int = 4, max_cohort: int = 1024,
                 poll_s: float = 0.0005, **kw):
        super().__init__(backend, memory_budget, **kw)
        self.lanes = [backend.stream(k) for k in range(n_streams)]
        self.inflight: List[Optional[tuple]] = [None] * n_streams
        self.max_cohort = int(max_cohort)
        self.poll_s = float(poll_s)
        self.concurrency: List[int] = []

    def _complete(self) -> bool:
        any_done = False
        for k, fl in enumerate(self.inflight):
            if fl is None or not self.backend.query(fl[1]):
                continue
            cohort = fl[0]
            self.inflight[k] = None
            self.steps += 1
            self.step_sizes.append(len(cohort))
            t = self.now()
            for req in cohort:
                req.in_flight = False
                req.iteration += 1
                req.ready_at = t
                if req.iteration >= req.n_iterations:
                    req.result = self.backend.result(req, self.lanes[k])
                    req.completed_at = self.now()
                    req.state = DONE
                    self.active.remove(req)
                    self._release(req)
            any_done = True
        return any_done

    def _launch(self) -> bool:
        launched = False
        for k in range(len(self.lanes)):
            if self.inflight[k] is not None:
                continue
            ready = [r for r in self.active if not r.in_flight][: self.max_cohort]
            if not ready:
                break
            t = self.now()
            for r in ready:
                r.in_flight = True
                r.launched(t)
            ev = self.backend.launch(ready, self.lanes[k])
            self.inflight[k] = (ready, ev)
            self.concurrency.append(sum(f is not None for f in self.inflight))
            launched = True
        return launched

    def busy(self) -> bool:
        return any(f is not None for f in self.inflight)

    def advance(self) -> bool:
        """One scheduling round: complete the ended launches, admit, launch on
        the idle streams.  True when a launch ended or began."""
        done = self._complete()
        self._admit()
        return self._launch() or done

    def step(self) -> bool:
        """One scheduling round; False when nothing is running and nothing
        could be launched."""
        return self.advance() or self.busy()

    def _idle(self) -> None:
        # the next arrival still to come (one that has arrived but does not
        # fit waits for a launch to end, as everything else does)
        nxt = self.pending[0].arrival - self.now() if self.pending else None
        if nxt is not None and nxt <= 0.0:
            nxt = None
        if self.busy():
            self.sleep(self.poll_s if nxt is None else min(self.poll_s, nxt))
        elif nxt is not None:
            self.sleep(nxt)
        elif self.pending:
            # nothing runs, yet the head of the queue does not fit: only a
            # budget smaller than one request could do this, and submit
            # rejects those
            raise RuntimeError("stream server stalled with requests pending")

    def wait(self, rid: int) -> Optional[dict]:
        req = self.requests[rid]
        while req.state in (QUEUED, RUNNING):
            if not self.advance():
                if not self.busy() and not self.pending and req.state in (QUEUED, RUNNING):
                    break
                self._idle()
        return req.result

    def run(self) -> None:
        while self.pending or self.active:
            if self.advance():
                continue
            if not self.busy() and not self.pending:
                break
            self._idle()

    def stats(self) -> dict:
        st = super().stats()
        st["n_streams"] = len(self.lanes)
        st["mean_launches_in_flight"] = (float(np.mean(self.concurrency))
                                         if self.concurrency else 0.0)
        return st


def serve_plain(backend, reqs, clock=time.perf_counter, sleep=time.sleep,
                ordered: bool = False) -> dict:
    """The per-request path: one request at a time in arrival order, each
    iteration a single-model launch.  Latency = completion - arrival.
    ordered=True takes `reqs` as an iterable already in arrival order (for
    example one that builds each request as it is reached)."""
    t0 = clock()
    done = []
    for req in (reqs if ordered else sorted(reqs, key=lambda r: r.arrival)):
        wait = req.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        req.bytes = backend.workspace_bytes(req)
        req.handle = backend.load(req)
        req.admitted_at = clock() - t0
        req.first_launch_at = req.admitted_at
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
    return latency_stats(done)
