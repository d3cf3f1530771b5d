"""Serving-loop logic on the CPU with a fake device backend and a simulated
clock: admission by memory budget in arrival order, continuous batching (a
request that arrives while others run joins at the next step), completion
after its iterations, cancellation and rejection."""
import numpy as np
import pytest

from paper_1401_5469_amd import serve
from paper_1401_5469_amd import workloads as W


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBackend:
    """Records every step; a step costs 1 s plus 0.1 s per request."""

    def __init__(self, clock):
        self.clock = clock
        self.steps = []
        self.live = {}
        self.peak = 0
        self.loaded = 0

    def workspace_bytes(self, req):
        return req.n_packets * 10

    def load(self, req):
        self.loaded += 1
        h = object()
        self.live[id(h)] = req.n_packets * 10
        self.peak = max(self.peak, sum(self.live.values()))
        return h

    def free(self, h):
        del self.live[id(h)]

    def step(self, reqs):
        self.steps.append([(r.rid, r.iteration) for r in reqs])
        self.clock.t += 1.0 + 0.1 * len(reqs)

    def sync(self):
        pass

    def result(self, req):
        return dict(iterations=req.iteration)


def _req(n_packets, n_iter, arrival):
    m = W.small_model(seed=1, n_shells=2, n_lines=5)
    return serve.Request(model=m, n_iterations=n_iter, n_packets=n_packets, T_inner=9000.0,
                         arrival=arrival)


def _server(budget):
    clk = Clock()
    be = FakeBackend(clk)
    return serve.Server(be, memory_budget=budget, clock=clk, sleep=clk.sleep), be, clk


def test_continuous_batching_and_completion():
    srv, be, clk = _server(budget=10**9)
    a = srv.submit(_req(100, 3, 0.0))
    b = srv.submit(_req(100, 1, 1.0))   # arrives while a is running
    c = srv.submit(_req(100, 2, 10.0))  # arrives after both are done
    srv.run()
    assert [srv.poll(x) for x in (a, b, c)] == [serve.DONE] * 3
    # step 1: a alone; step 2: a + b (b joined); step 3: a; then c alone twice
    assert be.steps[0] == [(a, 0)]
    assert be.steps[1] == [(a, 1), (b, 0)]
    assert be.steps[2] == [(a, 2)]
    assert be.steps[3:] == [[(c, 0)], [(c, 1)]]
    assert srv.result(a)["iterations"] == 3 and srv.result(b)["iterations"] == 1
    st = srv.stats()
    assert st["completed"] == 3 and st["max_batch"] == 2
    assert be.live == {}  # every workspace released


def test_admission_never_exceeds_the_budget_and_keeps_order():
    srv, be, clk = _server(budget=2500)
    ids = [srv.submit(_req(100, k % 3 + 1, 0.01 * k)) for k in range(12)]  # 1000 B each
    srv.run()
    assert be.peak <= 2500
    assert max(len(s) for s in be.steps) == 2
    admitted = sorted(ids, key=lambda i: srv.requests[i].admitted_at)
    assert admitted == ids  # FIFO admission
    assert all(srv.poll(i) == serve.DONE for i in ids)


def test_oversized_request_is_rejected_and_cancel_works():
    srv, be, clk = _server(budget=5000)
    big = srv.submit(_req(1000, 1, 0.0))
    assert srv.poll(big) == serve.REJECTED
    a = srv.submit(_req(100, 5, 0.0))
    b = srv.submit(_req(100, 5, 0.0))
    q = srv.submit(_req(100, 5, 100.0))
    srv.step()
    assert srv.poll(a) == serve.RUNNING and srv.poll(b) == serve.RUNNING
    assert srv.cancel(b) and srv.poll(b) == serve.CANCELLED
    assert srv.cancel(q) and srv.poll(q) == serve.CANCELLED
    srv.run()
    assert srv.poll(a) == serve.DONE
    assert not srv.cancel(a)
    assert be.live == {}
    assert all(b not in [r for r, _ in s] for s in be.steps[1:])


def test_plain_path_runs_one_request_at_a_time():
    clk = Clock()
    be = FakeBackend(clk)
    reqs = [_req(100, 2, 0.0), _req(100, 1, 0.5), _req(100, 3, 0.6)]
    for i, r in enumerate(reqs):
        r.rid = i
    st = serve.serve_plain(be, reqs, clock=clk, sleep=clk.sleep)
    assert st["completed"] == 3
    assert all(len(s) == 1 for s in be.steps)
    assert [s[0] for s in be.steps] == [(0, 0), (0, 1), (1, 0), (2, 0), (2, 1), (2, 2)]
    lat = [r.latency for r in reqs]
    assert lat[0] == 2.2 and np.isclose(lat[1], 2.2 + 1.1 - 0.5)


def test_wait_serves_until_the_request_is_done():
    clock = Clock()
    be = FakeBackend(clock)
    srv = serve.Server(be, memory_budget=10**9, clock=clock, sleep=clock.sleep)
    a = srv.submit(_req(100, 2, 0.0))
    b = srv.submit(_req(100, 5, 0.5))
    c = srv.submit(_req(100, 1, 100.0))  # arrives long after the others
    assert srv.wait(a) == dict(iterations=2)
    assert srv.poll(a) == serve.DONE and srv.poll(b) == serve.RUNNING
    # b joined at the second step and ran alongside a: it is part-way
    assert srv.requests[b].iteration == 1
    assert srv.wait(c) == dict(iterations=1)  # sleeps until c arrives, finishing b first
    assert srv.poll(b) == serve.DONE and clock.t >= 100.0
    huge = srv.submit(_req(10**9, 1, 0.0))
    assert srv.wait(huge) is None and srv.poll(huge) == serve.REJECTED


class FakeStreams(FakeBackend):
    """Launch streams on the simulated clock: a launch on a stream ends
    `cost(reqs)` seconds after it starts; streams run concurrently."""

    def __init__(self, clock, cost=lambda reqs: 1.0 + 0.1 * len(reqs)):
        super().__init__(clock)
        self.cost = cost
        self.launches = []  # (stream, start, end, [(rid, iteration)])

    def stream(self, k):
        return k

    def launch(self, reqs, stream):
        t = self.clock.t
        end = t + self.cost(reqs)
        self.launches.append((stream, t, end, [(r.rid, r.iteration) for r in reqs]))
        self.steps.append([(r.rid, r.iteration) for r in reqs])
        return end

    def query(self, ev):
        return self.clock.t >= ev

    def result(self, req, stream=None):
        return dict(iterations=req.iteration)


def _stream_server(budget, n_streams=2, cost=None):
    clk = Clock()
    be = FakeStreams(clk) if cost is None else FakeStreams(clk, cost)
    return (serve.StreamServer(be, memory_budget=budget, n_streams=n_streams, poll_s=0.01,
                               clock=clk, sleep=clk.sleep), be, clk)


def test_stream_server_launches_arrivals_without_waiting_for_a_cohort():
    # a long launch (request a, 10 s per iteration) is running when b
    # arrives: b goes out on the idle stream at once, and finishes first
    srv, be, clk = _stream_server(10**9, cost=lambda reqs: 10.0 if reqs[0].rid == 0 else 1.0)
    a = srv.submit(_req(100, 2, 0.0))
    b = srv.submit(_req(100, 3, 0.5))
    srv.run()
    assert srv.poll(a) == serve.DONE and srv.poll(b) == serve.DONE
    ra, rb = srv.requests[a], srv.requests[b]
    assert rb.first_launch_at == pytest.approx(0.5, abs=0.02)
    assert rb.completed_at < ra.completed_at
    assert rb.queue_wait < 0.05
    # the step-synchronous server makes b wait for a's first iteration
    srv2, be2, clk2 = _server(10**9)
    a2 = srv2.submit(_req(100, 2, 0.0))
    b2 = srv2.submit(_req(100, 3, 0.5))
    srv2.run()
    assert srv2.requests[b2].queue_wait > 0.5  # until the step of a ends at 1.1 s


def test_stream_server_keeps_each_requests_iterations_in_order():
    srv, be, clk = _stream_server(10**9, n_streams=3,
                                  cost=lambda reqs: 0.3 + 0.7 * (len(reqs) % 3))
    ids = [srv.submit(_req(100, 1 + k % 4, 0.2 * k)) for k in range(15)]
    srv.run()
    assert all(srv.poll(i) == serve.DONE for i in ids)
    assert all(srv.result(i)["iterations"] == srv.requests[i].n_iterations for i in ids)
    for rid in ids:
        runs = [(s, e, it) for _, s, e, c in be.launches for r, it in c if r == rid]
        # iterations 0, 1, ... in order, each after the previous one ended
        assert [it for _, _, it in runs] == list(range(srv.requests[rid].n_iterations))
        for (s0, e0, _), (s1, _, _) in zip(runs, runs[1:]):
            assert s1 >= e0
    # no request is in two launches at once
    for k, (_, s, e, c) in enumerate(be.launches):
        for _, s2, e2, c2 in be.launches[k + 1:]:
            if s2 < e and s < e2:
                assert not ({r for r, _ in c} & {r for r, _ in c2})
    assert be.live == {}
    st = srv.stats()
    assert st["completed"] == 15 and st["n_streams"] == 3
    assert st["mean_launches_in_flight"] > 1.0
    assert st["queue_wait_s"]["p99"] is not None and st["service_s"]["p50"] > 0.0


def test_stream_server_budget_cancel_and_wait():
    srv, be, clk = _stream_server(budget=2500)
    ids = [srv.submit(_req(100, 2, 0.01 * k)) for k in range(6)]  # 1000 B each
    big = srv.submit(_req(1000, 1, 0.0))
    assert srv.poll(big) == serve.REJECTED
    assert srv.wait(ids[0]) == dict(iterations=2)
    assert srv.cancel(ids[5]) and srv.poll(ids[5]) == serve.CANCELLED
    srv.run()
    assert be.peak <= 2500
    assert all(srv.poll(i) == serve.DONE for i in ids[:5])
    assert be.live == {}
