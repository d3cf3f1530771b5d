"""Serving-loop logic on the CPU with a fake device backend and a simulated
clock: admission by memory budget in arrival order, continuous batching (a
request that arrives while others run joins at the next step), completion
after its iterations, cancellation and rejection."""
import numpy as np

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
