"""Served requests against their own oracle chains: requests of different
sizes and iteration counts arrive while others run and join the
multi-model launches (the step-synchronous server, and the stream server
with launches in flight on several streams); every result -- J, nu-bar,
T_R, W, J_blue, L_nu, the T_inner it ran at and the next one, the counters
-- matches the oracle run iteration by iteration with T_inner carried as
the library carries it (section 2.8), and the same request run alone."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1401_5469_amd import serve
from paper_1401_5469_amd import workloads as W

from gpu_helpers import REL, assert_close_or_zero

pytestmark = pytest.mark.gpu


class StepClock:
    """Simulated time: every device step takes one second."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


def _requests():
    spec = [  # (seed, shells, lines, packets, iterations, arrival)
        (201, 5, 400, 800, 3, 0.0), (202, 12, 3000, 1500, 1, 0.0), (203, 3, 60, 200, 2, 1.5),
        (204, 8, 1500, 1100, 3, 2.5), (205, 1, 20, 50, 1, 2.5), (206, 6, 900, 700, 2, 6.0)]
    out = []
    for seed, S, L, N, it, arr in spec:
        m = W.small_model(seed=seed, n_shells=S, n_lines=L, tau="lognormal")
        out.append(serve.Request(model=m, n_iterations=it, n_packets=N, T_inner=9000.0,
                                 L_requested=W.L_REQUESTED, damping=0.5, arrival=arr))
    return out


def test_results_are_the_same_alone_and_in_the_mix():
    clk = StepClock()

    class Backend(serve.GpuBackend):
        def step(self, reqs, stream=None):
            super().step(reqs, stream)
            clk.t += 1.0

    be = Backend(tune=dict(long_budget=6))
    srv = serve.Server(be, memory_budget=200 * 2**30, clock=clk, sleep=clk.sleep)
    mixed = _requests()
    for r in mixed:
        srv.submit(r)
    srv.run()
    st = srv.stats()
    assert st["completed"] == len(mixed)
    assert st["max_batch"] >= 3  # requests really shared launches

    alone = _requests()
    serve.serve_plain(serve.GpuBackend(), alone, clock=clk, sleep=clk.sleep)
    for a, b in zip(alone, mixed):
        ra, rb = a.result, b.result
        assert ra["counters"] == rb["counters"]
        for k in ("J", "nubar", "T_R", "W"):
            np.testing.assert_allclose(rb[k], ra[k], rtol=REL, atol=0)
        assert_close_or_zero(rb["jblue"], ra["jblue"], what="jblue")
        assert_close_or_zero(rb["L_nu"], ra["L_nu"], what="L_nu")
        assert rb["T_inner"] == pytest.approx(ra["T_inner"], rel=REL, abs=0)
        assert rb["T_inner_next"] == pytest.approx(ra["T_inner_next"], rel=REL, abs=0)


def test_wait_returns_each_result():
    """wait(id) in reverse arrival order: each call serves the whole active
    set until its request is done, and every result matches run()'s."""
    def served(use_wait):
        clk = StepClock()

        class Backend(serve.GpuBackend):
            def step(self, reqs, stream=None):
                super().step(reqs, stream)
                clk.t += 1.0

        srv = serve.Server(Backend(), memory_budget=200 * 2**30, clock=clk, sleep=clk.sleep)
        reqs = _requests()
        ids = [srv.submit(r) for r in reqs]
        if use_wait:
            out = {rid: srv.wait(rid) for rid in reversed(ids)}
            assert all(srv.poll(rid) == serve.DONE for rid in ids)
            return [out[rid] for rid in ids]
        srv.run()
        return [r.result for r in reqs]

    for ra, rb in zip(served(False), served(True)):
        assert ra["counters"] == rb["counters"]
        for k in ("J", "nubar", "T_R", "W"):
            np.testing.assert_allclose(rb[k], ra[k], rtol=REL, atol=0)
        assert rb["T_inner_next"] == pytest.approx(ra["T_inner_next"], rel=REL, abs=0)


def _oracle_chain(req):
    """The request's iterations on the oracle: T_inner and the radiation
    field carried from one iteration to the next."""
    T = req.T_inner
    T_R, W_ = O.initial_radiation_field(req.model)
    for it in range(req.n_iterations):
        raw = O.run(req.model, T, req.n_packets, iteration=it)
        fin = O.finalise(req.model, raw, T, L_requested=req.L_requested, T_R_prev=T_R,
                         W_prev=W_, damping=req.damping)
        T_R, W_ = fin["T_R"], fin["W"]
        fin["T_inner"] = T
        T = fin["T_inner_next"]
    return raw, fin


def _assert_oracle(req):
    raw, fin = _oracle_chain(req)
    r = req.result
    assert r["counters"] == raw["counters"]
    for k in ("J", "nubar", "T_R", "W"):
        np.testing.assert_allclose(r[k], fin[k], rtol=REL, atol=0)
    assert_close_or_zero(r["jblue"], fin["jblue"], what="jblue")
    assert_close_or_zero(r["L_nu"], fin["L_nu"], what="L_nu")
    assert r["T_inner"] == pytest.approx(fin["T_inner"], rel=REL, abs=0)
    assert r["T_inner_next"] == pytest.approx(fin["T_inner_next"], rel=REL, abs=0)


def test_each_served_request_matches_its_oracle_chain():
    clk = StepClock()

    class Backend(serve.GpuBackend):
        def step(self, reqs, stream=None):
            super().step(reqs, stream)
            clk.t += 1.0

    srv = serve.Server(Backend(tune=dict(long_budget=6)), memory_budget=200 * 2**30, clock=clk,
                       sleep=clk.sleep)
    reqs = _requests()
    for r in reqs:
        srv.submit(r)
    srv.run()
    assert srv.stats()["max_batch"] >= 3
    for r in reqs:
        _assert_oracle(r)


def test_stream_server_requests_match_their_oracle_chains():
    # real time: arrivals spread over 0.3 s, launches on three streams
    reqs = _requests()
    for r in reqs:
        r.arrival *= 0.05
    srv = serve.StreamServer(serve.GpuBackend(tune=dict(long_budget=6)),
                             memory_budget=200 * 2**30, n_streams=3)
    for r in reqs:
        srv.submit(r)
    srv.run()
    st = srv.stats()
    assert st["completed"] == len(reqs)
    for r in reqs:
        assert r.state == serve.DONE and r.iteration == r.n_iterations
        _assert_oracle(r)
