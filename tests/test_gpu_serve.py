"""Served requests give the same results alone and in the mix: requests of
different sizes and iteration counts arrive while others run, join the
multi-model launches, and each result matches the same request run alone
(one single-model launch per iteration) to the parity tolerance."""
import numpy as np
import pytest

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
        def step(self, reqs):
            super().step(reqs)
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
            def step(self, reqs):
                super().step(reqs)
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
