"""The allocation-free batch entry point (smc_batch_run_static, its
launch-wide scratch in a static device array) against smc_batch_run: two
calls in a row, the second with fewer and smaller models, give the same
histories, counters, estimators and spectra; more models than the scratch
holds are refused."""
import numpy as np
import pytest

from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import REL, assert_close_or_zero

pytestmark = pytest.mark.gpu

F_ALL = smc.F_JBLUE | smc.F_PACKETS


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _mix(n, seed, shells, lines, packets):
    out = []
    for i in range(n):
        if i % 4 == 3:
            mdl = W.small_downbranch_model(seed=seed + i, n_shells=3 + i % shells, n_ions=3,
                                           n_levels_per_ion=10, n_lines=40 + i)
        else:
            mdl = W.small_model(seed=seed + i, n_shells=2 + i % shells, n_lines=lines + 37 * i,
                                tau="lognormal")
        out.append((mdl, packets + 97 * i, 9000.0 + 700.0 * i))
    return out


def _run(ctx, mix, static, tune):
    models = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N, _ in mix]
    params = [dict(n_packets=N, T_inner=T, iteration=1, flags=F_ALL) for _, N, T in mix]
    (ctx.batch_run_static if static else ctx.batch_run)(models, params, tune=tune)
    return [dict(packets=m.read_packets(N), est=m.read_estimators(), spec=m.read_spectrum(),
                 counters=m.read_counters()) for m, (_, N, _) in zip(models, mix)]


@pytest.mark.parametrize("tune", [None, dict(long_budget=3, long_lanes=32)],
                         ids=["default", "handoff3-lanes32"])
def test_static_scratch_matches_batch_run(ctx, tune):
    first = _mix(24, 3100, 9, 900, 1500)   # 24 models
    second = _mix(5, 3200, 3, 120, 300)    # then fewer, smaller ones
    for mix in (first, second):
        ref = _run(ctx, mix, False, tune)
        got = _run(ctx, mix, True, tune)
        for a, b in zip(ref, got):
            assert np.array_equal(a["packets"]["hash"], b["packets"]["hash"])
            for f in ("nu", "energy", "mu", "r"):
                np.testing.assert_allclose(b["packets"][f], a["packets"][f], rtol=REL, atol=0)
            assert a["counters"] == b["counters"]
            for k in ("J", "nubar", "T_R", "W"):
                np.testing.assert_allclose(b["est"][k], a["est"][k], rtol=REL, atol=0)
            assert_close_or_zero(b["est"]["jblue"], a["est"]["jblue"], what="jblue")
            assert_close_or_zero(b["spec"]["L_nu"], a["spec"]["L_nu"], what="L_nu")
            assert b["spec"]["T_inner_next"] == pytest.approx(a["spec"]["T_inner_next"],
                                                              rel=REL, abs=0)


def test_static_scratch_refuses_more_models_than_it_holds(ctx):
    mix = _mix(smc.STATIC_MAX_MODELS + 1, 3300, 2, 20, 10)
    models = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N, _ in mix]
    params = [dict(n_packets=N, T_inner=T) for _, N, T in mix]
    with pytest.raises(smc.SmcError) as ei:
        ctx.batch_run_static(models, params)
    assert ei.value.code == smc.SMC_EINVAL
    ctx.batch_run(models, params)  # the context's own buffers take them
