"""Captured iteration sequences (HIP graphs) and the batch autotuner."""
import numpy as np
import pytest

from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import assert_packets_match

pytestmark = pytest.mark.gpu

F_ALL = smc.F_JBLUE | smc.F_PACKETS


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _iters(T0, n_iter, N, L_req):
    # the first iteration fixes T_inner, later ones take the device-side update
    return [dict(n_packets=N, T_inner=T0 if i == 0 else 0.0, iteration=i, flags=F_ALL,
                 L_requested=L_req, damping=0.5) for i in range(n_iter)]


def _state(m, N):
    return dict(packets=m.read_packets(N), est=m.read_estimators(), spec=m.read_spectrum())


def _same(a, b):
    assert np.array_equal(a["packets"], b["packets"])
    for k in ("J", "nubar", "T_R", "W"):
        np.testing.assert_allclose(b["est"][k], a["est"][k], rtol=1e-12, atol=0)
    np.testing.assert_allclose(b["est"]["jblue"], a["est"]["jblue"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(b["spec"]["L_nu"], a["spec"]["L_nu"], rtol=1e-12, atol=1e-300)
    assert b["spec"]["T_inner"] == pytest.approx(a["spec"]["T_inner"], rel=1e-12, abs=0)


def test_graph_replays_match_eager_single_model(ctx):
    import torch
    w = W.config2(n_lines=20_000)
    N = 3000
    seq = _iters(w.T_inner, 3, N, w.L_requested)
    eager = smc.Model(ctx, w.model, N, flags=F_ALL)
    for p in seq:
        eager.run_iteration(**p)
    ref = _state(eager, N)
    assert ref["spec"]["T_inner"] != w.T_inner  # the update was carried on the device

    m = smc.Model(ctx, w.model, N, flags=F_ALL)
    g = ctx.capture([m], [[p] for p in seq])
    for replay in range(3):
        g.launch()
        torch.cuda.synchronize()
        _same(ref, _state(m, N))
        # eager work on the same stream between replays
        scratch = torch.ones(1 << 20, device="cuda").sum().item()
        assert scratch == float(1 << 20)
    g.destroy()


def test_graph_replays_match_eager_multi_model(ctx):
    import torch
    mix = [(W.small_model(seed=s, n_shells=S, n_lines=L), N)
           for s, S, L, N in [(1, 4, 300, 500), (2, 9, 2000, 1300), (3, 2, 50, 70)]]
    seqs = [_iters(9500.0, 2, N, 0.0) for _, N in mix]
    eager = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N in mix]
    for i in range(2):
        ctx.batch_run(eager, [s[i] for s in seqs], tune=dict(long_budget=4))
    refs = [_state(m, N) for m, (_, N) in zip(eager, mix)]
    models = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N in mix]
    g = ctx.capture(models, [[s[i] for s in seqs] for i in range(2)], tune=dict(long_budget=4))
    for replay in range(2):
        g.launch()
        torch.cuda.synchronize()
        for ref, m, (_, N) in zip(refs, models, mix):
            _same(ref, _state(m, N))
    g.destroy()


def test_autotune_picks_a_valid_config(ctx):
    mix = [(W.small_model(seed=s, n_shells=6, n_lines=3000, tau="lognormal"), 4000)
           for s in range(3)]
    models = [smc.Model(ctx, mdl, N, flags=smc.F_JBLUE) for mdl, N in mix]
    params = [dict(n_packets=N, T_inner=9000.0) for _, N in mix]
    best, ms = ctx.batch_autotune(models, params)
    assert ms > 0.0
    assert best["long_budget"] in (0, 256, 1024, 4096, 2**32 - 1)
    assert best["long_lanes"] in (0, 16, 32, 64)
    cands = [dict(long_budget=8, long_lanes=64), dict(long_budget=2**32 - 1, blocks_per_cu=1)]
    best2, ms2 = ctx.batch_autotune(models, params, candidates=cands)
    assert best2 in [dict(blocks_per_cu=c.get("blocks_per_cu", 0), long_waves_per_cu=0,
                          long_budget=c["long_budget"], long_lanes=c.get("long_lanes", 0))
                     for c in cands]
    with pytest.raises(smc.SmcError):
        ctx.batch_autotune(models, params, candidates=[dict(long_lanes=48)])
    with pytest.raises(smc.SmcError):
        ctx.batch_autotune(models, [dict(n_packets=N, T_inner=0.0) for _, N in mix])


@pytest.mark.parametrize("nlte", [False, True], ids=["plasma", "plasma-nlte"])
def test_graph_with_plasma_updates_matches_eager(ctx, nlte):
    """The loop of section 2.8 captured whole: every iteration followed by the
    plasma update from the model's own field (NLTE with J_b from the J_blue
    estimator).  Replays continue the eager sequence: after replay r the
    state equals that of the eager loop after its (r+1)-th pass."""
    import torch
    model, spec = W.plasma_model(seed=31, n_shells=6, n_elements=6, n_stages=5,
                                 n_levels_per_ion=25, n_lines=2500,
                                 nlte_ions=(6, 11) if nlte else (), n_levels_nlte=20)
    N = 2500
    seq = _iters(11000.0, 3, N, 0.0)
    upd = dict(ionization=smc.ION_NEBULAR, excitation=smc.EXC_DILUTE_LTE, delta=0.8, nlte=nlte,
               jblue_mode=smc.JB_DETAILED if nlte else smc.JB_DILUTE_BLACKBODY)
    eager = smc.Model(ctx, model, N, flags=F_ALL)
    pe = smc.Plasma(eager, spec)
    pe.update(upd["ionization"], upd["excitation"], upd["delta"])  # opacities of the initial field
    m = smc.Model(ctx, model, N, flags=F_ALL)
    pg = smc.Plasma(m, spec)
    pg.update(upd["ionization"], upd["excitation"], upd["delta"])
    g = ctx.capture([m], [[p] for p in seq], plasmas=[pg], plasma_params=[upd])
    for rep in range(2):
        for p in seq:
            eager.run_iteration(**p)
            pe.update(**upd)
        ref, ref_pl = _state(eager, N), pe.read()
        g.launch()
        torch.cuda.synchronize()
        got, got_pl = _state(m, N), pg.read()
        # n_e from the plasma state moves Thomson events by the last bits of
        # the estimators' (order-dependent) sums, so the comparison is to the
        # parity tolerance rather than bit for bit
        assert_packets_match(got["packets"], ref["packets"], rel=1e-9, allow_fraction=0.0)
        for k in ("J", "nubar", "T_R", "W"):
            np.testing.assert_allclose(got["est"][k], ref["est"][k], rtol=1e-9, atol=0)
        np.testing.assert_allclose(got["spec"]["L_nu"], ref["spec"]["L_nu"], rtol=1e-9,
                                   atol=1e-300)
        np.testing.assert_allclose(got_pl["tau"], ref_pl["tau"], rtol=1e-8, atol=1e-300)
        np.testing.assert_allclose(got_pl["n_e"], ref_pl["n_e"], rtol=1e-8, atol=0)
        np.testing.assert_allclose(got_pl["level_pop"], ref_pl["level_pop"], rtol=1e-8,
                                   atol=1e-250)
        assert got_pl["n_singular"] == 0
    g.destroy()
    with pytest.raises(smc.SmcError):  # an unknown J_b mode is refused at capture
        ctx.capture([m], [[p] for p in seq], plasmas=[pg],
                    plasma_params=[dict(upd, jblue_mode=7)])


@pytest.mark.parametrize("jb", ["dilute", "detailed"])
def test_graph_of_the_macroatom_loop_matches_eager(ctx, jb):
    """A macroatom model whose transition tables are derived by every plasma
    update: the captured loop (iteration, plasma update with new depths and
    tables) replays the eager one, tables included."""
    import torch
    model, spec = W.macroatom_plasma_model(seed=33, n_shells=5, n_elements=5, n_stages=4,
                                           n_levels_per_ion=15, n_lines=1500)
    N = 2500
    seq = _iters(11000.0, 3, N, 0.0)
    upd = dict(ionization=smc.ION_NEBULAR, excitation=smc.EXC_DILUTE_LTE, delta=1.0,
               jblue_mode=smc.JB_DETAILED if jb == "detailed" else smc.JB_DILUTE_BLACKBODY)
    eager = smc.Model(ctx, model, N, flags=F_ALL)
    pe = smc.Plasma(eager, spec)
    pe.update(upd["ionization"], upd["excitation"], upd["delta"])
    m = smc.Model(ctx, model, N, flags=F_ALL)
    pg = smc.Plasma(m, spec)
    pg.update(upd["ionization"], upd["excitation"], upd["delta"])
    g = ctx.capture([m], [[p] for p in seq], plasmas=[pg], plasma_params=[upd])
    for rep in range(2):
        for p in seq:
            eager.run_iteration(**p)
            pe.update(**upd)
        ref, ref_tab = _state(eager, N), eager.read_macroatom()
        g.launch()
        torch.cuda.synchronize()
        got, got_tab = _state(m, N), m.read_macroatom()
        assert_packets_match(got["packets"], ref["packets"], rel=1e-9, allow_fraction=0.0)
        for k in ("J", "nubar", "T_R", "W"):
            np.testing.assert_allclose(got["est"][k], ref["est"][k], rtol=1e-9, atol=0)
        assert np.array_equal(got_tab[0], ref_tab[0]) and np.array_equal(got_tab[1], ref_tab[1])
        np.testing.assert_allclose(got_tab[2], ref_tab[2], rtol=0, atol=1e-9)
        assert m.read_counters()["line_events"] > 100
    g.destroy()
