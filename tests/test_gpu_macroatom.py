"""Macroatom line mode (section 2.5, Table 1) on the GPU against the oracle,
with caller-given transition tables: packet histories, estimators and
spectrum, in both transport kernels and in a multi-model launch; the
degenerate tables (no internal jumps: downbranch; no deactivation: CAPPED)
behave as in the oracle.  Tables derived from the plasma state are tested in
test_gpu_macroatom_plasma.py."""
import numpy as np
import pytest

from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import (REL, assert_close_or_zero, assert_packets_match, divergent, gpu_run,
                         oracle_run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _compare(ctx, model, N, T, ids=None, tune=None):
    g = gpu_run(ctx, model, N, T, packet_ids=ids, tune=tune)
    raw, fin = oracle_run(model, N, T, packet_ids=ids)
    bad = assert_packets_match(g["packets"], raw["packets"])
    if bad.size:
        all_ids = np.asarray(ids if ids is not None else np.arange(N), dtype=np.uint64)
        keep = np.delete(all_ids, bad)
        g = gpu_run(ctx, model, N, T, packet_ids=keep, tune=tune)
        raw, fin = oracle_run(model, N, T, packet_ids=keep)
        assert divergent(g["packets"], raw["packets"]).size == 0
    e, s = g["est"], g["spec"]
    assert_close_or_zero(e["J"], fin["J"], what="J")
    assert_close_or_zero(e["nubar"], fin["nubar"], what="nubar")
    assert_close_or_zero(e["jblue"], fin["jblue"], what="jblue")
    assert_close_or_zero(s["L_nu"], fin["L_nu"], what="L_nu")
    for k in ("L_emitted", "L_reabsorbed", "L_capped"):
        assert s[k] == pytest.approx(fin[k], rel=REL, abs=0 if fin[k] else 1e-300), k
    assert g["counters"] == raw["counters"]
    return g, raw


def _small():
    return W.macroatom_model(seed=3, n_shells=6, n_ions=4, n_levels_per_ion=12, n_lines=200)


@pytest.mark.parametrize("tune", [dict(long_budget=2**32 - 1), dict(long_budget=1, long_lanes=16),
                                  dict(long_budget=3, long_lanes=32),
                                  dict(long_budget=1, long_lanes=64)],
                         ids=["lane", "group16", "group32", "group64"])
def test_macroatom_small_model(ctx, tune):
    g, raw = _compare(ctx, _small(), 4000, 12000.0, tune=tune)
    assert raw["counters"]["line_events"] > 1000


def test_macroatom_30shell_20kline_sample(ctx):
    # caller-given tables at the size of the macroatom workload
    model = W.macroatom_model(seed=0)
    N = 500_000
    ids = np.sort(np.random.default_rng(9).choice(N, 3000, replace=False)).astype(np.uint64)
    _compare(ctx, model, N, 9000.0, ids=ids)


def test_macroatom_without_internal_jumps_is_downbranch(ctx):
    m = W.small_downbranch_model(seed=8, n_shells=5, n_ions=4, n_levels_per_ion=10,
                                 n_lines=150)
    ma = W.Model(**{**m.__dict__})
    ma.line_mode = W.MACROATOM
    ma.em_cum = np.ascontiguousarray(np.tile(m.em_cum, (m.n_shells, 1)))
    for tune in (dict(long_budget=2**32 - 1), dict(long_budget=1)):
        a = gpu_run(ctx, m, 3000, 12000.0, tune=tune)
        b = gpu_run(ctx, ma, 3000, 12000.0, tune=tune)
        # every history takes the same events; after a hand-off the two modes
        # run in kernels that sum the lines' depths over windows of different
        # widths, so positions and energies agree to rounding
        assert divergent(a["packets"], b["packets"]).size == 0
        assert_packets_match(a["packets"], b["packets"])
        assert a["counters"] == b["counters"]


def test_macro_atom_that_never_deactivates(ctx):
    # level 4 (upper level of the strong line) and level 1 jump to each other
    C = 2.99792458e10
    line_nu = C / (np.array([3000.0, 3800.0, 4200.0, 5000.0, 6200.0, 7000.0]) * 1e-8)
    line_upper = np.array([3, 4, 4, 2, 3, 1], dtype=np.int32)
    level_ptr = np.array([0, 1, 2, 3, 4, 5])
    em_line = np.array([0, -5, 3, 0, -2], dtype=np.int32)
    tau = np.zeros((1, 6))
    tau[0, 2] = 1e6
    v = np.array([11000.0, 20000.0]) * 1e5
    m = W.Model(v_bounds=v, t_exp=13 * 86400.0, n_e=np.zeros(1), line_nu=line_nu,
                tau_sobolev=tau, line_mode=W.MACROATOM, line_upper=line_upper, n_levels=5,
                level_ptr=level_ptr, em_line=em_line, em_cum=np.ones((1, 5)), seed=5)
    for tune in (dict(long_budget=2**32 - 1), dict(long_budget=1)):
        g, raw = _compare(ctx, m, 3000, 12000.0, tune=tune)
        assert raw["counters"]["capped"] > 30


def test_macroatom_in_a_multi_model_launch(ctx):
    mix = [(W.small_model(seed=80, n_shells=5, n_lines=400), 1500, 10000.0),
           (_small(), 2500, 12000.0),
           (W.small_downbranch_model(seed=81, n_shells=4), 1000, 11000.0)]
    F = smc.F_JBLUE | smc.F_PACKETS
    models = [smc.Model(ctx, mdl, N, flags=F) for mdl, N, _ in mix]
    ctx.batch_run(models, [dict(n_packets=N, T_inner=T, flags=F) for _, N, T in mix],
                  tune=dict(long_budget=4))
    for m, (mdl, N, T) in zip(models, mix):
        raw, fin = oracle_run(mdl, N, T)
        if assert_packets_match(m.read_packets(N), raw["packets"]).size == 0:
            assert_close_or_zero(m.read_spectrum()["L_nu"], fin["L_nu"], what="L_nu")
            assert m.read_counters() == raw["counters"]


@pytest.mark.parametrize("seed", range(12))
def test_random_small_macroatom_configurations(ctx, seed):
    """Seeded random macro-atom models: shells, ions, levels per ion, lines,
    packets, temperature and launch tuning (including a hand-off at the
    first segment and none at all)."""
    rng = np.random.default_rng(500 + seed)
    n_ions = int(rng.integers(1, 7))
    nl = int(rng.integers(4, 16))
    L = int(rng.integers(5, min(400, n_ions * nl * (nl - 1) // 2) + 1))
    model = W.macroatom_model(seed=500 + seed, n_shells=int(rng.integers(1, 25)), n_ions=n_ions,
                              n_levels_per_ion=nl, n_lines=L)
    tune = [None, dict(long_budget=1, long_lanes=int(rng.choice([16, 32, 64]))),
            dict(long_budget=2**32 - 1)][seed % 3]
    _compare(ctx, model, int(rng.integers(1, 2500)), float(rng.uniform(6000.0, 30000.0)),
             tune=tune)
