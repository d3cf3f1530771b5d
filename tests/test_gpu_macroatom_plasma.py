"""Macro-atom tables derived on the device from the plasma state (section 2.5
with 2.3 and the loop of 2.8) against the oracle's own tables
(oracle/macroatom.py) on the oracle's own plasma state: the row layout bit
for bit, the cumulative probabilities element by element, in the
dilute-blackbody and the detailed (J_blue) modes; then the macroatom
feedback loop (iteration -> plasma update with new tables -> iteration)
packet by packet, and the errors.

Tolerance: the tables are cumulative sums of products of a few factors
(beta from tau_S, Einstein coefficients, a Planck function) divided by the
row total, so a relative difference of order 1e-13 in tau_S or the field
moves them by about as much; 1e-10 absolute on values in [0, 1].  After an
iteration, J_blue and T_R / W carry the estimators' 1e-9, so the tables are
held to 1e-8 there."""
import numpy as np
import pytest

from oracle import macroatom as MA
from oracle import oracle as O
from oracle import plasma as P
from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import assert_packets_match, divergent

pytestmark = pytest.mark.gpu

ION, EXC = W.ION_NEBULAR, W.EXC_DILUTE_LTE


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _small(seed, n_lines=2000, n_shells=6):
    return W.macroatom_plasma_model(seed=seed, n_shells=n_shells, n_elements=6, n_stages=5,
                                    n_levels_per_ion=20, n_lines=n_lines)


def _oracle_model(model, spec, T_R, Wd, jblue=None):
    """The oracle's chain step: its plasma state at (T_R, W), its tables on
    those depths, and the model that carries both."""
    st = P.plasma_state(spec.atom, spec.number_density, model.line_nu, model.t_exp, T_R, Wd,
                        ION, EXC)
    ptr, line, cum = MA.tables(spec.atom, model.line_nu, st["tau"], T_R, Wd, jblue=jblue)
    m = W.Model(**{**model.__dict__, "tau_sobolev": np.ascontiguousarray(st["tau"]),
                   "n_e": np.ascontiguousarray(st["n_e"]), "level_ptr": ptr, "em_line": line,
                   "em_cum": np.ascontiguousarray(cum)})
    return m, st


def _assert_tables(g, o, tol):
    ptr, line, cum = g
    assert np.array_equal(ptr, o.level_ptr)
    assert np.array_equal(line, o.em_line)
    err = np.abs(cum - o.em_cum)
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= tol, f"em_cum {worst}: {cum[worst]} vs {o.em_cum[worst]}"
    assert np.all(cum[:, ptr[1:][ptr[1:] > ptr[:-1]] - 1] == 1.0)


@pytest.mark.parametrize("seed", [1, 2])
def test_tables_from_the_initial_field(ctx, seed):
    model, spec = _small(seed)
    m = smc.Model(ctx, model, 1000, flags=smc.F_JBLUE)
    pl = smc.Plasma(m, spec)
    pl.update(ION, EXC)
    T0, W0 = O.initial_radiation_field(model)
    o, _ = _oracle_model(model, spec, T0, W0)
    _assert_tables(m.read_macroatom(), o, 1e-10)


def test_paper_size_macroatom_tables(ctx):
    w, spec = W.config_macroatom()
    m = smc.Model(ctx, w.model, 1000, flags=smc.F_JBLUE)
    pl = smc.Plasma(m, spec)
    pl.update(ION, EXC)
    T0, W0 = O.initial_radiation_field(w.model)
    o, _ = _oracle_model(w.model, spec, T0, W0)
    _assert_tables(m.read_macroatom(), o, 1e-10)


def test_paper_size_macroatom_sample(ctx):
    # the macroatom workload (5e5 packets): sampled packets against the
    # oracle on its own plasma state and tables
    w, spec = W.config_macroatom()
    N = w.n_packets
    ids = np.sort(np.random.default_rng(9).choice(N, 3000, replace=False)).astype(np.uint64)
    m = smc.Model(ctx, w.model, N, flags=smc.F_JBLUE | smc.F_PACKETS)
    pl = smc.Plasma(m, spec)
    pl.update(ION, EXC)
    m.run_iteration(N, w.T_inner, flags=smc.F_JBLUE | smc.F_PACKETS, packet_ids=ids)
    T0, W0 = O.initial_radiation_field(w.model)
    o, _ = _oracle_model(w.model, spec, T0, W0)
    raw = O.run(o, w.T_inner, N, packet_ids=ids)
    assert raw["counters"]["line_events"] > 1000
    assert_packets_match(m.read_packets(len(ids)), raw["packets"])


def test_detailed_mode_takes_the_jblue_estimator(ctx):
    model, spec = _small(3)
    N, T = 20000, 12000.0
    flags = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, N, flags=flags)
    pl = smc.Plasma(m, spec)
    # before any iteration the detailed mode starts from W B_nu(T_R)
    pl.update(ION, EXC, jblue_mode=smc.JB_DETAILED)
    T0, W0 = O.initial_radiation_field(model)
    o0, _ = _oracle_model(model, spec, T0, W0)
    _assert_tables(m.read_macroatom(), o0, 1e-10)
    m.run_iteration(N, T, flags=flags)
    g_packets = m.read_packets(N)
    pl.update(ION, EXC, jblue_mode=smc.JB_DETAILED)
    g = m.read_macroatom()
    raw0 = O.run(o0, T, N, iteration=0)
    assert assert_packets_match(g_packets, raw0["packets"]).size == 0
    fin0 = O.finalise(o0, raw0, T, T_R_prev=T0, W_prev=W0)
    o1, _ = _oracle_model(model, spec, fin0["T_R"], fin0["W"], jblue=fin0["jblue"])
    _assert_tables(g, o1, 1e-8)
    d1, _ = _oracle_model(model, spec, fin0["T_R"], fin0["W"])
    assert np.abs(d1.em_cum - o1.em_cum).max() > 1e-3  # the estimator did change them


def test_macroatom_feedback_loop_packet_by_packet(ctx):
    model, spec = _small(4, n_lines=3000)
    N, T = 4000, 11000.0
    flags = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, N, flags=flags)
    pl = smc.Plasma(m, spec)
    pl.update(ION, EXC)
    m.run_iteration(N, T, iteration=0, flags=flags)
    g0 = m.read_packets(N)
    pl.update(ION, EXC)
    g_tables1 = m.read_macroatom()
    m.run_iteration(N, T, iteration=1, flags=flags)
    g1 = m.read_packets(N)
    c1 = m.read_counters()

    T0, W0 = O.initial_radiation_field(model)
    o0, _ = _oracle_model(model, spec, T0, W0)
    raw0 = O.run(o0, T, N, iteration=0)
    fin0 = O.finalise(o0, raw0, T, T_R_prev=T0, W_prev=W0)
    o1, _ = _oracle_model(model, spec, fin0["T_R"], fin0["W"])
    raw1 = O.run(o1, T, N, iteration=1)

    assert raw0["counters"]["line_events"] > 1000
    assert_packets_match(g0, raw0["packets"])
    if divergent(g0, raw0["packets"]).size == 0:
        _assert_tables(g_tables1, o1, 1e-8)
    assert_packets_match(g1, raw1["packets"])
    if divergent(g1, raw1["packets"]).size == 0:
        assert c1 == raw1["counters"]
    assert not np.array_equal(o0.em_cum, o1.em_cum)


def test_macroatom_with_derived_tables_in_a_batch(ctx):
    model, spec = _small(5)
    other = W.small_model(seed=81, n_shells=4, n_lines=300)
    F = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, 2000, flags=F)
    pl = smc.Plasma(m, spec)
    pl.update(ION, EXC)
    m2 = smc.Model(ctx, other, 1500, flags=F)
    ctx.batch_run([m, m2], [dict(n_packets=2000, T_inner=12000.0, flags=F),
                            dict(n_packets=1500, T_inner=10000.0, flags=F)],
                  tune=dict(long_budget=4))
    T0, W0 = O.initial_radiation_field(model)
    o, _ = _oracle_model(model, spec, T0, W0)
    raw = O.run(o, 12000.0, 2000)
    if assert_packets_match(m.read_packets(2000), raw["packets"]).size == 0:
        assert m.read_counters() == raw["counters"]


def test_errors(ctx):
    import torch
    model, spec = _small(6, n_lines=500, n_shells=3)
    m = smc.Model(ctx, model, 100, flags=smc.F_JBLUE)
    # no iteration, and no table read, before the first update
    with pytest.raises(smc.SmcError, match="plasma"):
        m.run_iteration(100, 10000.0)
    with pytest.raises(smc.SmcError, match="derived"):
        m.read_macroatom()
    # the atom must be the model's
    other, spec2 = _small(7, n_lines=500, n_shells=3)
    with pytest.raises(smc.SmcError):
        smc.Plasma(m, spec2)
    # detailed J_b needs J_blue tallies
    m_nojb = smc.Model(ctx, model, 100, flags=0)
    pl = smc.Plasma(m_nojb, spec)
    with pytest.raises(smc.SmcError, match="JBLUE"):
        pl.update(ION, EXC, jblue_mode=smc.JB_DETAILED)
    # workspaces must be device memory from hipMalloc
    need = smc.workspace_bytes(model, 100, smc.F_JBLUE)
    host = torch.empty(need + 256, dtype=torch.uint8).pin_memory()
    off = (-host.data_ptr()) % 256
    with pytest.raises(smc.SmcError, match="device memory"):
        smc.Model(ctx, model, 100, flags=smc.F_JBLUE, workspace=host[off:off + need])
    # a scatter model has no tables to read
    sm = smc.Model(ctx, W.small_model(seed=1), 100, flags=0)
    with pytest.raises(smc.SmcError, match="no macro-atom"):
        sm.read_macroatom()
