"""Plasma state and Sobolev depths (sections 2.3, 2.5) on the GPU against the
plasma oracle: n_e, partition functions, ion densities, level populations
and tau_S in every ionization / excitation mode, at the paper-scale size
(20 shells, 3e5 lines) and on small and degenerate atoms; the radiation
field taken from the host or from the model's last iteration; and the
feedback loop of section 2.8 (iteration -> plasma update -> iteration)
packet by packet.

Tolerance: every quantity is a short FP64 chain (a partition sum, a few
logarithms, an n_e found to ~1e-15 by Newton here and bisection in the
oracle, ion fractions as exponentials of sums of at most a few log ratios of
size <= ~500, a product of five factors), so relative differences of order
1e-13 are expected; the tests use 1e-10.  tau_S is compared against the
scale of its terms, coef * n_l, because 1 - g_l n_u / (g_u n_l) cancels
near population inversion.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import plasma as P
from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import assert_packets_match, divergent

pytestmark = pytest.mark.gpu

TOL = 1e-10
TINY = 1e-250  # absolute floor for values that underflow toward denormals

MODES = [(W.ION_LTE, W.EXC_LTE), (W.ION_NEBULAR, W.EXC_DILUTE_LTE),
         (W.ION_NEBULAR, W.EXC_LTE), (W.ION_LTE, W.EXC_DILUTE_LTE)]
MODE_IDS = ["lte-lte", "nebular-dilute", "nebular-lte", "lte-dilute"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _oracle(model, spec, T_R, Wd, ion, exc, delta=1.0):
    return P.plasma_state(spec.atom, spec.number_density, model.line_nu, model.t_exp, T_R, Wd,
                          ion, exc, delta)


def _tau_scale(model, spec, o):
    a = spec.atom
    const = math.pi * P.E_CHARGE ** 2 / (P.M_E * P.C_LIGHT)
    coef = const * a.line_f * (P.C_LIGHT / model.line_nu) * model.t_exp
    return coef[None, :] * o["level_pop"][:, a.line_lower]


def _assert_state(g, o, model, spec):
    ntot = float(spec.number_density.sum(axis=1).max())
    np.testing.assert_allclose(g["n_e"], o["n_e"], rtol=TOL, atol=0)
    np.testing.assert_allclose(g["Z"], o["Z"], rtol=TOL, atol=0)
    np.testing.assert_allclose(g["N_ion"], o["N_ion"], rtol=TOL, atol=TINY * ntot)
    np.testing.assert_allclose(g["level_pop"], o["level_pop"], rtol=TOL, atol=TINY * ntot)
    if model.n_lines:
        err = np.abs(g["tau"] - o["tau"])
        lim = TOL * (np.abs(o["tau"]) + _tau_scale(model, spec, o)) + 1e-300
        worst = np.unravel_index(np.argmax(err / lim), err.shape)
        assert np.all(err <= lim), f"tau {worst}: {g['tau'][worst]} vs {o['tau'][worst]}"
        assert np.all(g["tau"] >= 0.0)
    assert g["n_clamped"] == o["n_clamped"]


def _field(model, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(5000.0, 30000.0, model.n_shells), rng.uniform(0.05, 0.7, model.n_shells)


def _small(seed=1, n_lines=3000, **kw):
    return W.plasma_model(seed=seed, n_shells=6, n_elements=6, n_stages=5, n_levels_per_ion=25,
                          n_lines=n_lines, **kw)


@pytest.mark.parametrize("ion,exc", MODES, ids=MODE_IDS)
def test_small_atom_host_field(ctx, ion, exc):
    model, spec = _small()
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 11)
    pl.update(ion, exc, delta=0.7, T_R=T_R, W=Wd)
    g = pl.read()
    o = _oracle(model, spec, T_R, Wd, ion, exc, 0.7)
    _assert_state(g, o, model, spec)
    assert o["n_e"].min() > 0


@pytest.mark.parametrize("ion,exc", [MODES[0], MODES[1]], ids=MODE_IDS[:2])
def test_paper_scale_plasma_from_the_initial_field(ctx, ion, exc):
    w, spec = W.config_plasma()
    model = w.model
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    pl.update(ion, exc)  # the model's initial field: 10^4 K, geometric dilution
    g = pl.read()
    T_R, Wd = O.initial_radiation_field(model)
    o = _oracle(model, spec, T_R, Wd, ion, exc)
    _assert_state(g, o, model, spec)
    # the depths reach the transport: the model's n_e is the solved one
    assert np.all(g["n_e"] > 0)
    frac = float((o["tau"] > 1.0).mean())
    assert 0.05 < frac < 0.5


def test_field_of_the_last_iteration(ctx):
    """A plasma update from the radiation field the last iteration left on
    the device (no host field), with delta = 0.5; the oracle takes the same
    steps: its plasma state from the initial field, its own transport on
    those depths, its estimators, its plasma state from them."""
    model, spec = _small(seed=2)
    N, T = 20000, 11000.0
    m = smc.Model(ctx, model, N, flags=smc.F_PACKETS)
    pl = smc.Plasma(m, spec)
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE)
    m.run_iteration(N, T, flags=smc.F_PACKETS)
    g_packets = m.read_packets(N)
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE, delta=0.5)
    g = pl.read()

    T0, W0 = O.initial_radiation_field(model)
    o0 = _oracle(model, spec, T0, W0, W.ION_NEBULAR, W.EXC_DILUTE_LTE)
    m0 = _with(model, o0["tau"], o0["n_e"])
    raw0 = O.run(m0, T, N, iteration=0, want_jblue=False)
    fin0 = O.finalise(m0, raw0, T, T_R_prev=T0, W_prev=W0)
    assert not np.allclose(fin0["T_R"], T0)
    # same histories (none taken the other way at a tie for this seed): the
    # fields agree to the tally tolerance, and so do the plasma states
    assert assert_packets_match(g_packets, raw0["packets"]).size == 0
    o = _oracle(model, spec, fin0["T_R"], fin0["W"], W.ION_NEBULAR, W.EXC_DILUTE_LTE, 0.5)
    _assert_state(g, o, model, spec)


def _with(model, tau, n_e):
    return W.Model(**{**model.__dict__, "tau_sobolev": np.ascontiguousarray(tau),
                      "n_e": np.ascontiguousarray(n_e)})


def test_feedback_loop_packet_by_packet(ctx):
    # iteration 0 on the opacities of the initial field, a plasma update from
    # its estimators, iteration 1 on the new opacities; the oracle takes the
    # same steps with its own transport and plasma state
    model, spec = _small(seed=3, n_lines=2000)
    N, T = 3000, 11000.0
    ion, exc = W.ION_NEBULAR, W.EXC_DILUTE_LTE
    flags = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, N, flags=flags)
    pl = smc.Plasma(m, spec)
    pl.update(ion, exc)
    m.run_iteration(N, T, iteration=0, flags=flags)
    g0 = m.read_packets(N)
    pl.update(ion, exc)
    g_state = pl.read()
    m.run_iteration(N, T, iteration=1, flags=flags)
    g1 = m.read_packets(N)

    T0, W0 = O.initial_radiation_field(model)
    o_state0 = _oracle(model, spec, T0, W0, ion, exc)
    m0 = _with(model, o_state0["tau"], o_state0["n_e"])
    raw0 = O.run(m0, T, N, iteration=0)
    fin0 = O.finalise(m0, raw0, T, T_R_prev=T0, W_prev=W0)
    o_state1 = _oracle(model, spec, fin0["T_R"], fin0["W"], ion, exc)
    m1 = _with(model, o_state1["tau"], o_state1["n_e"])
    raw1 = O.run(m1, T, N, iteration=1)

    assert raw0["counters"]["line_events"] > 1000
    assert_packets_match(g0, raw0["packets"])
    if divergent(g0, raw0["packets"]).size == 0:
        # same histories: the radiation fields agree to the tally tolerance,
        # so the second plasma state does too
        _assert_state(g_state, o_state1, model, spec)
    assert_packets_match(g1, raw1["packets"])
    assert not np.array_equal(o_state0["tau"], o_state1["tau"])


def test_model_without_lines(ctx):
    model, spec = _small(seed=4, n_lines=0)
    assert model.n_lines == 0
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 12)
    pl.update(W.ION_NEBULAR, W.EXC_LTE, T_R=T_R, W=Wd)
    _assert_state(pl.read(), _oracle(model, spec, T_R, Wd, W.ION_NEBULAR, W.EXC_LTE), model, spec)


def _degenerate_spec(model, spec, mode):
    import dataclasses
    a = spec.atom
    dens = spec.number_density.copy()
    if mode == "empty-element":
        dens[:, 1] = 0.0
        return W.PlasmaSpec(atom=a, number_density=dens)
    if mode == "zero-nebular-factor":
        z = a.ion_zeta.copy()
        z[[0, 6, 7]] = 1.0  # with delta = 0: W [delta zeta + W (1 - zeta)] = 0
        return W.PlasmaSpec(atom=dataclasses.replace(a, ion_zeta=z), number_density=dens)
    raise ValueError(mode)


@pytest.mark.parametrize("mode", ["empty-element", "zero-nebular-factor"])
def test_degenerate_compositions(ctx, mode):
    model, spec = _small(seed=5)
    spec = _degenerate_spec(model, spec, mode)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 13)
    delta = 0.0 if mode == "zero-nebular-factor" else 1.0
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE, delta=delta, T_R=T_R, W=Wd)
    o = _oracle(model, spec, T_R, Wd, W.ION_NEBULAR, W.EXC_DILUTE_LTE, delta)
    _assert_state(pl.read(), o, model, spec)
    if mode == "zero-nebular-factor":
        assert np.all(o["N_ion"][:, 1] == 0.0)


def test_single_stage_atom_has_no_electrons(ctx):
    # every element has one stage: no charge is possible and n_e = 0
    a = W.PlasmaAtom(
        element_ion_ptr=np.array([0, 1, 2], dtype=np.int32), ion_chi=np.array([1e-11, 1e-11]),
        ion_zeta=np.array([0.5, 0.5]), ion_level_ptr=np.array([0, 3, 5], dtype=np.int32),
        level_energy=np.array([0.0, 2e-12, 4e-12, 0.0, 3e-12]),
        level_g=np.array([1.0, 3.0, 5.0, 2.0, 4.0]),
        level_metastable=np.array([1, 0, 1, 1, 0], dtype=np.uint8),
        line_lower=np.array([0, 1, 3], dtype=np.int32),
        line_upper=np.array([2, 2, 4], dtype=np.int32), line_f=np.array([0.1, 0.2, 0.3]))
    de = np.array([4e-12, 2e-12, 3e-12]) / W.H
    order = np.argsort(-de, kind="stable")
    a.line_lower, a.line_upper, a.line_f = a.line_lower[order], a.line_upper[order], a.line_f[order]
    v, t, _ = W.shells(3, 11000.0, 20000.0, 13.0)
    model = W.Model(v_bounds=v, t_exp=t, n_e=np.zeros(3), line_nu=de[order].copy(),
                    tau_sobolev=np.zeros((3, 3)))
    spec = W.PlasmaSpec(atom=a, number_density=np.full((3, 2), 1e9))
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = np.array([6000.0, 9000.0, 15000.0]), np.array([0.5, 0.3, 0.1])
    for exc in (W.EXC_LTE, W.EXC_DILUTE_LTE):
        pl.update(W.ION_LTE, exc, T_R=T_R, W=Wd)
        g = pl.read()
        assert np.all(g["n_e"] == 0.0)
        _assert_state(g, _oracle(model, spec, T_R, Wd, W.ION_LTE, exc), model, spec)


def test_extreme_fields(ctx):
    model, spec = _small(seed=6)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R = np.array([2500.0, 3000.0, 50000.0, 2.0e5, 1.0e6, 8000.0])
    Wd = np.array([1.0, 1e-4, 0.9, 0.5, 1.0, 1e-6])
    for ion, exc in MODES:
        pl.update(ion, exc, delta=1.3, T_R=T_R, W=Wd)
        _assert_state(pl.read(), _oracle(model, spec, T_R, Wd, ion, exc, 1.3), model, spec)


def test_errors(ctx):
    model, spec = _small(seed=7, n_lines=100)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    with pytest.raises(smc.SmcError):
        pl.read()  # no update yet
    with pytest.raises(smc.SmcError):
        pl.update(5, W.EXC_LTE)
    with pytest.raises(smc.SmcError):
        pl.update(W.ION_LTE, 7)
    with pytest.raises(smc.SmcError):
        pl.update(W.ION_LTE, W.EXC_LTE, delta=-1.0)
    T_R, Wd = _field(model, 14)
    with pytest.raises(smc.SmcError):
        pl.update(W.ION_LTE, W.EXC_LTE, T_R=T_R)  # W missing
    bad = T_R.copy()
    bad[2] = 0.0
    with pytest.raises(smc.SmcError):
        pl.update(W.ION_LTE, W.EXC_LTE, T_R=bad, W=Wd)
    # a plasma description whose line list is not the model's
    other, ospec = _small(seed=7, n_lines=120)
    with pytest.raises(ValueError):
        smc.Plasma(m, ospec)
    pl.update(W.ION_LTE, W.EXC_LTE, T_R=T_R, W=Wd)
    assert pl.read()["n_e"].min() > 0


# ---------------------------------------------------------------------------
# NLTE statistical equilibrium (section 2.3): the HIP LU solve against the
# oracle's LAPACK solve.  Eliminating the same systems in the kernel's order
# on the CPU differs from LAPACK by < 4e-15 relative on these atoms, so the
# tolerance above holds for the NLTE populations too.
# ---------------------------------------------------------------------------
def _nlte_small(seed=21, n_levels_nlte=20, n_lines=3000):
    return W.plasma_model(seed=seed, n_shells=6, n_elements=6, n_stages=5, n_levels_per_ion=25,
                          n_lines=n_lines, nlte_ions=(6, 11, 27), n_levels_nlte=n_levels_nlte)


def _oracle_nlte(model, spec, T_R, Wd, ion, exc, tau_prev, jblue=None, delta=1.0):
    return P.plasma_state(spec.atom, spec.number_density, model.line_nu, model.t_exp, T_R, Wd,
                          ion, exc, delta, nlte_ions=spec.nlte_ions, tau_prev=tau_prev,
                          jblue=jblue)


@pytest.mark.parametrize("n_levels_nlte", [1, 20, 64])
@pytest.mark.parametrize("ion,exc", [MODES[1], MODES[0]], ids=MODE_IDS[:2][::-1])
def test_nlte_host_field(ctx, n_levels_nlte, ion, exc):
    model, spec = _nlte_small(n_levels_nlte=n_levels_nlte,
                              n_lines=5000 if n_levels_nlte == 64 else 3000)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 31)
    # a first update gives the depths that the escape probabilities use;
    # each side takes its own
    pl.update(ion, exc, T_R=T_R, W=Wd)
    pl.update(ion, exc, T_R=T_R, W=Wd, nlte=True)
    g = pl.read()
    tau0 = _oracle(model, spec, T_R, Wd, ion, exc)["tau"]
    o = _oracle_nlte(model, spec, T_R, Wd, ion, exc, tau0)
    _assert_state(g, o, model, spec)
    assert g["n_singular"] == 0
    base = _oracle(model, spec, T_R, Wd, ion, exc)
    if n_levels_nlte > 1:
        lp = spec.atom.ion_level_ptr
        assert not np.allclose(o["level_pop"][:, lp[6]:lp[7]], base["level_pop"][:, lp[6]:lp[7]])


def test_nlte_paper_scale(ctx):
    w, spec = W.config_plasma_nlte()
    model = w.model
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE, nlte=True)  # initial field, tau_S = 0: beta = 1
    g = pl.read()
    T_R, Wd = O.initial_radiation_field(model)
    o = _oracle_nlte(model, spec, T_R, Wd, W.ION_NEBULAR, W.EXC_DILUTE_LTE,
                     np.zeros((model.n_shells, model.n_lines)))
    _assert_state(g, o, model, spec)
    pl.update(W.ION_NEBULAR, W.EXC_DILUTE_LTE, nlte=True)  # now with the depths just written
    g2 = pl.read()
    o2 = _oracle_nlte(model, spec, T_R, Wd, W.ION_NEBULAR, W.EXC_DILUTE_LTE, o["tau"])
    _assert_state(g2, o2, model, spec)


def test_nlte_detailed_jblue_after_an_iteration(ctx):
    model, spec = _nlte_small(seed=22)
    flags = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, 30000, flags=flags)
    pl = smc.Plasma(m, spec)
    ion, exc = W.ION_NEBULAR, W.EXC_DILUTE_LTE
    # before any iteration the detailed mode starts from W B_nu(T_R)
    pl.update(ion, exc, nlte=True, jblue_mode=smc.JB_DETAILED)
    T0, W0 = O.initial_radiation_field(model)
    g0 = pl.read()
    _assert_state(g0, _oracle_nlte(model, spec, T0, W0, ion, exc,
                                   np.zeros((model.n_shells, model.n_lines))), model, spec)
    m.run_iteration(30000, 12000.0, flags=flags)
    g_packets = m.read_packets(30000)
    pl.update(ion, exc, nlte=True, jblue_mode=smc.JB_DETAILED)
    g = pl.read()
    # the oracle's own chain: its transport on its depths, its estimators
    o0 = _oracle_nlte(model, spec, T0, W0, ion, exc, np.zeros((model.n_shells, model.n_lines)))
    m0 = _with(model, o0["tau"], o0["n_e"])
    raw0 = O.run(m0, 12000.0, 30000, iteration=0)
    fin0 = O.finalise(m0, raw0, 12000.0, T_R_prev=T0, W_prev=W0)
    assert assert_packets_match(g_packets, raw0["packets"]).size == 0
    o = _oracle_nlte(model, spec, fin0["T_R"], fin0["W"], ion, exc, o0["tau"],
                     jblue=fin0["jblue"])
    _assert_state(g, o, model, spec)
    d = _oracle_nlte(model, spec, fin0["T_R"], fin0["W"], ion, exc, o0["tau"])
    lp = spec.atom.ion_level_ptr
    assert not np.allclose(o["level_pop"][:, lp[6]:lp[7]], d["level_pop"][:, lp[6]:lp[7]])


def test_nlte_feedback_loop_packet_by_packet(ctx):
    model, spec = _nlte_small(seed=23, n_lines=2000)
    N, T = 3000, 11000.0
    ion, exc = W.ION_NEBULAR, W.EXC_DILUTE_LTE
    flags = smc.F_JBLUE | smc.F_PACKETS
    m = smc.Model(ctx, model, N, flags=flags)
    pl = smc.Plasma(m, spec)
    pl.update(ion, exc, nlte=True)
    g_state0 = pl.read()
    m.run_iteration(N, T, iteration=0, flags=flags)
    g0 = m.read_packets(N)
    pl.update(ion, exc, nlte=True, jblue_mode=smc.JB_DETAILED)
    g_state1 = pl.read()
    m.run_iteration(N, T, iteration=1, flags=flags)
    g1 = m.read_packets(N)

    T0, W0 = O.initial_radiation_field(model)
    o0 = _oracle_nlte(model, spec, T0, W0, ion, exc, np.zeros((model.n_shells, model.n_lines)))
    _assert_state(g_state0, o0, model, spec)
    m0 = _with(model, o0["tau"], o0["n_e"])
    raw0 = O.run(m0, T, N, iteration=0)
    fin0 = O.finalise(m0, raw0, T, T_R_prev=T0, W_prev=W0)
    assert_packets_match(g0, raw0["packets"])
    o1 = _oracle_nlte(model, spec, fin0["T_R"], fin0["W"], ion, exc, o0["tau"],
                      jblue=fin0["jblue"])
    if divergent(g0, raw0["packets"]).size == 0:
        _assert_state(g_state1, o1, model, spec)
    m1 = _with(model, o1["tau"], o1["n_e"])
    raw1 = O.run(m1, T, N, iteration=1)
    assert_packets_match(g1, raw1["packets"])


def test_nlte_singular_system_keeps_the_excitation_populations(ctx):
    import dataclasses
    model, spec = _nlte_small(seed=24)
    a = spec.atom
    lp = a.ion_level_ptr
    mine = (a.line_lower >= lp[11]) & (a.line_lower < lp[12])
    f = a.line_f.copy()
    ups = a.line_upsilon.copy()
    f[mine] = 0.0
    ups[mine] = 0.0  # no rate at all: the system of ion 11 is singular
    spec = W.PlasmaSpec(atom=dataclasses.replace(a, line_f=f, line_upsilon=ups),
                        number_density=spec.number_density, nlte_ions=spec.nlte_ions)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 32)
    pl.update(W.ION_LTE, W.EXC_LTE, T_R=T_R, W=Wd, nlte=True)
    g = pl.read()
    assert g["n_singular"] == model.n_shells
    base = _oracle(model, spec, T_R, Wd, W.ION_LTE, W.EXC_LTE)
    np.testing.assert_allclose(g["level_pop"][:, lp[11]:lp[12]],
                               base["level_pop"][:, lp[11]:lp[12]], rtol=TOL)
    with_nlte = dataclasses.replace(spec, nlte_ions=(6, 27))
    o = _oracle_nlte(model, with_nlte, T_R, Wd, W.ION_LTE, W.EXC_LTE,
                     np.zeros((model.n_shells, model.n_lines)))
    np.testing.assert_allclose(g["level_pop"][:, lp[6]:lp[7]], o["level_pop"][:, lp[6]:lp[7]],
                               rtol=TOL)


def test_nlte_errors(ctx):
    model, spec = _nlte_small(seed=25, n_lines=2000)
    m = smc.Model(ctx, model, 16, flags=0)
    pl = smc.Plasma(m, spec)
    with pytest.raises(smc.SmcError):  # no J_blue tally in this model
        pl.update(W.ION_LTE, W.EXC_LTE, nlte=True, jblue_mode=smc.JB_DETAILED)
    with pytest.raises(smc.SmcError):
        pl.update(W.ION_LTE, W.EXC_LTE, nlte=True, jblue_mode=3)
    m2 = smc.Model(ctx, model, 1000, flags=smc.F_JBLUE)
    pl2 = smc.Plasma(m2, spec)
    m2.run_iteration(1000, 10000.0, flags=0)  # this iteration does not tally J_blue
    with pytest.raises(smc.SmcError):
        pl2.update(W.ION_LTE, W.EXC_LTE, nlte=True, jblue_mode=smc.JB_DETAILED)
    pl2.update(W.ION_LTE, W.EXC_LTE, nlte=True)  # dilute blackbody is fine


def test_maximum_shells(ctx):
    """4096 shells, the most a model takes (a 3-element atom, 60 lines, two
    NLTE ions of 8 levels): the dilute-LTE state, then the NLTE state whose
    escape probabilities use each side's own first depths."""
    model, spec = W.plasma_model(seed=5, n_shells=4096, n_elements=3, n_stages=3,
                                 n_levels_per_ion=8, n_lines=60, nlte_ions=(1, 4),
                                 n_levels_nlte=8)
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 33)
    ion, exc = W.ION_NEBULAR, W.EXC_DILUTE_LTE
    pl.update(ion, exc, T_R=T_R, W=Wd)
    g0 = pl.read()
    o0 = _oracle(model, spec, T_R, Wd, ion, exc)
    _assert_state(g0, o0, model, spec)
    pl.update(ion, exc, T_R=T_R, W=Wd, nlte=True)
    g1 = pl.read()
    _assert_state(g1, _oracle_nlte(model, spec, T_R, Wd, ion, exc, o0["tau"]), model, spec)
    assert g1["n_singular"] == 0


@pytest.mark.parametrize("ion,exc", [MODES[1], MODES[0]], ids=MODE_IDS[:2][::-1])
def test_atom_beyond_the_staged_level_table(ctx, ion, exc):
    """8800 levels: more than the 8192 whose n/g the depth kernel stages in
    LDS, so the depths gather the populations from device memory instead."""
    model, spec = W.plasma_model(seed=6, n_shells=4, n_elements=8, n_stages=5,
                                 n_levels_per_ion=220, n_lines=5000)
    assert spec.atom.n_levels > 8192
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 34)
    pl.update(ion, exc, T_R=T_R, W=Wd)
    _assert_state(pl.read(), _oracle(model, spec, T_R, Wd, ion, exc), model, spec)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_plasma_configurations(ctx, seed):
    """Seeded random atoms (elements, stages, levels, lines, NLTE ions and
    their level counts), shell counts, fields and modes: the state after a
    plasma update, then after an NLTE update whose escape probabilities use
    each side's own first depths."""
    rng = np.random.default_rng(900 + seed)
    E, St = int(rng.integers(1, 9)), int(rng.integers(1, 6))
    nl = int(rng.integers(2, 30))
    n_ions = E * St
    nlte = tuple(sorted(set(int(i) for i in rng.integers(0, n_ions, int(rng.integers(0, 4))))))
    nl_nlte = int(rng.integers(1, 65))
    L = int(rng.integers(0, 400))
    if nlte:  # room for the ground-state line of every excited NLTE level
        L = max(L, len(nlte) * (nl_nlte - 1) + 10)
    model, spec = W.plasma_model(seed=900 + seed, n_shells=int(rng.integers(1, 30)), n_elements=E,
                                 n_stages=St, n_levels_per_ion=nl, n_lines=L, nlte_ions=nlte,
                                 n_levels_nlte=nl_nlte)
    ion, exc = MODES[seed % 4]
    delta = float(rng.uniform(0.3, 1.5))
    m = smc.Model(ctx, model, 16)
    pl = smc.Plasma(m, spec)
    T_R, Wd = _field(model, 950 + seed)
    pl.update(ion, exc, T_R=T_R, W=Wd, delta=delta)
    o0 = _oracle(model, spec, T_R, Wd, ion, exc, delta)
    _assert_state(pl.read(), o0, model, spec)
    if nlte and model.n_lines:
        pl.update(ion, exc, T_R=T_R, W=Wd, delta=delta, nlte=True)
        o1 = _oracle_nlte(model, spec, T_R, Wd, ion, exc, o0["tau"], delta=delta)
        _assert_state(pl.read(), o1, model, spec)
