"""Pins of the plasma oracle (section 2.3 ionization and excitation, the
Sobolev depth of section 2.5) against what the mathematics and published
constants fix, independently of the oracle's own formulas:

* the thermal factor (2 pi m_e k / h^2)^{3/2} = 2.4147e15 cm^-3 K^-3/2 and
  the classical line constant pi e^2 / (m_e c) = 2.6540e-2 cm^2 s^-1
  (textbook values);
* a hydrogen-like element (two stages) solves a quadratic, a three-stage
  element a cubic: their roots, from numpy's polynomial solver, are n_e;
* the nebular factor W [delta zeta + W (1 - zeta)] (T_e/T_R)^{1/2} with
  T_e = 0.9 T_R, checked through the same closed forms;
* two-level partition functions and populations, Boltzmann and dilute;
* the stimulated-emission factor 1 - exp(-h nu / k T) (LTE) and
  1 - W exp(-h nu / k T) (dilute, metastable lower level), and the clamp of
  inverted lines;
* invariants on a random synthetic atom: every element's stages sum to its
  density, the ion charges sum to n_e, every ion's levels sum to its
  density, n_e grows with T_R in LTE and tends to full ionization.
None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest

from oracle import plasma as P
from paper_1401_5469_amd import workloads as W

EV = 1.602176634e-12
K_B = 1.380649e-16
H = 6.62607015e-27
C = 2.99792458e10

SAHA_THERMAL = 2.4147e15      # (2 pi m_e k / h^2)^{3/2}, cm^-3 K^-3/2 (textbook value)
LINE_CONST = 2.6540e-2        # pi e^2 / (m_e c), cm^2 s^-1 (textbook value)


def _atom(stages, lines=(), line_f=None):
    """stages: per element a list of ions, each a list of (energy eV, g,
    metastable) levels, plus the ion's chi [eV] and zeta."""
    ion_ptr, chi, zeta, lev_ptr, e, g, meta = [0], [], [], [0], [], [], []
    for elem in stages:
        for ion in elem:
            levels, c, z = ion
            chi.append(c * EV)
            zeta.append(z)
            for en, gg, mm in levels:
                e.append(en * EV)
                g.append(gg)
                meta.append(mm)
            lev_ptr.append(len(e))
        ion_ptr.append(len(chi))
    lo = np.array([a for a, _ in lines], dtype=np.int32)
    up = np.array([b for _, b in lines], dtype=np.int32)
    f = np.asarray(line_f if line_f is not None else np.full(len(lines), 0.5), dtype=np.float64)
    return W.PlasmaAtom(
        element_ion_ptr=np.array(ion_ptr, dtype=np.int32), ion_chi=np.array(chi),
        ion_zeta=np.array(zeta), ion_level_ptr=np.array(lev_ptr, dtype=np.int32),
        level_energy=np.array(e), level_g=np.array(g, dtype=np.float64),
        level_metastable=np.array(meta, dtype=np.uint8), line_lower=lo, line_upper=up,
        line_f=f)


HYDROGEN = [[([(0.0, 2.0, 1)], 13.598, 0.5), ([(0.0, 1.0, 1)], 0.0, 0.0)]]


def _state(atom, N, T, Wd, ion=P.ION_LTE, exc=P.EXC_LTE, delta=1.0, nu=None, t_exp=1.0e6):
    S = len(T)
    nu = np.zeros(0) if nu is None else np.asarray(nu, dtype=np.float64)
    return P.plasma_state(atom, np.asarray(N, dtype=np.float64).reshape(S, -1), nu, t_exp,
                          np.asarray(T, dtype=np.float64), np.asarray(Wd, dtype=np.float64),
                          ion, exc, delta)


def _quadratic_ne(N, phi):
    # n_e^2 / (N - n_e) = phi: the positive root of n_e^2 + phi n_e - N phi
    r = np.roots([1.0, phi, -N * phi])
    return float(r[(r.real > 0) & (abs(r.imag) < 1e-9 * abs(r.real))].real[0])


@pytest.mark.parametrize("T,N", [(6000.0, 1e9), (9000.0, 3e10), (12000.0, 1e12), (20000.0, 1e8)])
def test_hydrogen_saha_is_a_quadratic(T, N):
    atom = _atom(HYDROGEN)
    r = _state(atom, [[N]], [T], [1.0])
    phi = (2.0 * 1.0 / 2.0) * SAHA_THERMAL * T ** 1.5 * math.exp(-13.598 * EV / (K_B * T))
    ne = _quadratic_ne(N, phi)
    assert r["n_e"][0] == pytest.approx(ne, rel=5e-5)
    # the neutral density n_e^2 / phi stays sensitive to phi when nearly all
    # of the gas is ionized
    np.testing.assert_allclose(r["N_ion"][0], [ne * ne / phi, ne], rtol=2e-4)


@pytest.mark.parametrize("Wd,zeta,delta", [(1.0, 0.5, 1.0), (0.5, 0.3, 2.0), (0.05, 0.9, 1.0),
                                           (0.2, 0.0, 0.3)])
def test_nebular_factor_through_the_quadratic(Wd, zeta, delta):
    atom = _atom([[([(0.0, 2.0, 1)], 13.598, zeta), ([(0.0, 1.0, 1)], 0.0, 0.0)]])
    for T, N in ((6000.0, 1e9), (10000.0, 1e10)):
        r = _state(atom, [[N]], [T], [Wd], ion=P.ION_NEBULAR, delta=delta)
        phi = SAHA_THERMAL * T ** 1.5 * math.exp(-13.598 * EV / (K_B * T))
        phi *= Wd * (delta * zeta + Wd * (1.0 - zeta)) * math.sqrt(0.9)
        ne = _quadratic_ne(N, phi)
        assert r["n_e"][0] == pytest.approx(ne, rel=5e-5)
        np.testing.assert_allclose(r["N_ion"][0], [ne * ne / phi, ne], rtol=2e-4)


def test_three_stages_solve_a_cubic():
    # stage charges 0, 1, 2: n_e = N (r1 + 2 r2) / (1 + r1 + r2), r1 = p1/x,
    # r2 = p1 p2 / x^2  =>  x^3 + p1 x^2 + (p1 p2 - N p1) x - 2 N p1 p2 = 0
    atom = _atom([[([(0.0, 1.0, 1)], 24.587, 0.5), ([(0.0, 2.0, 1)], 54.418, 0.5),
                   ([(0.0, 1.0, 1)], 0.0, 0.0)]])
    T, N = 25000.0, 1e11
    r = _state(atom, [[N]], [T], [1.0])
    th = SAHA_THERMAL * T ** 1.5
    p1 = 2.0 * (2.0 / 1.0) * th * math.exp(-24.587 * EV / (K_B * T))
    p2 = 2.0 * (1.0 / 2.0) * th * math.exp(-54.418 * EV / (K_B * T))
    roots = np.roots([1.0, p1, p1 * p2 - N * p1, -2.0 * N * p1 * p2])
    x = float(roots[(abs(roots.imag) < 1e-6 * abs(roots.real)) & (roots.real > 0)].real[0])
    assert r["n_e"][0] == pytest.approx(x, rel=5e-5)
    r1, r2 = p1 / x, p1 * p2 / x ** 2
    want = N * np.array([1.0, r1, r2]) / (1.0 + r1 + r2)
    np.testing.assert_allclose(r["N_ion"][0], want, rtol=2e-4)


def test_two_level_partition_function_and_populations():
    # neutral stage with a ground level (g 2) and a non-metastable level
    # (g 6, 2 eV); a second element-less check of dilute weighting
    levels = [(0.0, 2.0, 1), (2.0, 6.0, 0)]
    atom = _atom([[(levels, 13.0, 0.5), ([(0.0, 1.0, 1)], 0.0, 0.0)]])
    T, Wd, N = np.array([8000.0, 15000.0]), np.array([0.4, 0.1]), [[1e9], [1e9]]
    b = 6.0 * np.exp(-2.0 * EV / (K_B * T))
    for exc, w in ((P.EXC_LTE, np.ones(2)), (P.EXC_DILUTE_LTE, Wd)):
        r = _state(atom, N, T, Wd, exc=exc)
        np.testing.assert_allclose(r["Z"][:, 0], 2.0 + w * b, rtol=1e-14)
        np.testing.assert_allclose(r["Z"][:, 1], 1.0, rtol=0)
        pop = r["level_pop"]
        N0 = r["N_ion"][:, 0]
        np.testing.assert_allclose(pop[:, 0], N0 * 2.0 / (2.0 + w * b), rtol=1e-13)
        np.testing.assert_allclose(pop[:, 1], N0 * w * b / (2.0 + w * b), rtol=1e-13)


def test_sobolev_constant_and_stimulated_emission():
    # one ion with levels 0 (ground), 1 (metastable, 1.5 eV), 2 (not
    # metastable, 3.1 eV) and 3 (metastable, 3.3 eV); lines 0->2 and 1->2
    # have a metastable lower level, line 2->3 a non-metastable lower and a
    # metastable upper level, which inverts in dilute-LTE
    levels = [(0.0, 2.0, 1), (1.5, 4.0, 1), (3.1, 6.0, 0), (3.3, 2.0, 1)]
    lines = [(0, 2), (1, 2), (2, 3)]
    atom = _atom([[(levels, 20.0, 0.5), ([(0.0, 1.0, 1)], 0.0, 0.0)]], lines,
                 line_f=[0.3, 0.05, 0.01])
    e = np.array([0.0, 1.5, 3.1, 3.3]) * EV
    g = np.array([2.0, 4.0, 6.0, 2.0])
    nu = np.array([(e[u] - e[l]) / H for l, u in lines])
    t_exp = 13 * 86400.0
    T, Wd = np.array([9000.0]), np.array([0.3])
    for exc in (P.EXC_LTE, P.EXC_DILUTE_LTE):
        r = _state(atom, [[1e9]], T, Wd, exc=exc, nu=nu, t_exp=t_exp)
        pop = r["level_pop"][0]
        for k, (l, u) in enumerate(lines):
            x = H * nu[k] / (K_B * T[0])
            if exc == P.EXC_LTE:
                stim = -math.expm1(-x)
            else:
                wl = 1.0 if l in (0, 1, 3) else Wd[0]
                wu = 1.0 if u in (0, 1, 3) else Wd[0]
                stim = 1.0 - (wu / wl) * math.exp(-x)
            want = LINE_CONST * atom.line_f[k] * (C / nu[k]) * t_exp * pop[l] * stim
            if stim > 0:
                assert r["tau"][0, k] == pytest.approx(want, rel=1e-4)
            else:
                assert r["tau"][0, k] == 0.0
        # line 2 (lower level not metastable, upper metastable) inverts in
        # dilute-LTE: exp(-0.2 eV / kT) / W > 1
        assert r["n_clamped"] == (1 if exc == P.EXC_DILUTE_LTE else 0)
        assert math.exp(-0.2 * EV / (K_B * T[0])) / Wd[0] > 1.0


def _random_atom(seed=3, n_lines=3000):
    rng = np.random.default_rng(seed)
    atom, nu = W.synthetic_plasma_atom(rng, n_elements=6, n_stages=5, n_levels_per_ion=25,
                                       n_lines=n_lines)
    return atom, nu


@pytest.mark.parametrize("ion,exc", [(P.ION_LTE, P.EXC_LTE), (P.ION_NEBULAR, P.EXC_DILUTE_LTE),
                                     (P.ION_NEBULAR, P.EXC_LTE), (P.ION_LTE, P.EXC_DILUTE_LTE)])
def test_conservation_invariants(ion, exc):
    atom, nu = _random_atom()
    S = 6
    rng = np.random.default_rng(9)
    N = 10.0 ** rng.uniform(6.0, 10.0, (S, atom.n_elements))
    T = rng.uniform(5000.0, 30000.0, S)
    Wd = rng.uniform(0.05, 0.6, S)
    r = P.plasma_state(atom, N, nu, 1e6, T, Wd, ion, exc, delta=0.7)
    ep = atom.element_ion_ptr
    charge = np.concatenate([np.arange(ep[e + 1] - ep[e]) for e in range(atom.n_elements)])
    for s in range(S):
        for e in range(atom.n_elements):
            assert r["N_ion"][s, ep[e]:ep[e + 1]].sum() == pytest.approx(N[s, e], rel=1e-13)
        assert (r["N_ion"][s] * charge).sum() == pytest.approx(r["n_e"][s], rel=1e-13)
        lp = atom.ion_level_ptr
        for i in range(atom.n_ions):
            got = r["level_pop"][s, lp[i]:lp[i + 1]].sum()
            assert got == pytest.approx(r["N_ion"][s, i], rel=1e-12, abs=1e-300)
    assert np.all(r["level_pop"] >= 0) and np.all(r["tau"] >= 0)
    # the root is bracketed to adjacent doubles: the charge balance changes
    # sign across n_e
    for s in range(S):
        tab, n_st = P._stage_table(atom, r["log_ratio"][s])
        q = np.arange(tab.shape[1] + 1.0)

        def g(x):
            return np.sum(N[s] * (P.stage_fractions(tab, x) @ q)) - x
        x = r["n_e"][s]
        assert g(x * (1 - 1e-12)) > 0 > g(x * (1 + 1e-12))


def test_electron_density_grows_with_temperature_to_full_ionization():
    atom, nu = _random_atom(seed=4)
    N = np.full((1, atom.n_elements), 1e8)
    full = float(np.sum(N[0] * (np.diff(atom.element_ion_ptr) - 1)))
    prev = 0.0
    for T in (3000.0, 6000.0, 10000.0, 20000.0, 40000.0):
        ne = P.plasma_state(atom, N, nu, 1e6, [T], [1.0], P.ION_LTE, P.EXC_LTE)["n_e"][0]
        assert ne > prev
        prev = ne
    hot = P.plasma_state(atom, N, nu, 1e6, [3e6], [1.0], P.ION_LTE, P.EXC_LTE)["n_e"][0]
    assert hot == pytest.approx(full, rel=1e-3)
