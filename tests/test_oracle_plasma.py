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


# ---------------------------------------------------------------------------
# NLTE statistical equilibrium (section 2.3)
# ---------------------------------------------------------------------------
SIGMA_SB = 5.670374419e-5
A_CONST_AA = 6.670e15     # A_ul = 6.670e15 (g_l / g_u) f / lambda[A]^2 s^-1 (textbook value)
COLL_TEXTBOOK = 8.629e-6  # C_ul = 8.629e-6 Upsilon / (g_u T^{1/2}) cm^3 s^-1 (textbook value)


def test_collision_and_einstein_constants():
    assert P.COLL_CONST == pytest.approx(COLL_TEXTBOOK, rel=2e-4)
    # H-alpha: f = 0.6407, g_l = 8, g_u = 18, 6562.8 A -> A_ul = 4.41e7 s^-1
    lam = 6562.8
    A, B_ul, B_lu = P.einstein_coefficients(0.6407, C / (lam * 1e-8), 8.0, 18.0)
    assert A == pytest.approx(A_CONST_AA * 8.0 / 18.0 * 0.6407 / lam ** 2, rel=1e-3)
    assert A == pytest.approx(4.41e7, rel=5e-3)
    assert B_ul * 18.0 == pytest.approx(B_lu * 8.0, rel=1e-14)


def test_planck_and_escape_probability():
    from scipy import integrate
    for T in (5000.0, 12000.0, 30000.0):
        x = np.linspace(1e-4, 60.0, 200001)
        nu = x * K_B * T / H
        tot = integrate.simpson(P.planck(nu, T), x=nu)
        assert tot == pytest.approx(SIGMA_SB * T ** 4 / math.pi, rel=1e-7)
    b = P.sobolev_beta(np.array([0.0, 1e-8, 1.0, 50.0, 1e4]))
    np.testing.assert_allclose(b, [1.0, 1.0 - 5e-9, 1.0 - math.exp(-1.0), 1.0 / 50.0, 1e-4],
                               rtol=1e-14)


def _nlte_atom(n_levels=6, seed=0, all_pairs=False):
    rng = np.random.default_rng(seed)
    e = np.concatenate([[0.0], np.sort(rng.uniform(1.0, 9.0, n_levels - 1))])
    g = rng.integers(1, 8, n_levels).astype(float)
    if all_pairs:
        pairs = [(l, u) for u in range(n_levels) for l in range(u)]
    else:
        pairs = [(0, u) for u in range(1, n_levels)] + [(1, 3), (2, 4)][: max(0, n_levels - 4)]
    de = np.array([e[u] - e[l] for l, u in pairs])
    order = np.argsort(-de, kind="stable")
    pairs = [pairs[i] for i in order]
    f = rng.uniform(0.01, 0.5, len(pairs))
    levels = [(float(e[i]), float(g[i]), 1 if i == 0 else 0) for i in range(n_levels)]
    atom = _atom([[(levels, 20.0, 0.5), ([(0.0, 1.0, 1)], 0.0, 0.0)]], pairs, line_f=f)
    atom.line_upsilon = rng.uniform(0.1, 5.0, len(pairs))
    nu = de[order] * EV / H
    return atom, nu, e * EV, g


def _boltzmann(e, g, T, N):
    w = g * np.exp(-e / (K_B * T))
    return N * w / w.sum()


@pytest.mark.parametrize("tau", [0.0, 3.0, 1e3])
def test_nlte_radiative_equilibrium_is_boltzmann(tau):
    # no electrons, an undiluted Planck field: detailed balance line by line
    # at T_R for any escape probability
    atom, nu, e, g = _nlte_atom(all_pairs=True)
    T, N = 9000.0, 1e7
    taus = np.full(len(nu), tau)
    pop = P.nlte_populations(atom, 0, nu, N, 0.0, T, 1.0, taus, P.planck(nu, T))
    np.testing.assert_allclose(pop, _boltzmann(e, g, T, N), rtol=1e-9)


def test_nlte_collisional_equilibrium_is_boltzmann_at_te():
    # collisions dominate (huge n_e, negligible field): Boltzmann at T_e = 0.9 T_R
    atom, nu, e, g = _nlte_atom(seed=1)
    T, N = 12000.0, 1e7
    pop = P.nlte_populations(atom, 0, nu, N, 1e30, T, 1e-300, np.zeros(len(nu)),
                             np.zeros(len(nu)))
    np.testing.assert_allclose(pop, _boltzmann(e, g, 0.9 * T, N), rtol=1e-8)


@pytest.mark.parametrize("n_e,W,tau", [(0.0, 0.3, 0.0), (1e9, 0.3, 5.0), (1e12, 0.05, 100.0)])
def test_nlte_two_levels_closed_form(n_e, W, tau):
    atom, nu, e, g = _nlte_atom(n_levels=2, seed=2)
    T, N = 10000.0, 1e8
    lam_aa = C / nu[0] / 1e-8
    f, ups = atom.line_f[0], atom.line_upsilon[0]
    A = A_CONST_AA * g[0] / g[1] * f / lam_aa ** 2
    B_ul = A * C ** 2 / (2.0 * H * nu[0] ** 3)
    B_lu = g[1] / g[0] * B_ul
    J = W * 2.0 * H * nu[0] ** 3 / C ** 2 / math.expm1(H * nu[0] / (K_B * T))
    Te = 0.9 * T
    C_ul = COLL_TEXTBOOK * ups / (g[1] * math.sqrt(Te))
    C_lu = C_ul * g[1] / g[0] * math.exp(-H * nu[0] / (K_B * Te))
    b = 1.0 if tau == 0.0 else -math.expm1(-tau) / tau
    ratio = (b * B_lu * J + C_lu * n_e) / (b * A + b * B_ul * J + C_ul * n_e)
    pop = P.nlte_populations(atom, 0, nu, N, n_e, T, W, np.array([tau]),
                             W * P.planck(nu, T))
    np.testing.assert_allclose(pop, [N / (1 + ratio), N * ratio / (1 + ratio)], rtol=2e-3)
    assert pop.sum() == pytest.approx(N, rel=1e-14)


def test_nlte_flux_balance_and_detailed_j():
    # a J_blue array per line (as the estimator gives it): every level's
    # inflow equals its outflow, computed line by line from the oracle's
    # coefficients
    atom, nu, e, g = _nlte_atom(n_levels=7, seed=3, all_pairs=True)
    rng = np.random.default_rng(5)
    T, Wd, n_e, N = 8000.0, 0.4, 3e8, 1e9
    J = P.planck(nu, T) * rng.uniform(0.05, 2.0, len(nu))
    taus = 10.0 ** rng.uniform(-2, 3, len(nu))
    pop = P.nlte_populations(atom, 0, nu, N, n_e, T, Wd, taus, J)
    flow = np.zeros(7)
    scale = np.zeros(7)
    for k in range(len(nu)):
        lo, up = atom.line_lower[k], atom.line_upper[k]
        A, B_ul, B_lu = P.einstein_coefficients(atom.line_f[k], nu[k], g[lo], g[up])
        C_ul, C_lu = P.collision_coefficients(atom.line_upsilon[k], nu[k], g[lo], g[up], 0.9 * T)
        b = float(P.sobolev_beta(taus[k]))
        down = pop[up] * (b * A + b * B_ul * J[k] + C_ul * n_e)
        upw = pop[lo] * (b * B_lu * J[k] + C_lu * n_e)
        flow[lo] += down - upw
        flow[up] += upw - down
        scale[lo] += down + upw
        scale[up] += down + upw
    assert np.all(np.abs(flow) <= 1e-9 * scale)
    assert pop.sum() == pytest.approx(N, rel=1e-13)
    assert np.all(pop > 0)


def test_plasma_state_with_an_nlte_ion():
    rng = np.random.default_rng(6)
    atom, nu = W.synthetic_plasma_atom(rng, n_elements=4, n_stages=4, n_levels_per_ion=20,
                                       n_lines=1500, nlte_ions=(9,), n_levels_nlte=12)
    S = 3
    N = 10.0 ** rng.uniform(7.0, 9.0, (S, atom.n_elements))
    T, Wd = rng.uniform(7000, 15000, S), rng.uniform(0.1, 0.5, S)
    base = P.plasma_state(atom, N, nu, 1e6, T, Wd, P.ION_NEBULAR, P.EXC_DILUTE_LTE)
    r = P.plasma_state(atom, N, nu, 1e6, T, Wd, P.ION_NEBULAR, P.EXC_DILUTE_LTE,
                       nlte_ions=(9,), tau_prev=base["tau"])
    l0, l1 = atom.ion_level_ptr[9], atom.ion_level_ptr[10]
    np.testing.assert_array_equal(r["level_pop"][:, :l0], base["level_pop"][:, :l0])
    np.testing.assert_array_equal(r["level_pop"][:, l1:], base["level_pop"][:, l1:])
    np.testing.assert_allclose(r["level_pop"][:, l0:l1].sum(axis=1), r["N_ion"][:, 9],
                               rtol=1e-12)
    assert not np.allclose(r["level_pop"][:, l0:l1], base["level_pop"][:, l0:l1])
    # the dilute-blackbody J_b = W B_nu(T_R) and the previous depths reach the
    # solve of every shell
    for s in range(S):
        want = P.nlte_populations(atom, 9, nu, r["N_ion"][s, 9], r["n_e"][s], T[s], Wd[s],
                                  base["tau"][s], Wd[s] * P.planck(nu, T[s]))
        np.testing.assert_array_equal(r["level_pop"][s, l0:l1], want)
    mine = (atom.line_lower >= l0) & (atom.line_lower < l1)
    assert mine.sum() >= 11
    np.testing.assert_array_equal(r["tau"][:, ~mine], base["tau"][:, ~mine])
