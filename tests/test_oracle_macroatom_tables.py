"""Pins of the oracle's macro-atom tables from the plasma state (section 2.5:
the macro atom of Lucy 2002, 2003 with bound-bound radiative transitions)
against what the physics and the mathematics fix, not against its formulas:

* detailed balance: in LTE (J_b = B_nu(T), Boltzmann populations) every
  line's radiative rates balance, n_l R_lu = n_u R_ul, which holds only with
  the Einstein relations, the statistical weights, the Planck function and
  stimulated emission all right;
* Kirchhoff: in LTE a macro atom activated by each line's absorbed energy
  re-emits, on average, exactly that energy in that same line;
* Lucy's theorem out of LTE: with populations in statistical equilibrium
  under the same rates (any J_b: dilute blackbody or an arbitrary J_blue),
  the energy the activated macro atom returns in each line is
  n_u R_ul (e_u - e_l), its emissivity -- the property the energy-flow
  weights exist for; a wrong energy factor in any kind of entry breaks it;
* the weights of a row add up to e_i times the total rate out of level i;
* the row layout (three entries per line, kinds and line order) and the
  degenerate rows (a two-level atom always deactivates; a row of zero weight
  takes equal steps).
The emitted energy per line is the absorption probability of the Markov
chain the tables define, computed by a linear solve.  No GPU is needed.
"""
import numpy as np

from oracle import macroatom as MA
from oracle import plasma as P
from paper_1401_5469_amd import workloads as W

EV = 1.602176634e-12


def _atom(seed, n_levels=5, f_zero=()):
    """One ion with a line between every pair of its levels."""
    rng = np.random.default_rng(seed)
    e = np.concatenate([[0.0], np.sort(rng.uniform(1.0, 9.0, n_levels - 1))]) * EV
    g = rng.integers(1, 10, n_levels).astype(np.float64)
    lo, up = np.triu_indices(n_levels, k=1)
    nu = (e[up] - e[lo]) / P.H
    order = np.argsort(-nu, kind="stable")
    lo, up, nu = lo[order], up[order], nu[order]
    f = 10.0 ** rng.uniform(-3.0, 0.0, lo.size)
    for k in f_zero:
        f[k] = 0.0
    atom = W.PlasmaAtom(
        element_ion_ptr=np.array([0, 1], dtype=np.int32), ion_chi=np.array([12.0 * EV]),
        ion_zeta=np.array([0.5]), ion_level_ptr=np.array([0, n_levels], dtype=np.int32),
        level_energy=e, level_g=g, level_metastable=np.zeros(n_levels, dtype=np.uint8),
        line_lower=lo.astype(np.int32), line_upper=up.astype(np.int32), line_f=f)
    tau = 10.0 ** rng.uniform(-3.0, 3.0, lo.size)
    return atom, nu, tau


def _emitted(atom, level_ptr, em_line, cum, activation):
    """Energy returned per line when levels are activated at `activation`
    (energy per unit time into each level): E = a + Q^T E, emission E R."""
    n, L = atom.n_levels, atom.line_lower.shape[0]
    Q = np.zeros((n, n))
    R = np.zeros((n, L))
    for i in range(n):
        a, b = level_ptr[i], level_ptr[i + 1]
        p = np.diff(np.concatenate([[0.0], cum[a:b]]))
        for j, pj in zip(range(a, b), p):
            if em_line[j] >= 0:
                R[i, em_line[j]] += pj
            else:
                Q[i, -em_line[j] - 1] += pj
    E = np.linalg.solve(np.eye(n) - Q.T, activation)
    return E @ R


def _close(got, want):
    # the linear solve spans many decades of line strength: relative 1e-8,
    # or 1e-12 of the strongest line (a wrong weight is off by O(1))
    np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-12 * np.abs(want).max())


def _activation(atom, pop, R_up):
    """Absorbed energy per unit time into each upper level, and per line."""
    e = atom.level_energy
    lo, up = atom.line_lower, atom.line_upper
    per_line = pop[lo] * R_up * (e[up] - e[lo])
    act = np.zeros(atom.n_levels)
    np.add.at(act, up, per_line)
    return act, per_line


def test_detailed_balance_and_kirchhoff_in_lte():
    atom, nu, tau = _atom(1)
    T = 9000.0
    R_down, R_up = MA.line_rates(atom, nu, tau, P.planck(nu, T))
    e, g = atom.level_energy, atom.level_g
    pop = g * np.exp(-e / (P.K_B * T))
    lo, up = atom.line_lower, atom.line_upper
    np.testing.assert_allclose(pop[lo] * R_up, pop[up] * R_down, rtol=1e-12)
    level_ptr, em_line, cum = MA.tables(atom, nu, tau[None, :], np.array([T]), np.array([1.0]))
    act, absorbed = _activation(atom, pop, R_up)
    _close(_emitted(atom, level_ptr, em_line, cum[0], act), absorbed)


def _equilibrium(atom, R_down, R_up):
    """Populations (summing to 1) in statistical equilibrium of the radiative
    rates."""
    n = atom.n_levels
    M = np.zeros((n, n))
    for k, (lo, up) in enumerate(zip(atom.line_lower, atom.line_upper)):
        M[lo, up] += R_down[k]
        M[up, up] -= R_down[k]
        M[up, lo] += R_up[k]
        M[lo, lo] -= R_up[k]
    M[0, :] = 1.0
    rhs = np.zeros(n)
    rhs[0] = 1.0
    return np.linalg.solve(M, rhs)


def test_lucy_energy_flow_out_of_lte():
    for seed, jblue in ((2, None), (3, None), (4, "random")):
        atom, nu, tau = _atom(seed, n_levels=6)
        T_R, Wd = 14000.0, 0.2
        J_b = Wd * P.planck(nu, T_R)
        if jblue is not None:
            J_b = J_b * 10.0 ** np.random.default_rng(seed).uniform(-2.0, 1.0, nu.size)
        R_down, R_up = MA.line_rates(atom, nu, tau, J_b)
        pop = _equilibrium(atom, R_down, R_up)
        assert np.all(pop > 0.0)
        level_ptr, em_line, cum = MA.tables(atom, nu, tau[None, :], np.array([T_R]),
                                            np.array([Wd]),
                                            jblue=None if jblue is None else J_b[None, :])
        act, _ = _activation(atom, pop, R_up)
        e = atom.level_energy
        lo, up = atom.line_lower, atom.line_upper
        emissivity = pop[up] * R_down * (e[up] - e[lo])
        _close(_emitted(atom, level_ptr, em_line, cum[0], act), emissivity)


def test_row_weights_add_up_to_the_energy_flow_out_of_the_level():
    atom, nu, tau = _atom(5, n_levels=7)
    J_b = 0.3 * P.planck(nu, 11000.0)
    lay = MA.layout(atom.n_levels, atom.line_lower, atom.line_upper)
    w = MA.row_weights(atom, nu, tau, J_b, lay)
    R_down, R_up = MA.line_rates(atom, nu, tau, J_b)
    for i in range(atom.n_levels):
        out = R_down[atom.line_upper == i].sum() + R_up[atom.line_lower == i].sum()
        a, b = lay[0][i], lay[0][i + 1]
        assert np.isclose(w[a:b].sum(), atom.level_energy[i] * out, rtol=1e-13, atol=0.0)


def test_layout_three_entries_per_line():
    model, spec = W.macroatom_plasma_model(seed=3, n_shells=2, n_levels_per_ion=12,
                                           n_lines=300)
    a = spec.atom
    level_ptr, em_line, em_via, em_kind = MA.layout(a.n_levels, a.line_lower, a.line_upper)
    L = a.line_lower.shape[0]
    assert level_ptr[-1] == 3 * L == em_line.shape[0]
    assert np.array_equal(np.bincount(em_via, minlength=L), np.full(L, 3))
    for i in range(a.n_levels):
        r = slice(level_ptr[i], level_ptr[i + 1])
        kinds, via, line = em_kind[r], em_via[r], em_line[r]
        assert np.all(np.diff(kinds) >= 0)  # deactivations, jumps down, jumps up
        for kind in (MA.EMIT, MA.DOWN, MA.UP):
            assert np.all(np.diff(via[kinds == kind]) > 0)  # line order
        assert np.array_equal(line[kinds == MA.EMIT], via[kinds == MA.EMIT])
        assert np.all(a.line_upper[via[kinds != MA.UP]] == i)
        assert np.all(a.line_lower[via[kinds == MA.UP]] == i)
        assert np.array_equal(-line[kinds == MA.DOWN] - 1, a.line_lower[via[kinds == MA.DOWN]])
        assert np.array_equal(-line[kinds == MA.UP] - 1, a.line_upper[via[kinds == MA.UP]])
        assert np.array_equal(via[kinds == MA.EMIT], np.flatnonzero(a.line_upper == i))


def test_degenerate_rows():
    # two levels: the upper one always deactivates (its jump down would land
    # on the ground state, energy 0); the ground row has weight 0
    atom, nu, tau = _atom(6, n_levels=2)
    level_ptr, em_line, cum = MA.tables(atom, nu, tau[None, :], np.array([9000.0]),
                                        np.array([0.5]))
    assert list(level_ptr) == [0, 1, 3]
    assert list(em_line) == [-2, 0, -1]
    assert list(cum[0]) == [1.0, 1.0, 1.0]
    # a level whose lines all have f = 0 has a row of zero weight: equal steps
    atom, nu, tau = _atom(7, n_levels=3, f_zero=(0, 1, 2))
    level_ptr, em_line, cum = MA.tables(atom, nu, tau[None, :], np.array([9000.0]),
                                        np.array([0.5]))
    top = slice(level_ptr[2], level_ptr[3])
    assert np.allclose(cum[0][top], np.arange(1, 5) / 4.0, rtol=0, atol=0)


def test_shells_take_their_own_state():
    atom, nu, tau = _atom(8, n_levels=5)
    taus = np.stack([tau, tau * 100.0])
    level_ptr, em_line, cum = MA.tables(atom, nu, taus, np.array([9000.0, 12000.0]),
                                        np.array([0.5, 0.1]))
    one = MA.tables(atom, nu, taus[1:], np.array([12000.0]), np.array([0.1]))[2]
    assert np.array_equal(cum[1], one[0])
    assert not np.array_equal(cum[0], cum[1])
