"""CPU oracle of the macro-atom transition tables (section 2.5: the macro
atom of Lucy 2002, 2003 with bound-bound radiative transitions only), from
the plasma state of section 2.3.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the benchmark's CPU
baseline use this module; the product path never does.  Plain numpy in FP64,
sharing no code with the HIP path.

A bound-bound absorption in line l -> u activates the macro atom in level u.
From a level i the atom either deactivates radiatively (returns an r-packet
in a downward line i -> l) or makes an internal jump to another level, with
probabilities proportional to the energy each transition carries (Lucy's
energy-flow form of the rate equations).  With the radiative rates of a
Sobolev line (the same rates the NLTE statistical equilibrium of the plasma
oracle uses):

    downward, per atom in the upper level:  R_ul = beta (A_ul + B_ul J_b)
    upward, per atom in the lower level:    R_lu = beta B_lu J_b

with beta = (1 - exp(-tau_S)) / tau_S of the line in the shell and J_b the
mean intensity at the line (W B_nu(T_R) in the dilute-blackbody mode, the
J_blue estimator in the detailed mode), the weights from level i (energy
e_i above its ion's ground state) are

    radiative deactivation in a line i -> l:  R_il (e_i - e_l)
    internal downward jump to l:              R_il e_l
    internal upward jump along a line i -> u: R_iu e_i

and they add up to e_i times the total rate out of i.  A row whose weights
are all zero (the ground state: e = 0) takes equal probabilities; no
absorption ever activates such a level, and no jump reaches it.

Row layout (one row per level, the order both implementations use): the
level's downward lines as deactivations, in line order; the same lines as
internal downward jumps, in line order; the level's upward lines as
internal upward jumps, in line order.  em_line holds the line of a
deactivation and -(j + 1) for a jump to level j; em_cum the cumulative
probabilities, one set per shell, with the last entry of every row 1.
"""
from __future__ import annotations

import numpy as np

from oracle import plasma as P

EMIT, DOWN, UP = 0, 1, 2


def layout(n_levels, line_lower, line_upper):
    """The rows: level_ptr [n_levels+1], em_line, and per entry its line
    (em_via) and kind (EMIT, DOWN, UP)."""
    line_lower = np.asarray(line_lower)
    line_upper = np.asarray(line_upper)
    rows = [[] for _ in range(n_levels)]
    for k in range(line_lower.shape[0]):
        rows[int(line_upper[k])].append((EMIT, k))
    for k in range(line_lower.shape[0]):
        rows[int(line_upper[k])].append((DOWN, k))
    for k in range(line_lower.shape[0]):
        rows[int(line_lower[k])].append((UP, k))
    level_ptr = np.zeros(n_levels + 1, dtype=np.int64)
    em_line, em_via, em_kind = [], [], []
    for i, row in enumerate(rows):
        for kind, k in row:
            if kind == EMIT:
                em_line.append(k)
            elif kind == DOWN:
                em_line.append(-(int(line_lower[k]) + 1))
            else:
                em_line.append(-(int(line_upper[k]) + 1))
            em_via.append(k)
            em_kind.append(kind)
        level_ptr[i + 1] = len(em_line)
    return (level_ptr, np.array(em_line, dtype=np.int32), np.array(em_via, dtype=np.int64),
            np.array(em_kind, dtype=np.int8))


def line_rates(atom, line_nu, tau_s, J_b):
    """R_ul and R_lu of every line in one shell."""
    g_l = atom.level_g[atom.line_lower]
    g_u = atom.level_g[atom.line_upper]
    A_ul, B_ul, B_lu = P.einstein_coefficients(atom.line_f, np.asarray(line_nu), g_l, g_u)
    beta = P.sobolev_beta(tau_s)
    return beta * (A_ul + B_ul * J_b), beta * B_lu * J_b


def row_weights(atom, line_nu, tau_s, J_b, lay):
    """The unnormalised weights of every entry in one shell."""
    level_ptr, em_line, em_via, em_kind = lay
    R_down, R_up = line_rates(atom, line_nu, tau_s, J_b)
    e = atom.level_energy
    e_row = e[np.repeat(np.arange(level_ptr.shape[0] - 1), np.diff(level_ptr))]
    e_low = e[atom.line_lower[em_via]]
    return np.where(em_kind == EMIT, R_down[em_via] * (e_row - e_low),
                    np.where(em_kind == DOWN, R_down[em_via] * e_low, R_up[em_via] * e_row))


def cumulative(w, level_ptr):
    """Per row: running sums in entry order over the row's total (equal
    steps if the total is 0), the last entry exactly 1."""
    cum = np.zeros(w.shape[0])
    for i in range(level_ptr.shape[0] - 1):
        a, b = int(level_ptr[i]), int(level_ptr[i + 1])
        if b == a:
            continue
        run = np.cumsum(w[a:b])
        total = run[-1]
        cum[a:b] = run / total if total > 0.0 else np.arange(1, b - a + 1) / (b - a)
        cum[b - 1] = 1.0
    return cum


def tables(atom, line_nu, tau, T_R, W, jblue=None):
    """level_ptr, em_line and em_cum [S, n_em] of the macroatom mode for the
    Sobolev depths tau [S, L] and the radiation field: J_b = W B_nu(T_R) per
    shell, or the J_blue estimator jblue [S, L] (detailed mode)."""
    lay = layout(atom.n_levels, atom.line_lower, atom.line_upper)
    level_ptr, em_line = lay[0], lay[1]
    S = np.asarray(T_R).shape[0]
    line_nu = np.asarray(line_nu, dtype=np.float64)
    em_cum = np.zeros((S, em_line.shape[0]))
    for s in range(S):
        J_b = W[s] * P.planck(line_nu, T_R[s]) if jblue is None else np.asarray(jblue[s])
        em_cum[s] = cumulative(row_weights(atom, line_nu, tau[s], J_b, lay), level_ptr)
    return level_ptr, em_line, em_cum
