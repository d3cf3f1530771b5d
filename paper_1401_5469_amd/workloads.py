"""Seeded synthetic workloads for the packet-transport path.

This module builds INPUTS only: shell velocities, electron densities, line
lists, Sobolev optical depths and downbranch emission tables, drawn with
``numpy.random.default_rng(seed)`` in a fixed order.  It holds none of the
transport arithmetic and is shared by the HIP path and the CPU oracle.

The paper's own workloads use Kurucz/CHIANTI atomic data and explosion models
that are not available; these generators stand in for them with the shapes of
the paper's models: 1-D spherical shells in homologous expansion
(Kerzendorf & Sim 2014, section 2.1), a W7-like rho ~ v^-7 density (section
5.3), a frequency-sorted line list with per-shell Sobolev depths (section 2.5).

Draw order of every generator is part of its definition; changing it changes
every downstream value.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# CGS constants needed to build inputs (CODATA 2018 / IAU nominal)
C_LIGHT = 2.99792458e10  # cm/s
M_PROTON = 1.67262192369e-24  # g
ANGSTROM = 1.0e-8  # cm
DAY = 86400.0  # s
KM = 1.0e5  # cm
L_SUN = 3.828e33  # erg/s
H = 6.62607015e-27  # erg s
K_B = 1.380649e-16  # erg/K

SCATTER = 0
DOWNBRANCH = 1
MACROATOM = 2

# emergent spectrum grid: 1000 bins linear in frequency, 500-20000 Angstrom
SPEC_NU_MIN = C_LIGHT / (20000.0 * ANGSTROM)
SPEC_NU_MAX = C_LIGHT / (500.0 * ANGSTROM)
SPEC_BINS = 1000

# requested emergent luminosity: log L/Lsun = 9.44 at 13 days (section 5.3)
L_REQUESTED = 10.0 ** 9.44 * L_SUN


@dataclasses.dataclass
class Model:
    """Arrays in the layout both implementations consume."""

    v_bounds: np.ndarray  # [S+1] cm/s, increasing
    t_exp: float  # s
    n_e: np.ndarray  # [S] cm^-3
    line_nu: np.ndarray  # [L] Hz, non-increasing
    tau_sobolev: np.ndarray  # [S, L] shell-major
    line_mode: int = SCATTER
    line_upper: Optional[np.ndarray] = None  # [L] int32
    n_levels: int = 0
    level_ptr: Optional[np.ndarray] = None  # [n_levels+1] int64
    em_line: Optional[np.ndarray] = None  # [nnz] int32
    em_cum: Optional[np.ndarray] = None  # [nnz] float64
    nu_min: float = SPEC_NU_MIN
    nu_max: float = SPEC_NU_MAX
    n_bins: int = SPEC_BINS
    seed: int = 0

    @property
    def n_shells(self) -> int:
        return int(self.v_bounds.shape[0] - 1)

    @property
    def n_lines(self) -> int:
        return int(self.line_nu.shape[0])

    def nbytes(self) -> int:
        n = self.v_bounds.nbytes + self.n_e.nbytes + self.line_nu.nbytes + self.tau_sobolev.nbytes
        for a in (self.line_upper, self.level_ptr, self.em_line, self.em_cum):
            if a is not None:
                n += a.nbytes
        return n


@dataclasses.dataclass
class Workload:
    name: str
    model: Model
    T_inner: float
    n_packets: int
    n_iterations: int
    L_requested: float = L_REQUESTED
    damping: float = 0.5  # exponent scale of the T_inner update


def _contig(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def shells(n_shells: int, v_inner_kms: float, v_outer_kms: float, t_exp_days: float,
           rho_inner: float = 1.0e-13):
    """Shells evenly spaced in velocity with rho ~ v^-7 at the shell centre,
    normalised to rho_inner in the innermost shell; n_e = rho / (2 m_p)."""
    v = np.linspace(v_inner_kms * KM, v_outer_kms * KM, n_shells + 1)
    v_mid = 0.5 * (v[:-1] + v[1:])
    rho = rho_inner * (v_mid / v_mid[0]) ** -7.0
    n_e = rho / (2.0 * M_PROTON)
    return _contig(v, np.float64), t_exp_days * DAY, _contig(n_e, np.float64)


def log_uniform_lines(rng, n_lines: int, lam_lo_aa: float, lam_hi_aa: float):
    """Wavelengths log-uniform in [lam_lo, lam_hi] Angstrom -> frequencies,
    sorted non-increasing (stable)."""
    lam = np.exp(rng.uniform(math.log(lam_lo_aa), math.log(lam_hi_aa), n_lines)) * ANGSTROM
    nu = C_LIGHT / lam
    order = np.argsort(-nu, kind="stable")
    return _contig(nu[order], np.float64)


def tau_log_uniform(rng, n_shells, n_lines, lo_dex=-3.0, hi_dex=3.0):
    return _contig(10.0 ** rng.uniform(lo_dex, hi_dex, size=(n_shells, n_lines)), np.float64)


def tau_log_normal(rng, n_shells, n_lines, mu=math.log(0.1), sigma=3.0, clip=1.0e6):
    t = np.exp(rng.normal(mu, sigma, size=(n_shells, n_lines)))
    return _contig(np.clip(t, 0.0, clip), np.float64)


def config1(seed: int = 0, n_packets: int = 10_000) -> Workload:
    """Scatter mode, 20 shells 11000-20000 km/s at 13 d, 2000 lines
    log-uniform in 3000-10000 A, tau log-uniform in [1e-3, 1e3], T_i = 1e4 K."""
    rng = np.random.default_rng(seed)
    v, t, n_e = shells(20, 11000.0, 20000.0, 13.0)
    nu = log_uniform_lines(rng, 2000, 3000.0, 10000.0)
    tau = tau_log_uniform(rng, 20, 2000)
    m = Model(v_bounds=v, t_exp=t, n_e=n_e, line_nu=nu, tau_sobolev=tau, seed=seed)
    return Workload("scatter-20shell-2000line", m, T_inner=10000.0, n_packets=n_packets,
                    n_iterations=1)


def config2_model(rng, n_shells=20, n_lines=300_000, seed=0, v_lo=10000.0, v_hi=25000.0):
    v, t, n_e = shells(n_shells, v_lo, v_hi, 13.0)
    nu = log_uniform_lines(rng, n_lines, 500.0, 20000.0)
    tau = tau_log_normal(rng, n_shells, n_lines)
    return Model(v_bounds=v, t_exp=t, n_e=n_e, line_nu=nu, tau_sobolev=tau, seed=seed)


def config2(seed: int = 0, n_lines: int = 300_000, n_packets: int = 1_000_000,
            n_iterations: int = 10) -> Workload:
    """Paper-scale scatter model: 20 shells 10000-25000 km/s, 3e5 lines
    log-uniform in 500-20000 A, tau log-normal (ln 0.1, 3) clipped to 1e6,
    T_i = 9000 K, 1e6 packets, 10 iterations with the T_i update."""
    rng = np.random.default_rng(seed)
    m = config2_model(rng, 20, n_lines, seed)
    return Workload("scatter-20shell-300kline", m, T_inner=9000.0, n_packets=n_packets,
                    n_iterations=n_iterations)


def synthetic_atom(rng, n_ions=30, n_levels_per_ion=40, n_lines=20_000):
    """Synthetic downbranch atom: per ion, level energies (in frequency units)
    0 and sorted U(0, c/500A); n_lines distinct (ion, lower<upper) pairs drawn
    without replacement; A_ul log-uniform in 1e5-1e9 s^-1.  Emission
    probabilities of an upper level are proportional to A_ul * nu_ul over its
    downward lines.  Returns lines sorted by non-increasing frequency."""
    nl = n_levels_per_ion
    e = np.zeros((n_ions, nl))
    for i in range(n_ions):
        e[i, 1:] = np.sort(rng.uniform(0.0, C_LIGHT / (500.0 * ANGSTROM), nl - 1))
    pairs = [(i, lo, up) for i in range(n_ions) for up in range(nl) for lo in range(up)]
    pick = rng.choice(len(pairs), size=n_lines, replace=False)
    ion = np.array([pairs[p][0] for p in pick])
    lower = np.array([pairs[p][1] for p in pick])
    upper = np.array([pairs[p][2] for p in pick])
    nu = e[ion, upper] - e[ion, lower]
    a_ul = 10.0 ** rng.uniform(5.0, 9.0, n_lines)
    order = np.argsort(-nu, kind="stable")
    nu, ion, upper, a_ul = nu[order], ion[order], upper[order], a_ul[order]
    up_global = (ion * nl + upper).astype(np.int32)
    n_levels = n_ions * nl
    # CSR rows over upper levels, entries in line-index order
    counts = np.bincount(up_global, minlength=n_levels)
    level_ptr = np.zeros(n_levels + 1, dtype=np.int64)
    level_ptr[1:] = np.cumsum(counts)
    em_line = np.argsort(up_global, kind="stable").astype(np.int32)
    weight = a_ul[em_line] * nu[em_line]
    em_cum = np.zeros(n_lines, dtype=np.float64)
    for lev in range(n_levels):
        a, b = level_ptr[lev], level_ptr[lev + 1]
        if b > a:
            c = np.cumsum(weight[a:b])
            em_cum[a:b] = c / c[-1]
            em_cum[b - 1] = 1.0
    return dict(line_nu=_contig(nu, np.float64), line_upper=_contig(up_global, np.int32),
                n_levels=int(n_levels), level_ptr=_contig(level_ptr, np.int64),
                em_line=_contig(em_line, np.int32), em_cum=_contig(em_cum, np.float64))


def _levels_and_lines(rng, n_ions, n_levels_per_ion, n_lines):
    """Levels and lines of a synthetic atom: per ion, level energies (in
    frequency units) 0 and sorted U(0, c/500A); n_lines distinct (ion,
    lower < upper) pairs drawn without replacement.  Returns per line (sorted
    by non-increasing frequency) its frequency and global lower and upper
    level, and the number of levels."""
    nl = n_levels_per_ion
    e = np.zeros((n_ions, nl))
    for i in range(n_ions):
        e[i, 1:] = np.sort(rng.uniform(0.0, C_LIGHT / (500.0 * ANGSTROM), nl - 1))
    pairs = [(i, lo, up) for i in range(n_ions) for up in range(nl) for lo in range(up)]
    pick = rng.choice(len(pairs), size=n_lines, replace=False)
    ion = np.array([pairs[p][0] for p in pick])
    lower = np.array([pairs[p][1] for p in pick])
    upper = np.array([pairs[p][2] for p in pick])
    nu = e[ion, upper] - e[ion, lower]
    order = np.argsort(-nu, kind="stable")
    nu, ion, lower, upper = nu[order], ion[order], lower[order], upper[order]
    return nu, (ion * nl + lower).astype(np.int32), (ion * nl + upper).astype(np.int32), n_ions * nl


def macroatom_model(seed: int = 0, n_shells: int = 30, n_ions: int = 30,
                    n_levels_per_ion: int = 40, n_lines: int = 20_000):
    """Macroatom mode with caller-given tables, for the transport: a
    synthetic atom (as the downbranch workload's) whose level rows hold
    deactivations in the level's downward lines, jumps to their lower levels
    and jumps to the upper levels of its upward lines, with probabilities
    from weights U(0.05, 1) drawn per shell and entry (random tables: the
    method's own tables come from the plasma state, macroatom_plasma_model).
    tau log-normal as the paper-scale model."""
    rng = np.random.default_rng(seed)
    v, t, n_e = shells(n_shells, 10000.0, 25000.0, 13.0)
    nu, lower, upper, n_levels = _levels_and_lines(rng, n_ions, n_levels_per_ion, n_lines)
    tau = tau_log_normal(rng, n_shells, n_lines)
    rows = [[] for _ in range(n_levels)]
    for k in range(n_lines):
        rows[upper[k]].append(k)
    for k in range(n_lines):
        rows[upper[k]].append(-(int(lower[k]) + 1))
    for k in range(n_lines):
        rows[lower[k]].append(-(int(upper[k]) + 1))
    level_ptr = np.zeros(n_levels + 1, dtype=np.int64)
    level_ptr[1:] = np.cumsum([len(r) for r in rows])
    em_line = np.array([x for r in rows for x in r], dtype=np.int32)
    w = rng.uniform(0.05, 1.0, (n_shells, em_line.shape[0]))
    em_cum = np.zeros_like(w)
    for lev in range(n_levels):
        a, b = level_ptr[lev], level_ptr[lev + 1]
        if b > a:
            c = np.cumsum(w[:, a:b], axis=1)
            em_cum[:, a:b] = c / c[:, -1:]
            em_cum[:, b - 1] = 1.0
    return Model(v_bounds=v, t_exp=t, n_e=n_e, line_nu=_contig(nu, np.float64),
                 tau_sobolev=tau, line_mode=MACROATOM, line_upper=_contig(upper, np.int32),
                 n_levels=int(n_levels), level_ptr=_contig(level_ptr, np.int64),
                 em_line=_contig(em_line, np.int32), em_cum=_contig(em_cum, np.float64),
                 seed=seed)


def config_macroatom(seed: int = 0, n_packets: int = 500_000) -> tuple:
    """Macroatom mode with tables from the plasma state, at the size of the
    downbranch workload: 30 shells over 10000-25000 km/s at 13 d, 2e4 lines
    of 8 elements x 5 stages x 40 levels, T_i = 9000 K.  Returns the
    workload and its plasma description."""
    model, spec = macroatom_plasma_model(seed, n_shells=30, n_levels_per_ion=40,
                                         n_lines=20_000)
    w = Workload("macroatom-30shell-20kline", model, T_inner=9000.0, n_packets=n_packets,
                 n_iterations=1)
    return w, spec


def config3(seed: int = 0, n_packets: int = 500_000, n_lines: int = 20_000,
            n_shells: int = 30) -> Workload:
    """Downbranch mode: 30 ions x 40 levels, 2e4 lines, 30 shells over
    10000-25000 km/s at 13 d, tau log-normal as config 2, T_i = 9000 K."""
    rng = np.random.default_rng(seed)
    v, t, n_e = shells(n_shells, 10000.0, 25000.0, 13.0)
    atom = synthetic_atom(rng, 30, 40, n_lines)
    tau = tau_log_normal(rng, n_shells, n_lines)
    m = Model(v_bounds=v, t_exp=t, n_e=n_e, tau_sobolev=tau, line_mode=DOWNBRANCH,
              seed=seed, **atom)
    return Workload("downbranch-30shell-20kline", m, T_inner=9000.0, n_packets=n_packets,
                    n_iterations=1)


def config4_model(i: int) -> Workload:
    """Model i of the batched mix: S ~ U{10..100}, L log-uniform in 1e4-3e5,
    N log-uniform in 1e5-1e6, otherwise as config 2; Philox seed i."""
    rng = np.random.default_rng(i)
    S = int(rng.integers(10, 101))
    L = int(round(math.exp(rng.uniform(math.log(1e4), math.log(3e5)))))
    N = int(round(math.exp(rng.uniform(math.log(1e5), math.log(1e6)))))
    m = config2_model(rng, S, L, seed=i)
    return Workload(f"batch-model-{i}", m, T_inner=9000.0, n_packets=N, n_iterations=1)


def config5_requests(duration_s: float = 60.0, rate_hz: float = 20.0, seed: int = 5):
    """Poisson arrivals; request j is a config-4 style model from seed 1000+j
    with U{1..10} iterations.  Returns (arrival_time, seed, n_iterations)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    j = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append((t, 1000 + j, int(rng.integers(1, 11))))
        j += 1
    return out


def small_model(seed: int = 0, n_shells: int = 5, n_lines: int = 300, v_lo=11000.0,
                v_hi=20000.0, lam=(3000.0, 10000.0), tau="loguniform", rho_inner=1e-13,
                t_exp_days=13.0) -> Model:
    """Small scatter-mode model for tests: same recipe, any size."""
    rng = np.random.default_rng(seed)
    v, t, n_e = shells(n_shells, v_lo, v_hi, t_exp_days, rho_inner)
    nu = log_uniform_lines(rng, n_lines, lam[0], lam[1])
    if tau == "loguniform":
        ts = tau_log_uniform(rng, n_shells, n_lines)
    else:
        ts = tau_log_normal(rng, n_shells, n_lines)
    return Model(v_bounds=v, t_exp=t, n_e=n_e, line_nu=nu, tau_sobolev=ts, seed=seed)


def small_downbranch_model(seed: int = 0, n_shells: int = 6, n_ions: int = 4,
                           n_levels_per_ion: int = 12, n_lines: int = 200) -> Model:
    rng = np.random.default_rng(seed)
    v, t, n_e = shells(n_shells, 10000.0, 25000.0, 13.0)
    atom = synthetic_atom(rng, n_ions, n_levels_per_ion, n_lines)
    tau = tau_log_normal(rng, n_shells, n_lines)
    return Model(v_bounds=v, t_exp=t, n_e=n_e, tau_sobolev=tau, line_mode=DOWNBRANCH,
                 seed=seed, **atom)


# ---------------------------------------------------------------------------
# plasma inputs: a synthetic atom (elements, ion stages, levels, lines with
# oscillator strengths) and element number densities per shell
# ---------------------------------------------------------------------------
EV = 1.602176634e-12  # erg
M_U = 1.66053906660e-24  # g

ION_LTE, ION_NEBULAR = 0, 1
EXC_LTE, EXC_DILUTE_LTE = 0, 1

# (atomic number, mass number, first ionization energy [eV]) of the
# synthetic elements; the energies of the higher stages follow _CHI_SCALE
PLASMA_ELEMENTS = ((8, 16.0, 13.62), (12, 24.3, 7.65), (14, 28.1, 8.15), (16, 32.1, 10.36),
                   (20, 40.1, 6.11), (26, 55.8, 7.90), (27, 58.9, 7.88), (28, 58.7, 7.64))
_CHI_SCALE = (1.0, 2.0, 3.9, 5.8, 8.0, 10.5, 13.0, 16.0)


@dataclasses.dataclass
class PlasmaAtom:
    """Atomic data of the plasma update, in the layout both implementations
    consume.  Ions of an element are consecutive, stage j (charge j) at
    element_ion_ptr[e] + j; levels of an ion are consecutive, its ground
    state (energy 0, metastable) first."""

    element_ion_ptr: np.ndarray  # [E+1] int32
    ion_chi: np.ndarray  # [n_ions] ionization energy from this stage to the next [erg]
    ion_zeta: np.ndarray  # [n_ions] fraction of recombinations into this stage's ground state
    ion_level_ptr: np.ndarray  # [n_ions+1] int32
    level_energy: np.ndarray  # [n_levels] excitation energy above the ion's ground state [erg]
    level_g: np.ndarray  # [n_levels] statistical weight
    level_metastable: np.ndarray  # [n_levels] uint8
    line_lower: np.ndarray  # [L] int32, global level index
    line_upper: np.ndarray  # [L] int32
    line_f: np.ndarray  # [L] absorption oscillator strength
    line_upsilon: Optional[np.ndarray] = None  # [L] collision strengths (NLTE ions' lines)

    @property
    def n_elements(self) -> int:
        return int(self.element_ion_ptr.shape[0] - 1)

    @property
    def n_ions(self) -> int:
        return int(self.ion_chi.shape[0])

    @property
    def n_levels(self) -> int:
        return int(self.level_energy.shape[0])

    def level_ion(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_ions, dtype=np.int32), np.diff(self.ion_level_ptr))

    def nbytes(self) -> int:
        return sum(getattr(self, f.name).nbytes for f in dataclasses.fields(self)
                   if getattr(self, f.name) is not None)


@dataclasses.dataclass
class PlasmaSpec:
    atom: PlasmaAtom
    number_density: np.ndarray  # [S, E] element number densities [cm^-3]
    nlte_ions: tuple = ()  # ions whose populations come from statistical equilibrium


def synthetic_plasma_atom(rng, n_elements: int = 8, n_stages: int = 5,
                          n_levels_per_ion: int = 60, n_lines: int = 20_000,
                          lam=(300.0, 25000.0), nlte_ions=(), n_levels_nlte: int = 40):
    """Synthetic atom: the first n_elements of PLASMA_ELEMENTS with stages
    0 .. n_stages-1 each; ionization energies chi_0 * _CHI_SCALE[j]; per ion
    the ground state plus n_levels_per_ion-1 levels with energies U(0,
    0.95 chi) (sorted), statistical weights uniform in 1..9 (ground 1..5),
    metastable with probability 0.25 below 0.3 chi and 0.02 above; zeta
    U(0.1, 0.9).  Lines: n_lines distinct (ion, lower < upper) pairs whose
    wavelength h c / (e_u - e_l) lies in [lam] Angstrom, drawn without
    replacement, f log-uniform in [1e-4, 1], collision strengths
    log-uniform in [0.1, 10].  Ions listed in nlte_ions (global ion
    indices) get n_levels_nlte levels with excited energies U(0.6 eV,
    0.95 chi), and a line from the ground state to every excited level is
    always among the lines, so that statistical equilibrium connects all of
    their levels.  Returns the atom with lines sorted by non-increasing
    frequency, and the line frequencies."""
    elems = PLASMA_ELEMENTS[:n_elements]
    n_ions = n_elements * n_stages
    nlte = set(int(i) for i in nlte_ions)
    nls = np.array([n_levels_nlte if i in nlte else n_levels_per_ion for i in range(n_ions)])
    lptr = np.zeros(n_ions + 1, dtype=np.int64)
    lptr[1:] = np.cumsum(nls)
    chi = np.array([z[2] * _CHI_SCALE[j] * EV for z in elems for j in range(n_stages)])
    zeta = rng.uniform(0.1, 0.9, n_ions)
    energy = np.zeros(lptr[-1])
    g = np.zeros(lptr[-1])
    meta = np.zeros(lptr[-1], dtype=np.uint8)
    for i in range(n_ions):
        a, nl = lptr[i], nls[i]
        lo_e = 0.6 * EV if i in nlte else 0.0
        energy[a + 1:a + nl] = np.sort(rng.uniform(lo_e, 0.95 * chi[i], nl - 1))
        g[a] = rng.integers(1, 6)
        g[a + 1:a + nl] = rng.integers(1, 10, nl - 1)
        meta[a] = 1
        low = energy[a + 1:a + nl] < 0.3 * chi[i]
        u = rng.uniform(0.0, 1.0, nl - 1)
        meta[a + 1:a + nl] = np.where(low, u < 0.25, u < 0.02)
    ions, lowers, uppers = [], [], []
    for i in range(n_ions):
        lo_i, up_i = np.triu_indices(nls[i], k=1)
        ions.append(np.full(lo_i.size, i))
        lowers.append(lptr[i] + lo_i)
        uppers.append(lptr[i] + up_i)
    ion, lower, upper = np.concatenate(ions), np.concatenate(lowers), np.concatenate(uppers)
    de = energy[upper] - energy[lower]
    with np.errstate(divide="ignore"):
        lam_aa = np.where(de > 0.0, H * C_LIGHT / np.where(de > 0.0, de, 1.0) / ANGSTROM, np.inf)
    window = (lam_aa >= lam[0]) & (lam_aa <= lam[1])
    star = np.isin(ion, list(nlte)) & (lower == lptr[ion])
    ok = np.flatnonzero(window & ~star)
    must = np.flatnonzero(star)
    if ok.size < n_lines - must.size:
        raise ValueError(f"only {ok.size} level pairs in the wavelength window")
    pick = np.sort(np.concatenate([rng.choice(ok, size=n_lines - must.size, replace=False),
                                   must]))
    ion, lower, upper = ion[pick], lower[pick], upper[pick]
    f = 10.0 ** rng.uniform(-4.0, 0.0, n_lines)
    nu = (energy[upper] - energy[lower]) / H
    order = np.argsort(-nu, kind="stable")
    ion, lower, upper, f, nu = ion[order], lower[order], upper[order], f[order], nu[order]
    upsilon = 10.0 ** rng.uniform(-1.0, 1.0, n_lines)
    atom = PlasmaAtom(
        element_ion_ptr=_contig(np.arange(n_elements + 1) * n_stages, np.int32),
        ion_chi=_contig(chi, np.float64), ion_zeta=_contig(zeta, np.float64),
        ion_level_ptr=_contig(lptr, np.int32),
        level_energy=_contig(energy, np.float64),
        level_g=_contig(g, np.float64),
        level_metastable=_contig(meta, np.uint8),
        line_lower=_contig(lower, np.int32),
        line_upper=_contig(upper, np.int32),
        line_f=_contig(f, np.float64),
        line_upsilon=_contig(upsilon, np.float64))
    return atom, _contig(nu, np.float64)


def element_densities(rho, n_elements: int):
    """Number densities [S, E] of equal mass fractions of the first
    n_elements of PLASMA_ELEMENTS at mass densities rho [S]."""
    mass = np.array([z[1] for z in PLASMA_ELEMENTS[:n_elements]])
    return _contig(np.asarray(rho)[:, None] / n_elements / (mass[None, :] * M_U), np.float64)


def plasma_model(seed: int = 0, n_shells: int = 20, n_elements: int = 8, n_stages: int = 5,
                 n_levels_per_ion: int = 60, n_lines: int = 20_000,
                 v_lo: float = 10000.0, v_hi: float = 25000.0, t_exp_days: float = 13.0,
                 rho_inner: float = 3.0e-14, nlte_ions=(), n_levels_nlte: int = 40,
                 line_mode: int = SCATTER):
    """Model whose Sobolev depths and electron densities come from the
    plasma update: shells as config 2 (rho ~ v^-7), equal mass fractions of
    the synthetic elements.  tau_sobolev and n_e start at zero and are
    filled by the plasma state of the initial radiation field.  Scatter mode,
    or with line_mode = MACROATOM the macro atom of the plasma's atom with
    no tables (the plasma update derives them)."""
    rng = np.random.default_rng(seed)
    v = np.linspace(v_lo * KM, v_hi * KM, n_shells + 1)
    v_mid = 0.5 * (v[:-1] + v[1:])
    rho = rho_inner * (v_mid / v_mid[0]) ** -7.0
    atom, nu = synthetic_plasma_atom(rng, n_elements, n_stages, n_levels_per_ion, n_lines,
                                     nlte_ions=nlte_ions, n_levels_nlte=n_levels_nlte)
    macro = line_mode == MACROATOM
    model = Model(v_bounds=_contig(v, np.float64), t_exp=t_exp_days * DAY,
                  n_e=np.zeros(n_shells), line_nu=nu,
                  tau_sobolev=np.zeros((n_shells, n_lines)), seed=seed,
                  line_mode=MACROATOM if macro else SCATTER,
                  line_upper=atom.line_upper if macro else None,
                  n_levels=atom.n_levels if macro else 0)
    return model, PlasmaSpec(atom=atom, number_density=element_densities(rho, n_elements),
                             nlte_ions=tuple(int(i) for i in nlte_ions))


def macroatom_plasma_model(seed: int = 0, n_shells: int = 20, n_elements: int = 8,
                           n_stages: int = 5, n_levels_per_ion: int = 60,
                           n_lines: int = 20_000, **kw):
    """plasma_model in macroatom mode: tables derived from the plasma state."""
    return plasma_model(seed, n_shells=n_shells, n_elements=n_elements, n_stages=n_stages,
                        n_levels_per_ion=n_levels_per_ion, n_lines=n_lines,
                        line_mode=MACROATOM, **kw)


def config_plasma(seed: int = 0, n_packets: int = 1_000_000, n_lines: int = 300_000,
                  n_levels_per_ion: int = 150) -> tuple:
    """Plasma feedback at the size of the paper-scale model: 20 shells, 3e5
    lines of 8 elements x 5 stages x 150 levels, 1e6 packets, nebular
    ionization with dilute-LTE excitation (section 5.3's choice for all but
    the NLTE ion)."""
    model, spec = plasma_model(seed, n_shells=20, n_lines=n_lines,
                               n_levels_per_ion=n_levels_per_ion)
    w = Workload("plasma-20shell-300kline", model, T_inner=9000.0, n_packets=n_packets,
                 n_iterations=10)
    return w, spec


def config_plasma_nlte(seed: int = 0, n_packets: int = 1_000_000, n_lines: int = 300_000,
                       n_levels_per_ion: int = 150, n_levels_nlte: int = 40) -> tuple:
    """The plasma benchmark with the stage-1 ions of the Mg, Si, S and Ca
    analogues (Mg II, Si II, S II, Ca II: the ions of the paper's NLTE study)
    in NLTE excitation with n_levels_nlte levels each."""
    nlte = (1 * 5 + 1, 2 * 5 + 1, 3 * 5 + 1, 4 * 5 + 1)
    model, spec = plasma_model(seed, n_shells=20, n_lines=n_lines,
                               n_levels_per_ion=n_levels_per_ion, nlte_ions=nlte,
                               n_levels_nlte=n_levels_nlte)
    w = Workload("plasma-nlte-20shell-300kline", model, T_inner=9000.0, n_packets=n_packets,
                 n_iterations=10)
    return w, spec
