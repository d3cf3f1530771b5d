"""Pins of the oracle's virtual packets (section 2.9) against brute force and
against what the paper states about them.

* Each v-packet's optical depth is recomputed here by brute force along its
  straight path (Thomson depth from the chord pieces found by bisection,
  line resonances found by root-finding the comoving frequency along the
  ray), from the emission states in the oracle's event trace; the oracle's
  v-packet spectrum must equal the sum of the recomputed contributions.
* The paper states that the v-packet spectrum agrees with the spectrum of
  the escaping r-packets: checked statistically over independent batches.
* v-packets use their own random stream: the r-packet histories do not
  change when they are switched on.
None of these tests needs a GPU.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1401_5469_amd import workloads as W

C_LIGHT = 2.99792458e10
SIGMA_T = 6.6524587321e-25
TAU_MAX = 30.0


def _model(v_kms, n_e, line_nu=None, tau=None, t_days=13.0, seed=3, **kw):
    v = np.asarray(v_kms, dtype=np.float64) * 1e5
    S = v.shape[0] - 1
    if line_nu is None:
        line_nu = np.zeros(0)
        tau = np.zeros((S, 0))
    return W.Model(v_bounds=v, t_exp=t_days * 86400.0, n_e=np.asarray(n_e, dtype=np.float64),
                   line_nu=np.asarray(line_nu, dtype=np.float64),
                   tau_sobolev=np.ascontiguousarray(tau, dtype=np.float64), seed=seed, **kw)


def _vdraw(seed, pid, iteration, dv):
    """Draw dv of the v-packet stream of packet pid (the stream contract)."""
    key = [(seed & 0xFFFFFFFF) ^ 0x56504B54, (seed >> 32) & 0xFFFFFFFF]
    ctr = [dv // 2, pid & 0xFFFFFFFF, (pid >> 32) & 0xFFFFFFFF, iteration]
    x = O.philox4x32_10(ctr, key)
    j = dv % 2
    return O.uniform((int(x[2 * j + 1]) << 32) | int(x[2 * j]))


def _bin(m, nu):
    dnu = (m.nu_max - m.nu_min) / m.n_bins
    if nu < m.nu_min:
        return m.n_bins
    f = math.floor((nu - m.nu_min) / dnu)
    return m.n_bins + 1 if f >= m.n_bins else int(f)


def _exit_distance(r, mu, R):
    """Distance along the ray to radius R (outward crossing), by bisection."""
    lo, hi = 0.0, 4.0 * R
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if math.sqrt(r * r + mid * mid + 2 * r * mid * mu) < R:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _pieces(m, r, mu, shell):
    """Shell pieces of the ray from (r, mu) in `shell` to the outer boundary:
    (shell, start distance, end distance), boundaries found by bisection on
    the radius along the ray."""
    radii = m.v_bounds * m.t_exp
    R = radii[-1]
    d_exit = _exit_distance(r, mu, R)
    # radius along the ray is convex in s; sample finely, then refine each
    # crossing of a shell radius by bisection
    s = np.linspace(0.0, d_exit, 4001)
    rad = np.sqrt(r * r + s * s + 2 * r * s * mu)
    idx = np.searchsorted(radii, rad, side="right") - 1
    idx[0] = shell
    idx = np.clip(idx, 0, m.n_shells - 1)
    cuts = [0.0]
    for i in range(1, len(s)):
        if idx[i] != idx[i - 1]:
            target = radii[max(idx[i], idx[i - 1])]
            lo, hi = s[i - 1], s[i]
            f_lo = math.sqrt(r * r + lo * lo + 2 * r * lo * mu) - target
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                f = math.sqrt(r * r + mid * mid + 2 * r * mid * mu) - target
                if (f < 0) == (f_lo < 0):
                    lo, f_lo = mid, f
                else:
                    hi = mid
            cuts.append(0.5 * (lo + hi))
    cuts.append(d_exit)
    shells = [shell]
    for i in range(1, len(s)):
        if idx[i] != idx[i - 1]:
            shells.append(int(idx[i]))
    return [(shells[j], cuts[j], cuts[j + 1]) for j in range(len(shells))]


def _brute_tau(m, r, mu, shell, nu_lab, first_line):
    """Optical depth of a v-packet's path: Thomson depth of every piece with
    the Doppler factor at the piece's start, plus tau_S of every line whose
    resonance (comoving frequency along the ray equal to the line's) lies on
    the path, in the shell where it lies."""
    ct = C_LIGHT * m.t_exp
    tau = 0.0
    pieces = _pieces(m, r, mu, shell)
    for sh, a, b in pieces:
        ra = math.sqrt(r * r + a * a + 2 * r * a * mu)
        mua = (r * mu + a) / ra
        D = 1.0 - mua * ra / ct
        tau += SIGMA_T * m.n_e[sh] * D * (b - a)
    d_exit = pieces[-1][2]

    def nu_cmf(s):
        rs = math.sqrt(r * r + s * s + 2 * r * s * mu)
        mus = (r * mu + s) / rs
        return nu_lab * (1.0 - mus * rs / ct)

    for k in range(first_line, m.n_lines):
        nk = m.line_nu[k]
        if nu_cmf(0.0) < nk:
            continue
        if nu_cmf(d_exit) >= nk:
            continue  # resonance beyond the outer boundary
        lo, hi = 0.0, d_exit
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if nu_cmf(mid) >= nk:
                lo = mid
            else:
                hi = mid
        s_res = 0.5 * (lo + hi)
        sh = next(p[0] for p in pieces if p[1] <= s_res <= p[2])
        tau += m.tau_sobolev[sh, k]
    return tau


def _emissions(m, raw, N, iteration):
    """Emission states (packet, launch index, injection?, r, shell, next line,
    nu_cmf, E_cmf) read from the event trace and the packet records."""
    ct = C_LIGHT * m.t_exp
    r_in = m.v_bounds[0] * m.t_exp
    recs = {int(p["id"]): p for p in raw["packets"]}
    out = []
    launches = {}
    for ev in raw["trace"]:
        pid = int(ev["packet_id"])
        if ev["kind"] == 0:  # injection
            p = recs[pid]
            nu0 = float(p["nu_cmf0"])
            first = int(np.sum(m.line_nu >= nu0))  # first line with nu_k < nu_cmf
            out.append((pid, 0, True, r_in, 0, first, nu0, 1.0 / N))
            launches[pid] = 0
        elif ev["kind"] in (3, 4):  # Thomson, line
            launches[pid] += 1
            r, mu = float(ev["r"]), float(ev["mu_out"])
            D = 1.0 - mu * r / ct
            nu_cmf = float(ev["nu_out"]) * D
            e_cmf = float(ev["e_out"]) * D
            if ev["kind"] == 4:
                first = int(ev["emit_line"]) + 1
            else:
                first = int(np.sum(m.line_nu >= nu_cmf))
            out.append((pid, launches[pid], False, r, int(ev["shell"]), first, nu_cmf, e_cmf))
    return out


def _brute_vspec(m, raw, N, iteration, nv):
    ct = C_LIGHT * m.t_exp
    r_in = m.v_bounds[0] * m.t_exp
    spec = np.zeros(m.n_bins + 2)
    launched = counted = 0
    for pid, e, inj, r, sh, first, nu_cmf, e_cmf in _emissions(m, raw, N, iteration):
        mu_min = -math.sqrt(max(0.0, 1.0 - (r_in / r) ** 2))
        for j in range(nv):
            u = _vdraw(m.seed, pid, iteration, e * nv + j)
            mu_v = mu_min + (1.0 - mu_min) * u
            w = 2.0 * mu_v / nv if inj else (1.0 - mu_min) / (2.0 * nv)
            D = 1.0 - mu_v * r / ct
            nu_lab = nu_cmf / D
            tau = _brute_tau(m, r, mu_v, sh, nu_lab, first)
            launched += 1
            if tau <= TAU_MAX:
                counted += 1
                spec[_bin(m, nu_lab)] += e_cmf * w / D * math.exp(-tau)
    return spec, launched, counted


def test_virtual_thomson_depths_match_brute_force():
    # two electron-scattering shells, no lines: tau_v is the Thomson depth
    m = _model([11000, 14000, 20000], [2.5e9, 6e8], seed=11)
    N, nv = 60, 3
    raw = O.run(m, 10000.0, N, packet_ids=np.arange(N, dtype=np.uint64), n_virtual=nv,
                trace_cap=20000, want_jblue=False)
    assert raw["trace_len"] < 20000
    spec, launched, counted = _brute_vspec(m, raw, N, 0, nv)
    assert raw["counters"]["escatters"] > 20
    assert raw["vcounts"]["launched"] == launched == nv * (N + raw["counters"]["escatters"])
    assert raw["vcounts"]["counted"] == counted
    np.testing.assert_allclose(raw["vspec_raw"], spec, rtol=1e-9, atol=0)


def test_virtual_line_depths_match_brute_force():
    # three shells, no electrons, 40 lines with shell-dependent depths up to
    # 40 (so that some v-packets pass the cut-off), scatter and emission
    rng = np.random.default_rng(5)
    lam = np.sort(rng.uniform(4000.0, 6000.0, 40))
    nu = C_LIGHT / (lam * 1e-8)  # decreasing frequency for increasing wavelength
    tau = rng.uniform(0.0, 1.5, (3, 40))
    tau[:, ::13] = 40.0
    m = _model([11000, 13000, 16000, 20000], [0.0, 0.0, 0.0], line_nu=nu, tau=tau, seed=12,
               nu_min=C_LIGHT / 7000e-8, nu_max=C_LIGHT / 3500e-8, n_bins=50)
    N, nv = 60, 2
    # an inner boundary whose Planck peak lies in the line band
    raw = O.run(m, 9000.0, N, packet_ids=np.arange(N, dtype=np.uint64), n_virtual=nv,
                trace_cap=20000, want_jblue=False)
    assert raw["trace_len"] < 20000
    assert raw["counters"]["line_events"] > 20
    spec, launched, counted = _brute_vspec(m, raw, N, 0, nv)
    assert raw["vcounts"]["launched"] == launched
    assert 0 < raw["vcounts"]["counted"] == counted < launched  # some pass tau = 40 lines
    np.testing.assert_allclose(raw["vspec_raw"], spec, rtol=1e-9, atol=1e-300)


def test_virtual_packets_leave_r_histories_unchanged():
    m = W.small_model(seed=21, n_shells=6, n_lines=500)
    ids = np.arange(300, dtype=np.uint64)
    a = O.run(m, 10000.0, 300, packet_ids=ids)
    b = O.run(m, 10000.0, 300, packet_ids=ids, n_virtual=3)
    assert np.array_equal(a["packets"], b["packets"])
    for k in ("J_raw", "nubar_raw", "jblue_raw", "spec_raw", "L_raw"):
        assert np.array_equal(a[k], b[k]), k
    assert b["vcounts"]["launched"] == 3 * (300 + b["counters"]["line_events"] +
                                            b["counters"]["escatters"])


def _batches(m, T, N, n_batches, nv):
    """Per-batch escaping r-packet luminosity and v-packet luminosity in
    coarse bins (independent batches of packet ids)."""
    edges = np.linspace(0, m.n_bins, 11).astype(int)
    r_tot, v_tot, r_bins, v_bins = [], [], [], []
    for b in range(n_batches):
        ids = np.arange(b * N, (b + 1) * N, dtype=np.uint64)
        raw = O.run(m, T, n_batches * N, packet_ids=ids, n_virtual=nv, want_jblue=False)
        r_tot.append(raw["L_raw"][0])
        v_tot.append(raw["vspec_raw"].sum())
        r_bins.append(np.add.reduceat(raw["spec_raw"][: m.n_bins], edges[:-1]))
        v_bins.append(np.add.reduceat(raw["vspec_raw"][: m.n_bins], edges[:-1]))
    return (np.array(r_tot), np.array(v_tot), np.array(r_bins), np.array(v_bins))


def test_virtual_spectrum_estimates_the_escaping_spectrum():
    # lines and electrons; the paper states that the v-packet spectrum agrees
    # with direct binning of escaping r-packets
    m = W.small_model(seed=31, n_shells=8, n_lines=400, tau="lognormal")
    r_tot, v_tot, r_bins, v_bins = _batches(m, 11000.0, 400, 24, 3)
    nb = len(r_tot)
    diff = v_tot.mean() - r_tot.mean()
    se = math.sqrt(v_tot.var(ddof=1) / nb + r_tot.var(ddof=1) / nb)
    assert abs(diff) < 4.0 * se, (diff, se)
    # coarse spectral bins agree within their batch-to-batch errors
    for j in range(r_bins.shape[1]):
        d = v_bins[:, j].mean() - r_bins[:, j].mean()
        s = math.sqrt(v_bins[:, j].var(ddof=1) / nb + r_bins[:, j].var(ddof=1) / nb)
        assert abs(d) <= 4.5 * s + 1e-15, (j, d, s)


def test_virtual_thin_model_estimate_is_the_emitted_luminosity():
    # nothing to interact with: every r-packet escapes, every v-packet counts
    # with tau = 0, and both estimate the same luminosity (section 2.9)
    m = _model([11000, 20000], [0.0], seed=41)
    r_tot, v_tot, _, _ = _batches(m, 10000.0, 500, 20, 4)
    nb = len(r_tot)
    se = math.sqrt(v_tot.var(ddof=1) / nb + r_tot.var(ddof=1) / nb)
    assert abs(v_tot.mean() - r_tot.mean()) < 4.0 * se
    raw = O.run(m, 10000.0, 100, n_virtual=4)
    assert raw["vcounts"]["launched"] == raw["vcounts"]["counted"] == 400
