"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them."""
import numpy as np

from oracle import oracle as O
from paper_1401_5469_amd import smc

REL = 1e-9  # per-packet and estimator tolerance (relative)
DIVERGE_FRACTION = 1e-4


def gpu_run(ctx, model, n_packets, T_inner, iteration=0, packet_ids=None, flags=None,
            L_requested=0.0, damping=1.0, max_segments=10**7, n_packets_max=None, jblue=True,
            tune=None):
    if flags is None:
        flags = (smc.F_JBLUE if jblue else 0) | smc.F_PACKETS
    n_work = len(packet_ids) if packet_ids is not None else n_packets
    m = smc.Model(ctx, model, n_packets_max or max(n_work, 1), flags=flags)
    if tune:
        m.set_tune(**tune)
    m.run_iteration(n_packets, T_inner, iteration=iteration, flags=flags,
                    L_requested=L_requested, damping=damping, max_segments=max_segments,
                    packet_ids=packet_ids)
    out = dict(est=m.read_estimators(jblue=bool(flags & smc.F_JBLUE)), spec=m.read_spectrum(),
               counters=m.read_counters())
    if flags & smc.F_PACKETS:
        out["packets"] = m.read_packets(n_work)
    out["model"] = m
    return out


def oracle_run(model, n_packets, T_inner, iteration=0, packet_ids=None, L_requested=0.0,
               damping=1.0, max_segments=10**7, jblue=True, T_R_prev=None, W_prev=None):
    raw = O.run(model, T_inner, n_packets, iteration=iteration, packet_ids=packet_ids,
                max_segments=max_segments, want_jblue=jblue)
    fin = O.finalise(model, raw, T_inner, L_requested, T_R_prev, W_prev, damping=damping)
    return raw, fin


def divergent(gpu_packets, oracle_packets):
    """Indices whose event sequence differs (branch ties decided differently)."""
    return np.nonzero((gpu_packets["hash"] != oracle_packets["hash"]) |
                      (gpu_packets["status"] != oracle_packets["status"]))[0]


def assert_packets_match(g, o, rel=REL, allow_fraction=DIVERGE_FRACTION):
    """Per-packet parity; returns the indices of packets whose event sequence
    took the other branch at a rounding tie, at most allow_fraction of them
    (none below 1/allow_fraction packets)."""
    assert g.shape == o.shape
    assert np.array_equal(g["id"], o["id"])
    bad = divergent(g, o)
    assert bad.size <= int(allow_fraction * g.size), f"{bad.size} divergent of {g.size} packets"
    ok = np.ones(g.size, dtype=bool)
    ok[bad] = False
    a, b = g[ok], o[ok]
    for f in ("n_segments", "n_escatter", "n_line", "n_passes", "last_line", "shell"):
        assert np.array_equal(a[f], b[f]), f
    for f in ("nu", "energy", "r", "nu_cmf0"):
        np.testing.assert_allclose(a[f], b[f], rtol=rel, atol=0, err_msg=f)
    for f in ("mu", "mu0"):
        np.testing.assert_allclose(a[f], b[f], rtol=rel, atol=rel, err_msg=f)
    return bad


def assert_close_or_zero(gpu, ref, rel=REL, what=""):
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    zero = ref == 0.0
    assert np.all(gpu[zero] == 0.0), f"{what}: nonzero where the oracle has zero"
    np.testing.assert_allclose(gpu[~zero], ref[~zero], rtol=rel, atol=0, err_msg=what)


def assert_estimators_match(est, spec, fin, rel=REL, jblue=True, T_R_W=True):
    """Normalised estimators and spectrum of one GPU iteration against the
    oracle's (section 2.7 J, nu-bar, J_blue; section 2.9 L_nu; the
    luminosity scalars and the next T_inner of section 2.8)."""
    assert_close_or_zero(est["J"], fin["J"], rel=rel, what="J")
    assert_close_or_zero(est["nubar"], fin["nubar"], rel=rel, what="nubar")
    if T_R_W:
        np.testing.assert_allclose(est["T_R"], fin["T_R"], rtol=rel, err_msg="T_R")
        np.testing.assert_allclose(est["W"], fin["W"], rtol=rel, err_msg="W")
    if jblue and fin.get("jblue") is not None:
        assert_close_or_zero(est["jblue"], fin["jblue"], rel=rel, what="jblue")
    assert_close_or_zero(spec["L_nu"], fin["L_nu"], rel=rel, what="L_nu")
    for k in ("L_emitted", "L_reabsorbed", "L_capped", "L_inner", "T_inner_next"):
        ref = fin[k]
        assert abs(spec[k] - ref) <= rel * abs(ref), (k, spec[k], ref)


def spectrum_chi2_pvalue(a, b, n_packets):
    """Two-sample chi-square on binned luminosities, each spectrum scaled to
    n_packets counts in total (the packets that built it), for bins with
    enough weight."""
    from scipy import stats
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    if a.sum() <= 0.0 or b.sum() <= 0.0:
        return 1.0
    a = a * (n_packets / a.sum())
    b = b * (n_packets / b.sum())
    keep = (a + b) > 0
    a, b = a[keep], b[keep]
    if a.size < 2:
        return 1.0
    s = a.sum() + b.sum()
    ea = (a + b) * a.sum() / s
    eb = (a + b) * b.sum() / s
    big = (ea > 5) & (eb > 5)
    if big.sum() < 2:
        return 1.0
    chi2 = (((a - ea) ** 2 / ea) + ((b - eb) ** 2 / eb))[big].sum()
    return float(stats.chi2.sf(chi2, big.sum() - 1))
