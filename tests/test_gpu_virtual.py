"""Virtual packets (section 2.9) on the GPU against the oracle: the v-packet
spectrum, its summed luminosity and the v-packet counts agree; the r-packet
histories are the same with and without v-packets; a multi-model launch
gives every model what it gets alone."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import REL, assert_packets_match, divergent

pytestmark = pytest.mark.gpu

F_ALL = smc.F_JBLUE | smc.F_PACKETS


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _gpu(ctx, model, N, T, nv, ids=None, tune=None):
    n_work = len(ids) if ids is not None else N
    m = smc.Model(ctx, model, n_work, flags=F_ALL)
    if tune:
        m.set_tune(**tune)
    m.run_iteration(N, T, flags=F_ALL, packet_ids=ids, n_virtual=nv)
    return dict(packets=m.read_packets(n_work), v=m.read_virtual_spectrum(),
                spec=m.read_spectrum(), counters=m.read_counters())


def _oracle(model, N, T, nv, ids=None):
    raw = O.run(model, T, N, packet_ids=ids, n_virtual=nv)
    fin = O.finalise(model, raw, T)
    return raw, fin


def _assert_vspec(g, fin, raw):
    ref = fin["L_nu_virtual"]
    # a v-packet whose depth rounds across the cut-off of 30 changes a bin by
    # at most exp(-30) of one packet's energy
    atol = 1e-12 * max(np.abs(ref).max(), 1e-300)
    np.testing.assert_allclose(g["v"]["L_nu"], ref, rtol=REL, atol=atol)
    assert g["v"]["L_total"] == pytest.approx(fin["L_virtual"], rel=REL, abs=0)
    assert g["v"]["counts"]["launched"] == raw["vcounts"]["launched"]
    assert abs(g["v"]["counts"]["counted"] - raw["vcounts"]["counted"]) <= 2
    assert abs(g["v"]["counts"]["passes"] - raw["vcounts"]["passes"]) <= 2 * 64


def _compare(ctx, model, N, T, nv, ids=None, tune=None):
    g = _gpu(ctx, model, N, T, nv, ids, tune)
    raw, fin = _oracle(model, N, T, nv, ids)
    bad = assert_packets_match(g["packets"], raw["packets"])
    if bad.size:
        all_ids = np.asarray(ids if ids is not None else np.arange(N), dtype=np.uint64)
        keep = np.delete(all_ids, bad)
        g = _gpu(ctx, model, N, T, nv, keep, tune)
        raw, fin = _oracle(model, N, T, nv, keep)
        assert divergent(g["packets"], raw["packets"]).size == 0
    _assert_vspec(g, fin, raw)
    assert raw["vcounts"]["counted"] > 0
    return g, raw, fin


@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_virtual_scatter_model(ctx, lanes):
    m = W.small_model(seed=61, n_shells=8, n_lines=800, tau="lognormal")
    _compare(ctx, m, 3000, 11000.0, 3, tune=dict(long_lanes=lanes))


def test_virtual_electron_scattering_shells(ctx):
    v, t, n_e = W.shells(3, 11000.0, 20000.0, 13.0)
    m = W.Model(v_bounds=v, t_exp=t, n_e=n_e * 20, line_nu=np.zeros(0),
                tau_sobolev=np.zeros((3, 0)), seed=62)
    _compare(ctx, m, 2000, 10000.0, 4)


def test_virtual_downbranch_model(ctx):
    m = W.small_downbranch_model(seed=63, n_shells=6, n_ions=4, n_levels_per_ion=12,
                                 n_lines=200)
    _compare(ctx, m, 2000, 12000.0, 2)


def test_virtual_paper_scale_sample(ctx):
    w = W.config2()
    ids = np.sort(np.random.default_rng(4).choice(w.n_packets, 600, replace=False)).astype(
        np.uint64)
    _compare(ctx, w.model, w.n_packets, w.T_inner, 3, ids=ids)


def test_virtual_leaves_r_histories_unchanged(ctx):
    m = W.small_model(seed=64, n_shells=6, n_lines=500)
    plain = smc.Model(ctx, m, 1500, flags=F_ALL)
    plain.run_iteration(1500, 10000.0, flags=F_ALL, n_virtual=0)
    withv = smc.Model(ctx, m, 1500, flags=F_ALL)
    withv.run_iteration(1500, 10000.0, flags=F_ALL, n_virtual=3)
    p0, p1 = plain.read_packets(1500), withv.read_packets(1500)
    # the v-packet run takes every history in the group kernel from its first
    # segment: same events, equal results up to rounding
    assert divergent(p0, p1).size <= 1
    np.testing.assert_allclose(p1["nu"], p0["nu"], rtol=REL)
    with pytest.raises(smc.SmcError):
        plain.read_virtual_spectrum()  # no v-packets in its last iteration


def test_virtual_in_a_multi_model_launch(ctx):
    mix = [(W.small_model(seed=70 + i, n_shells=4 + i, n_lines=300 * (i + 1)), 800 + 300 * i,
            10000.0 + 1000 * i, nv) for i, nv in enumerate([0, 2, 3])]
    models = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N, _, _ in mix]
    ctx.batch_run(models, [dict(n_packets=N, T_inner=T, flags=F_ALL, n_virtual=nv)
                           for _, N, T, nv in mix])
    for m, (mdl, N, T, nv) in zip(models, mix):
        if nv == 0:
            with pytest.raises(smc.SmcError):
                m.read_virtual_spectrum()
            continue
        raw, fin = _oracle(mdl, N, T, nv)
        g = dict(packets=m.read_packets(N), v=m.read_virtual_spectrum())
        if assert_packets_match(g["packets"], raw["packets"]).size == 0:
            _assert_vspec(g, fin, raw)


def test_virtual_rejects_too_many(ctx):
    m = W.small_model(seed=65, n_shells=3, n_lines=50)
    mm = smc.Model(ctx, m, 10)
    with pytest.raises(smc.SmcError):
        mm.run_iteration(10, 10000.0, n_virtual=17)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_virtual_configurations(ctx, seed):
    """Seeded random models with 1-6 v-packets per launch: shells, lines,
    packets, temperature and group width."""
    rng = np.random.default_rng(700 + seed)
    m = W.small_model(seed=700 + seed, n_shells=int(rng.integers(1, 20)),
                      n_lines=int(rng.integers(1, 1500)),
                      tau="lognormal" if seed % 2 else "loguniform")
    m.n_bins = int(rng.integers(1, 400))
    _compare(ctx, m, int(rng.integers(50, 2000)), float(rng.uniform(8000.0, 30000.0)),
             int(rng.integers(1, 7)), tune=dict(long_lanes=int(rng.choice([16, 32, 64]))))
