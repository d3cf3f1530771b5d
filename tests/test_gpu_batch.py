"""Multi-model launches: a batch of models of uneven size in one set of
launches gives every model the results it gets alone (identical histories;
estimators equal up to the summation order) and the oracle's results."""
import numpy as np
import pytest

from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

from gpu_helpers import (REL, assert_close_or_zero, assert_estimators_match,
                         assert_packets_match, divergent, oracle_run)

pytestmark = pytest.mark.gpu

F_ALL = smc.F_JBLUE | smc.F_PACKETS


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return smc.Context(0)


def _mix():
    """Uneven models: shells, lines, packets and line modes all differ."""
    out = []
    for i, (S, L, N) in enumerate([(3, 50, 700), (12, 3000, 1500), (7, 800, 64), (20, 12000, 2500),
                                   (1, 10, 1), (9, 2000, 900)]):
        out.append((W.small_model(seed=100 + i, n_shells=S, n_lines=L, tau="lognormal"), N,
                    9000.0 + 500 * i))
    out.append((W.small_downbranch_model(seed=7, n_shells=5, n_ions=3, n_levels_per_ion=10,
                                         n_lines=120), 1200, 12000.0))
    return out


def _alone(ctx, model, N, T, tune=None):
    m = smc.Model(ctx, model, N, flags=F_ALL)
    if tune:
        m.set_tune(**tune)
    m.run_iteration(N, T, iteration=3, flags=F_ALL)
    return dict(packets=m.read_packets(N), est=m.read_estimators(), spec=m.read_spectrum(),
                counters=m.read_counters())


def _batch(ctx, mix, tune=None, ids=None, iteration=3, n_virtual=None):
    """One multi-model launch; ids: per model None (all packets) or the
    packet ids to run; n_virtual: per model v-packets per launch."""
    ids = ids or [None] * len(mix)
    nvs = n_virtual or [0] * len(mix)
    works = [N if k is None else len(k) for (_, N, _), k in zip(mix, ids)]
    models = [smc.Model(ctx, mdl, max(w, 1), flags=F_ALL) for (mdl, _, _), w in zip(mix, works)]
    params = [dict(n_packets=N, T_inner=T, iteration=iteration, flags=F_ALL, packet_ids=k,
                   n_virtual=nv) for (_, N, T), k, nv in zip(mix, ids, nvs)]
    ctx.batch_run(models, params, tune=tune)
    out = []
    for m, w, nv in zip(models, works, nvs):
        out.append(dict(packets=m.read_packets(w), est=m.read_estimators(),
                        spec=m.read_spectrum(), counters=m.read_counters(),
                        v=m.read_virtual_spectrum() if nv else None))
    return out


def _batch_against_oracle(ctx, mix, tune=None, iteration=3, n_virtual=None):
    """A multi-model launch against the oracle model by model: packets first;
    models with packets that took the other branch at a rounding tie are run
    again, in one launch, without them; then every model's estimators,
    spectrum, scalars and counters (and v-packet spectrum) are compared."""
    from oracle import oracle as O
    nvs = n_virtual or [0] * len(mix)
    together = _batch(ctx, mix, tune, iteration=iteration, n_virtual=nvs)
    keeps = []
    for (mdl, N, T), b, nv in zip(mix, together, nvs):
        raw = O.run(mdl, T, N, iteration=iteration, n_virtual=nv)
        bad = assert_packets_match(b["packets"], raw["packets"])
        keeps.append(None if bad.size == 0 else np.delete(np.arange(N, dtype=np.uint64), bad))
    if any(k is not None for k in keeps):
        together = _batch(ctx, mix, tune, ids=keeps, iteration=iteration, n_virtual=nvs)
    for (mdl, N, T), b, keep, nv in zip(mix, together, keeps, nvs):
        raw = O.run(mdl, T, N, iteration=iteration, packet_ids=keep, n_virtual=nv)
        fin = O.finalise(mdl, raw, T)
        assert divergent(b["packets"], raw["packets"]).size == 0
        assert_estimators_match(b["est"], b["spec"], fin, jblue=mdl.n_lines > 0)
        assert b["counters"] == raw["counters"]
        if nv:
            ref = fin["L_nu_virtual"]
            # a v-packet whose depth rounds across the cut-off changes a bin
            # by at most exp(-30) of one packet's energy
            atol = 1e-12 * max(np.abs(ref).max(), 1e-300)
            np.testing.assert_allclose(b["v"]["L_nu"], ref, rtol=REL, atol=atol)
            assert b["v"]["counts"]["launched"] == raw["vcounts"]["launched"]
    return together


@pytest.mark.parametrize("tune", [None, dict(long_budget=2), dict(long_budget=2, long_lanes=64),
                                  dict(long_budget=2**32 - 1),
                                  dict(blocks_per_cu=1, long_waves_per_cu=1, long_budget=5,
                                       long_lanes=32)],
                         ids=["default", "handoff2", "handoff2-lanes64", "nohandoff", "narrow"])
def test_batch_equals_alone(ctx, tune):
    mix = _mix()
    together = _batch(ctx, mix, tune)
    for (mdl, N, T), b in zip(mix, together):
        # the same hand-off budget and group width alone: each history takes
        # the same kernels with the same rounding (untuned, a multi-model
        # launch hands off after 4096 segments to 16 lanes per history, one
        # model alone after 256 to a wavefront per history)
        same = {k: v for k, v in (tune or {}).items() if k in ("long_budget", "long_lanes")}
        same.setdefault("long_budget", 4096)
        same.setdefault("long_lanes", 16)
        a = _alone(ctx, mdl, N, T, tune=same)
        assert np.array_equal(a["packets"], b["packets"])
        for k in ("J", "nubar", "T_R", "W"):
            np.testing.assert_allclose(b["est"][k], a["est"][k], rtol=1e-12, atol=0)
        assert_close_or_zero(b["est"]["jblue"], a["est"]["jblue"], rel=1e-12)
        assert_close_or_zero(b["spec"]["L_nu"], a["spec"]["L_nu"], rel=1e-12)
        assert a["counters"] == b["counters"]


def test_batch_matches_oracle(ctx):
    _batch_against_oracle(ctx, _mix(), dict(long_budget=3))


def test_batch_consecutive_calls_reuse_slots(ctx):
    """More batches in flight than staging slots: each still sees its own
    table (slots are reused only after their launch has finished)."""
    mix = _mix()[:3]
    models = [smc.Model(ctx, mdl, N, flags=F_ALL) for mdl, N, _ in mix]
    for it in range(6):
        params = [dict(n_packets=N, T_inner=T, iteration=it, flags=F_ALL) for _, N, T in mix]
        ctx.batch_run(models, params)
    for m, (mdl, N, T) in zip(models, mix):
        raw, _ = oracle_run(mdl, N, T, iteration=5)
        assert divergent(m.read_packets(N), raw["packets"]).size == 0


def test_batch_rejects_bad_calls(ctx):
    mdl, N, T = _mix()[0]
    m = smc.Model(ctx, mdl, N, flags=F_ALL)
    with pytest.raises(smc.SmcError):
        ctx.batch_run([m, m], [dict(n_packets=N, T_inner=T)] * 2)
    with pytest.raises(smc.SmcError):
        ctx.batch_run([m], [dict(n_packets=N + 1, T_inner=T)])  # beyond n_packets_max
    with pytest.raises(smc.SmcError):
        ctx.batch_run([m], [dict(n_packets=N, T_inner=0.0)])  # no T_inner yet


def test_batch_of_the_largest_model_count(ctx):
    """1024 models, the most one launch takes (2-6 shells, 20-49 lines, 1-89
    packets each, one of them downbranch every 64): every packet, estimator,
    spectrum and counter of every model matches the oracle."""
    mix = []
    for i in range(1024):
        if i % 64 == 63:
            mdl = W.small_downbranch_model(seed=2000 + i, n_shells=3, n_ions=2,
                                           n_levels_per_ion=6, n_lines=30)
        else:
            mdl = W.small_model(seed=2000 + i, n_shells=2 + i % 5, n_lines=20 + i % 30)
        mix.append((mdl, 1 + (i * 37) % 89, 8000.0 + 5.0 * i))
    _batch_against_oracle(ctx, mix)


@pytest.mark.parametrize("seed", range(6))
def test_random_mixed_batches(ctx, seed):
    """Seeded random batches of 2-24 models mixing scatter, downbranch and
    macroatom modes, some launching 1-4 v-packets per interaction, under a
    random tuning: every model's packets, estimators, spectrum, counters and
    v-packet spectrum against the oracle."""
    rng = np.random.default_rng(1200 + seed)
    mix, nvs = [], []
    for i in range(int(rng.integers(2, 25))):
        s = 1200 + 100 * seed + i
        kind = int(rng.integers(0, 3))
        if kind == 0:
            mdl = W.small_model(seed=s, n_shells=int(rng.integers(1, 15)),
                                n_lines=int(rng.integers(0, 1500)))
        elif kind == 1:
            mdl = W.small_downbranch_model(seed=s, n_shells=int(rng.integers(1, 10)), n_ions=3,
                                           n_levels_per_ion=10, n_lines=int(rng.integers(5, 120)))
        else:
            mdl = W.macroatom_model(seed=s, n_shells=int(rng.integers(1, 10)), n_ions=3,
                                    n_levels_per_ion=10, n_lines=int(rng.integers(5, 120)))
        mix.append((mdl, int(rng.integers(1, 1500)), float(rng.uniform(7000.0, 25000.0))))
        nvs.append(int(rng.integers(1, 5)) if (mdl.n_lines and rng.random() < 0.3) else 0)
    tune = [None, dict(long_budget=int(rng.integers(1, 64)), long_lanes=int(rng.choice([16, 32, 64]))),
            dict(long_budget=2**32 - 1)][seed % 3]
    _batch_against_oracle(ctx, mix, tune, iteration=2, n_virtual=nvs)
