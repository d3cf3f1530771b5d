"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, the Python structs match the header's layout, and host-side
validation rejects bad models before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1401_5469_amd import smc
from paper_1401_5469_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(smc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(smc.LIB_PATH):
        from paper_1401_5469_amd import build
        build.build()
    return smc.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 11
    assert set(names) == set(smc.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def _c_layout():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "smc.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("smc_model_desc %zu\n", sizeof(smc_model_desc));
  printf("smc_iter_params %zu\n", sizeof(smc_iter_params));
  printf("smc_packet_out %zu\n", sizeof(smc_packet_out));
  F(smc_model_desc, seed); F(smc_model_desc, n_em); F(smc_model_desc, nu_min);
  F(smc_iter_params, packet_ids); F(smc_iter_params, n_ids); F(smc_iter_params, damping);
  F(smc_packet_out, hash); F(smc_packet_out, last_line); F(smc_packet_out, nu_cmf0);
  printf("smc_plasma_desc %zu\n", sizeof(smc_plasma_desc));
  printf("smc_plasma_params %zu\n", sizeof(smc_plasma_params));
  F(smc_plasma_desc, element_ion_ptr); F(smc_plasma_desc, level_metastable);
  F(smc_plasma_desc, number_density); F(smc_plasma_params, delta); F(smc_plasma_params, W);
  F(smc_plasma_desc, n_nlte_ions); F(smc_plasma_desc, line_upsilon);
  F(smc_plasma_params, jblue_mode);
  return 0;
}
"""
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return dict(line.split() for line in out.strip().splitlines())


def test_python_structs_match_header_layout():
    lay = {k: int(v) for k, v in _c_layout().items()}
    assert lay["smc_model_desc"] == C.sizeof(smc.smc_model_desc)
    assert lay["smc_iter_params"] == C.sizeof(smc.smc_iter_params)
    assert lay["smc_packet_out"] == smc.PACKET_DTYPE.itemsize
    assert lay["smc_model_desc.seed"] == smc.smc_model_desc.seed.offset
    assert lay["smc_model_desc.n_em"] == smc.smc_model_desc.n_em.offset
    assert lay["smc_model_desc.nu_min"] == smc.smc_model_desc.nu_min.offset
    assert lay["smc_iter_params.packet_ids"] == smc.smc_iter_params.packet_ids.offset
    assert lay["smc_iter_params.n_ids"] == smc.smc_iter_params.n_ids.offset
    assert lay["smc_iter_params.damping"] == smc.smc_iter_params.damping.offset
    assert lay["smc_packet_out.hash"] == smc.PACKET_DTYPE.fields["hash"][1]
    assert lay["smc_packet_out.last_line"] == smc.PACKET_DTYPE.fields["last_line"][1]
    assert lay["smc_packet_out.nu_cmf0"] == smc.PACKET_DTYPE.fields["nu_cmf0"][1]
    assert lay["smc_plasma_desc"] == C.sizeof(smc.smc_plasma_desc)
    assert lay["smc_plasma_params"] == C.sizeof(smc.smc_plasma_params)
    for st, f in (("smc_plasma_desc", "element_ion_ptr"), ("smc_plasma_desc", "level_metastable"),
                  ("smc_plasma_desc", "number_density"), ("smc_plasma_params", "delta"),
                  ("smc_plasma_params", "W"), ("smc_plasma_desc", "n_nlte_ions"),
                  ("smc_plasma_desc", "line_upsilon"), ("smc_plasma_params", "jblue_mode")):
        assert lay[f"{st}.{f}"] == getattr(getattr(smc, st), f).offset


def test_workspace_size_grows_with_flags_and_packets(lib):
    m = W.small_model(seed=1, n_shells=5, n_lines=1000)
    base = smc.workspace_bytes(m, 1000, 0)
    jb = smc.workspace_bytes(m, 1000, smc.F_JBLUE)
    pk = smc.workspace_bytes(m, 1000, smc.F_JBLUE | smc.F_PACKETS)
    assert base >= m.nbytes()
    assert jb - base >= 5 * 1000 * 8
    assert pk - jb >= 1000 * smc.PACKET_DTYPE.itemsize
    assert smc.workspace_bytes(m, 2000, smc.F_PACKETS) > smc.workspace_bytes(m, 1000, smc.F_PACKETS)


def _expect_invalid(model):
    with pytest.raises(smc.SmcError) as ei:
        smc.workspace_bytes(model, 10, 0)
    assert ei.value.code == smc.SMC_EINVAL
    return str(ei.value)


def test_host_validation_rejects_bad_models(lib):
    m = W.small_model(seed=2, n_shells=4, n_lines=100)
    bad = W.Model(**{**m.__dict__})
    bad.line_nu = m.line_nu[::-1].copy()
    assert "non-increasing" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    bad.v_bounds = m.v_bounds[::-1].copy()
    assert "increasing" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    bad.v_bounds = m.v_bounds * (0.6 * 2.99792458e10 / m.v_bounds[-1])  # outer shell at 0.6 c
    assert "c/2" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    bad.n_e = -m.n_e
    assert "n_e" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    t = m.tau_sobolev.copy()
    t[1, 7] = -1.0
    bad.tau_sobolev = t
    assert "tau_sobolev" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    bad.nu_min, bad.nu_max = m.nu_max, m.nu_min
    assert "spectrum" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    bad.n_bins = 0
    assert "n_bins" in _expect_invalid(bad)
    # arrays shorter than the description's counts never reach the library
    for field, short in (("n_e", m.n_e[:-1]), ("tau_sobolev", m.tau_sobolev[:-1]),
                         ("tau_sobolev", m.tau_sobolev.T.copy())):
        bad = W.Model(**{**m.__dict__})
        setattr(bad, field, short)
        with pytest.raises(ValueError, match="tau_sobolev|n_e"):
            smc.workspace_bytes(bad, 10, 0)


def test_host_validation_rejects_bad_downbranch_tables(lib):
    m = W.small_downbranch_model(seed=3)
    assert smc.workspace_bytes(m, 10, 0) > 0
    bad = W.Model(**{**m.__dict__})
    lu = m.line_upper.copy()
    lu[0] = m.n_levels
    bad.line_upper = lu
    assert "line_upper" in _expect_invalid(bad)
    bad = W.Model(**{**m.__dict__})
    el = m.em_line.copy()
    el[0] = m.n_lines
    bad.em_line = el
    assert "em_line" in _expect_invalid(bad)
    for field in ("line_upper", "level_ptr", "em_cum"):
        bad = W.Model(**{**m.__dict__})
        setattr(bad, field, getattr(m, field)[:-1].copy())
        with pytest.raises(ValueError, match=field):
            smc.workspace_bytes(bad, 10, 0)
    # rows are searched by bisection: a decreasing pair inside a row is refused,
    # the step from one row's last entry to the next row's first is not
    lp = m.level_ptr
    v = int(np.nonzero(np.diff(lp) >= 2)[0][0])
    bad = W.Model(**{**m.__dict__})
    ec = m.em_cum.copy()
    ec[lp[v]], ec[lp[v] + 1] = 0.75, 0.5
    bad.em_cum = ec
    assert "non-decreasing" in _expect_invalid(bad)
    assert lp[v + 1] < len(m.em_cum) and m.em_cum[lp[v + 1]] < m.em_cum[lp[v + 1] - 1]


def test_host_validation_of_macroatom_tables(lib):
    m = W.macroatom_model(seed=1, n_shells=4, n_ions=3, n_levels_per_ion=10, n_lines=100)
    base = smc.workspace_bytes(m, 10, 0)
    assert base > 0
    bad = W.Model(**{**m.__dict__})
    el = m.em_line.copy()
    el[np.nonzero(el < 0)[0][0]] = -(m.n_levels + 5)
    bad.em_line = el
    assert "no row" in _expect_invalid(bad)
    # internal jumps are not allowed in downbranch mode
    bad = W.Model(**{**m.__dict__})
    bad.line_mode = W.DOWNBRANCH
    bad.em_cum = np.ascontiguousarray(m.em_cum[0])
    assert "em_line" in _expect_invalid(bad)
    # one probability set per shell
    bad = W.Model(**{**m.__dict__})
    ec = m.em_cum.copy()
    ec[-1, 3] = 1.5
    bad.em_cum = ec
    assert "em_cum" in _expect_invalid(bad)
    # each shell's rows must be sorted (here the last shell's)
    a, b = m.level_ptr[0], m.level_ptr[1]
    assert b - a >= 2
    bad = W.Model(**{**m.__dict__})
    ec = m.em_cum.copy()
    ec[-1, a:b] = ec[-1, a:b][::-1].copy()
    bad.em_cum = ec
    assert "non-decreasing" in _expect_invalid(bad)


def _plasma_spec():
    model, spec = W.plasma_model(seed=2, n_shells=3, n_elements=3, n_stages=3,
                                 n_levels_per_ion=8, n_lines=60)
    return model, spec


def _expect_plasma_invalid(spec, S=3, L=60):
    with pytest.raises(smc.SmcError) as ei:
        smc.plasma_workspace_bytes(spec, S, L)
    assert ei.value.code == smc.SMC_EINVAL
    return str(ei.value)


def _with_atom(spec, **kw):
    import dataclasses
    return W.PlasmaSpec(atom=dataclasses.replace(spec.atom, **kw),
                        number_density=spec.number_density)


def test_host_validation_of_plasma_descriptions(lib):
    model, spec = _plasma_spec()
    a = spec.atom
    base = smc.plasma_workspace_bytes(spec, 3, 60)
    assert base >= 3 * (a.n_levels + 2 * a.n_ions) * 8 + 60 * 32
    six = W.PlasmaSpec(atom=a, number_density=np.vstack([spec.number_density] * 2))
    assert smc.plasma_workspace_bytes(six, 6, 60) > base
    # arrays shorter than the description's counts never reach the library
    with pytest.raises(ValueError, match="number_density"):
        smc.plasma_workspace_bytes(spec, 6, 60)
    with pytest.raises(ValueError, match="line_lower"):
        smc.plasma_workspace_bytes(spec, 3, 61)
    with pytest.raises(ValueError, match="level_g"):
        smc.plasma_workspace_bytes(_with_atom(spec, level_g=a.level_g[:-1]), 3, 60)
    e = a.level_energy.copy()
    e[a.ion_level_ptr[1]] = 1e-12  # ground state above zero
    assert "ground state" in _expect_plasma_invalid(_with_atom(spec, level_energy=e))
    m = a.level_metastable.copy()
    m[a.ion_level_ptr[2]] = 0
    assert "ground state" in _expect_plasma_invalid(_with_atom(spec, level_metastable=m))
    lu = a.line_upper.copy()
    lu[0] = a.ion_level_ptr[-1] - 1 if a.line_lower[0] < a.ion_level_ptr[-2] else 0
    assert "different ions" in _expect_plasma_invalid(_with_atom(spec, line_upper=lu))
    lu = a.line_upper.copy()
    lu[3] = a.line_lower[3]
    assert "above the lower" in _expect_plasma_invalid(_with_atom(spec, line_upper=lu))
    z = a.ion_zeta.copy()
    z[1] = 1.5
    assert "zeta" in _expect_plasma_invalid(_with_atom(spec, ion_zeta=z))
    chi = a.ion_chi.copy()
    chi[0] = 0.0
    assert "ion_chi" in _expect_plasma_invalid(_with_atom(spec, ion_chi=chi))
    f = a.line_f.copy()
    f[5] = -1.0
    assert "line_f" in _expect_plasma_invalid(_with_atom(spec, line_f=f))
    g = a.level_g.copy()
    g[4] = 0.0
    assert "level_g" in _expect_plasma_invalid(_with_atom(spec, level_g=g))
    ptr = a.element_ion_ptr.copy()
    ptr[1] = ptr[0]
    assert "no ion stage" in _expect_plasma_invalid(_with_atom(spec, element_ion_ptr=ptr))
    d = spec.number_density.copy()
    d[2, 1] = -1.0
    assert "number_density" in _expect_plasma_invalid(W.PlasmaSpec(atom=a, number_density=d))
    # a model without lines needs no line records
    assert smc.plasma_workspace_bytes(spec, 3, 0) < base


def test_no_gpu_means_a_loud_error_not_a_fallback(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(smc.SmcError) as ei:
        smc.Context(0)
    assert ei.value.code in (smc.SMC_EDEVICE, smc.SMC_EINVAL)


def test_host_validation_of_nlte_ions(lib):
    import dataclasses
    model, spec = W.plasma_model(seed=3, n_shells=3, n_elements=3, n_stages=3,
                                 n_levels_per_ion=8, n_lines=60, nlte_ions=(4,),
                                 n_levels_nlte=6)
    L = model.n_lines
    assert smc.plasma_workspace_bytes(spec, 3, L) > smc.plasma_workspace_bytes(
        dataclasses.replace(spec, nlte_ions=()), 3, L)
    assert "listed twice" in _expect_plasma_invalid(dataclasses.replace(spec, nlte_ions=(4, 4)),
                                                    L=L)
    assert "out of range" in _expect_plasma_invalid(dataclasses.replace(spec, nlte_ions=(9,)),
                                                    L=L)
    a = spec.atom
    ups = a.line_upsilon.copy()
    l0, l1 = a.ion_level_ptr[4], a.ion_level_ptr[5]
    k = int(np.flatnonzero((a.line_lower >= l0) & (a.line_lower < l1))[0])
    ups[k] = -1.0
    bad = W.PlasmaSpec(atom=dataclasses.replace(a, line_upsilon=ups),
                       number_density=spec.number_density, nlte_ions=(4,))
    assert "line_upsilon" in _expect_plasma_invalid(bad, L=L)
    # an ion with more levels than the NLTE system holds
    big, bspec = W.plasma_model(seed=3, n_shells=3, n_elements=3, n_stages=3,
                                n_levels_per_ion=8, n_lines=300, nlte_ions=(4,),
                                n_levels_nlte=65)
    assert "levels" in _expect_plasma_invalid(bspec, L=big.n_lines)
    # a level that no line of the ion reaches
    ions = np.repeat(np.arange(a.n_ions), np.diff(a.ion_level_ptr))
    keep = ~((a.line_upper == l0 + 5) & (ions[a.line_lower] == 4))
    cut = W.PlasmaSpec(atom=dataclasses.replace(a, line_lower=a.line_lower[keep],
                                                line_upper=a.line_upper[keep],
                                                line_f=a.line_f[keep],
                                                line_upsilon=a.line_upsilon[keep]),
                       number_density=spec.number_density, nlte_ions=(4,))
    if not np.any((cut.atom.line_lower == l0 + 5) & (ions[cut.atom.line_upper] == 4)):
        assert "not joined" in _expect_plasma_invalid(cut, L=int(keep.sum()))
