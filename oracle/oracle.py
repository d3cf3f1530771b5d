"""ctypes binding of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads oracle/liboracle.so (built by oracle/build.py) and takes a
``paper_1401_5469_amd.workloads.Model`` as input.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

SCATTER, DOWNBRANCH, MACROATOM = 0, 1, 2
LIVE, ESCAPED, REABSORBED, CAPPED = 0, 1, 2, 3
EV_INJECT, EV_SHELL_OUT, EV_SHELL_IN, EV_ESCATTER, EV_LINE = 0, 1, 2, 3, 4
COUNTER_NAMES = ("segments", "line_passes", "line_events", "escatters", "escaped",
                 "reabsorbed", "capped", "crossings")

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


class _Model(C.Structure):
    _fields_ = [("n_shells", C.c_int32), ("v_bounds", _dp), ("t_exp", C.c_double),
                ("n_e", _dp), ("n_lines", C.c_int64), ("line_nu", _dp), ("tau_sobolev", _dp),
                ("line_mode", C.c_int32), ("line_upper", _i32p), ("n_levels", C.c_int32),
                ("level_ptr", _i64p), ("em_line", _i32p), ("em_cum", _dp),
                ("nu_min", C.c_double), ("nu_max", C.c_double), ("n_bins", C.c_int32),
                ("seed", C.c_uint64)]


class _Iter(C.Structure):
    _fields_ = [("n_packets", C.c_uint64), ("iteration", C.c_uint32), ("T_inner", C.c_double),
                ("max_segments", C.c_uint64), ("packet_ids", _u64p), ("n_ids", C.c_uint64),
                ("want_jblue", C.c_int32), ("n_virtual", C.c_uint32)]


PACKET_DTYPE = np.dtype([("id", np.uint64), ("status", np.int32), ("shell", np.int32),
                         ("nu", np.float64), ("energy", np.float64), ("mu", np.float64),
                         ("r", np.float64), ("mu0", np.float64), ("nu_cmf0", np.float64),
                         ("n_segments", np.uint64), ("n_escatter", np.uint64),
                         ("n_line", np.uint64), ("n_passes", np.uint64), ("hash", np.uint64),
                         ("last_line", np.int64)], align=True)

EVENT_DTYPE = np.dtype([("packet_id", np.uint64), ("kind", np.int32), ("shell", np.int32),
                        ("line", np.int64), ("emit_line", np.int64), ("r", np.float64),
                        ("d", np.float64), ("mu_in", np.float64), ("mu_out", np.float64),
                        ("nu_in", np.float64), ("nu_out", np.float64), ("e_in", np.float64),
                        ("e_out", np.float64)], align=True)


class _Out(C.Structure):
    _fields_ = [("J_raw", _dp), ("nubar_raw", _dp), ("jblue_raw", _dp), ("spec_raw", _dp),
                ("L_raw", _dp), ("counters", _u64p), ("vspec_raw", _dp),
                ("vcounts", C.c_uint64 * 3), ("packets", C.c_void_p),
                ("trace", C.c_void_p), ("trace_cap", C.c_uint64), ("trace_len", C.c_uint64)]


class _Final(C.Structure):
    _fields_ = [("J", _dp), ("nubar", _dp), ("jblue", _dp), ("T_R", _dp), ("W", _dp),
                ("L_nu", _dp), ("L_nu_virtual", _dp), ("L_virtual", C.c_double),
                ("L_emitted", C.c_double), ("L_reabsorbed", C.c_double),
                ("L_capped", C.c_double), ("L_inner", C.c_double),
                ("T_inner_next", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(LIB_PATH)
        L.oracle_run.argtypes = [C.POINTER(_Model), C.POINTER(_Iter), C.POINTER(_Out)]
        L.oracle_run.restype = C.c_int
        L.oracle_finalise.argtypes = [C.POINTER(_Model), C.c_double, C.c_double, C.c_double,
                                      C.POINTER(_Out), C.POINTER(_Final)]
        L.oracle_finalise.restype = C.c_int
        L.oracle_initial_radiation_field.argtypes = [C.POINTER(_Model), _dp, _dp]
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_uniform.argtypes = [C.c_uint64]
        L.oracle_uniform.restype = C.c_double
        L.oracle_distance_to_shell.argtypes = [C.c_double] * 4
        L.oracle_distance_to_shell.restype = C.c_double
        L.oracle_inject.argtypes = [C.POINTER(_Model), C.c_double, C.c_uint64, C.c_uint32,
                                    C.c_uint64, _dp, _dp, _dp, _dp, _i64p]
        L.oracle_version.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.refs.append(a)
        return a


def _model_struct(model, keep: _Keep) -> _Model:
    m = _Model()
    S = model.n_shells
    L = model.n_lines
    m.n_shells = S
    m.v_bounds = _ptr(keep.arr(model.v_bounds, np.float64), _dp)
    m.t_exp = float(model.t_exp)
    m.n_e = _ptr(keep.arr(model.n_e, np.float64), _dp)
    m.n_lines = L
    m.line_nu = _ptr(keep.arr(model.line_nu if L else np.zeros(1), np.float64), _dp)
    tau = model.tau_sobolev if L else np.zeros((S, 1))
    m.tau_sobolev = _ptr(keep.arr(tau, np.float64), _dp)
    m.line_mode = int(model.line_mode)
    if model.line_mode in (DOWNBRANCH, MACROATOM) and model.em_cum is None:
        # a model whose macro-atom tables are still to be derived from the
        # plasma state: only its geometry may be used (the initial field)
        m.line_mode = SCATTER
    elif model.line_mode in (DOWNBRANCH, MACROATOM):
        m.line_upper = _ptr(keep.arr(model.line_upper, np.int32), _i32p)
        m.n_levels = int(model.n_levels)
        m.level_ptr = _ptr(keep.arr(model.level_ptr, np.int64), _i64p)
        m.em_line = _ptr(keep.arr(model.em_line, np.int32), _i32p)
        m.em_cum = _ptr(keep.arr(model.em_cum, np.float64), _dp)
    m.nu_min = float(model.nu_min)
    m.nu_max = float(model.nu_max)
    m.n_bins = int(model.n_bins)
    m.seed = int(model.seed)
    return m


def run(model, T_inner, n_packets, iteration=0, packet_ids=None, max_segments=10**9,
        want_jblue=True, want_packets=True, trace_cap=0, n_virtual=0):
    """One oracle iteration.  Returns a dict of raw (un-normalised) tallies,
    counters, per-packet records and the optional event trace; with
    n_virtual > 0 also the v-packet spectrum (section 2.9) and its counts."""
    if model.line_mode in (DOWNBRANCH, MACROATOM) and model.em_cum is None:
        raise ValueError("the model's macro-atom tables are not given (oracle.macroatom "
                         "derives them from a plasma state)")
    keep = _Keep()
    m = _model_struct(model, keep)
    it = _Iter()
    it.n_packets = int(n_packets)
    it.iteration = int(iteration)
    it.T_inner = float(T_inner)
    it.max_segments = int(max_segments)
    it.want_jblue = 1 if want_jblue else 0
    it.n_virtual = int(n_virtual)
    if packet_ids is not None:
        ids = keep.arr(packet_ids, np.uint64)
        it.packet_ids = _ptr(ids, _u64p)
        it.n_ids = ids.shape[0]
        n_rec = ids.shape[0]
    else:
        n_rec = int(n_packets)
    S, L = model.n_shells, model.n_lines
    res = dict(J_raw=np.zeros(S), nubar_raw=np.zeros(S),
               jblue_raw=np.zeros((S, L)) if want_jblue else None,
               spec_raw=np.zeros(model.n_bins + 2), L_raw=np.zeros(3),
               vspec_raw=np.zeros(model.n_bins + 2) if n_virtual else None,
               counters=np.zeros(8, dtype=np.uint64),
               packets=np.zeros(n_rec, dtype=PACKET_DTYPE) if want_packets else None,
               trace=np.zeros(trace_cap, dtype=EVENT_DTYPE) if trace_cap else None)
    o = _Out()
    o.J_raw = _ptr(res["J_raw"], _dp)
    o.nubar_raw = _ptr(res["nubar_raw"], _dp)
    o.jblue_raw = _ptr(res["jblue_raw"], _dp) if want_jblue and L > 0 else None
    o.spec_raw = _ptr(res["spec_raw"], _dp)
    o.L_raw = _ptr(res["L_raw"], _dp)
    o.counters = _ptr(res["counters"], _u64p)
    o.vspec_raw = _ptr(res["vspec_raw"], _dp) if n_virtual else None
    o.packets = res["packets"].ctypes.data if want_packets else None
    o.trace = res["trace"].ctypes.data if trace_cap else None
    o.trace_cap = int(trace_cap)
    rc = lib().oracle_run(C.byref(m), C.byref(it), C.byref(o))
    if rc != 0:
        raise ValueError("oracle_run rejected its input")
    if trace_cap:
        res["trace_len"] = int(o.trace_len)
        res["trace"] = res["trace"][: min(int(o.trace_len), trace_cap)]
    res["counters"] = {k: int(v) for k, v in zip(COUNTER_NAMES, res["counters"])}
    res["vcounts"] = dict(launched=int(o.vcounts[0]), counted=int(o.vcounts[1]),
                          passes=int(o.vcounts[2]))
    return res


def initial_radiation_field(model):
    keep = _Keep()
    m = _model_struct(model, keep)
    T_R = np.zeros(model.n_shells)
    W = np.zeros(model.n_shells)
    lib().oracle_initial_radiation_field(C.byref(m), _ptr(T_R, _dp), _ptr(W, _dp))
    return T_R, W


def finalise(model, raw, T_inner, L_requested=0.0, T_R_prev=None, W_prev=None, damping=1.0):
    """Normalised estimators, T_R, W and the next T_inner from raw tallies."""
    keep = _Keep()
    m = _model_struct(model, keep)
    S, L = model.n_shells, model.n_lines
    o = _Out()
    o.J_raw = _ptr(keep.arr(raw["J_raw"], np.float64), _dp)
    o.nubar_raw = _ptr(keep.arr(raw["nubar_raw"], np.float64), _dp)
    has_jb = raw.get("jblue_raw") is not None and L > 0
    o.jblue_raw = _ptr(keep.arr(raw["jblue_raw"], np.float64), _dp) if has_jb else None
    o.spec_raw = _ptr(keep.arr(raw["spec_raw"], np.float64), _dp)
    o.L_raw = _ptr(keep.arr(raw["L_raw"], np.float64), _dp)
    has_v = raw.get("vspec_raw") is not None
    o.vspec_raw = _ptr(keep.arr(raw["vspec_raw"], np.float64), _dp) if has_v else None
    if T_R_prev is None or W_prev is None:
        T_R_prev, W_prev = initial_radiation_field(model)
    out = dict(J=np.zeros(S), nubar=np.zeros(S), jblue=np.zeros((S, L)) if has_jb else None,
               T_R=np.array(T_R_prev, dtype=np.float64, copy=True),
               W=np.array(W_prev, dtype=np.float64, copy=True),
               L_nu=np.zeros(model.n_bins + 2),
               L_nu_virtual=np.zeros(model.n_bins + 2) if has_v else None)
    f = _Final()
    f.J = _ptr(out["J"], _dp)
    f.nubar = _ptr(out["nubar"], _dp)
    f.jblue = _ptr(out["jblue"], _dp) if has_jb else None
    f.T_R = _ptr(out["T_R"], _dp)
    f.W = _ptr(out["W"], _dp)
    f.L_nu = _ptr(out["L_nu"], _dp)
    f.L_nu_virtual = _ptr(out["L_nu_virtual"], _dp) if has_v else None
    lib().oracle_finalise(C.byref(m), float(T_inner), float(L_requested), float(damping),
                          C.byref(o), C.byref(f))
    out.update(L_emitted=f.L_emitted, L_reabsorbed=f.L_reabsorbed, L_capped=f.L_capped,
               L_inner=f.L_inner, T_inner_next=f.T_inner_next, L_virtual=f.L_virtual)
    return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(o, _u32p))
    return o


def uniform(word):
    return lib().oracle_uniform(int(word))


def distance_to_shell(r, mu, r_in, r_out):
    return lib().oracle_distance_to_shell(float(r), float(mu), float(r_in), float(r_out))


def inject(model, T_inner, n_packets, iteration, packet_id):
    keep = _Keep()
    m = _model_struct(model, keep)
    vals = [C.c_double() for _ in range(4)]
    nl = C.c_int64()
    lib().oracle_inject(C.byref(m), float(T_inner), int(n_packets), int(iteration),
                        int(packet_id), *[C.byref(v) for v in vals], C.byref(nl))
    mu, nu_cmf, nu_lab, e_lab = (v.value for v in vals)
    return dict(mu=mu, nu_cmf=nu_cmf, nu_lab=nu_lab, e_lab=e_lab, next_line=nl.value)
