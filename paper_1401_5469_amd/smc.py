"""Python binding of libsmc (include/smc.h): argument marshalling only.

Every step of the transport runs in the HIP library; this module allocates
the device workspace as a torch uint8 tensor, passes torch's current HIP
stream, and copies results into numpy arrays.  torch is imported before the
library is loaded so that both share one HIP runtime.  There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmc.so")

SMC_OK, SMC_EINVAL, SMC_ENOMEM, SMC_EDEVICE, SMC_EBUSY = 0, -1, -2, -3, -4
SCATTER, DOWNBRANCH, MACROATOM = 0, 1, 2
LIVE, ESCAPED, REABSORBED, CAPPED = 0, 1, 2, 3
F_JBLUE, F_PACKETS, F_TIMING = 1, 2, 4
STATIC_MAX_MODELS = 64  # models one smc_batch_run_static call takes
COUNTER_NAMES = ("segments", "line_passes", "line_events", "escatters", "escaped",
                 "reabsorbed", "capped", "crossings")

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)


class smc_model_desc(C.Structure):
    _fields_ = [("n_shells", C.c_int32), ("v_bounds", _dp), ("t_exp", C.c_double), ("n_e", _dp),
                ("n_lines", C.c_int64), ("line_nu", _dp), ("tau_sobolev", _dp),
                ("line_mode", C.c_int32), ("line_upper", _i32p), ("n_levels", C.c_int32),
                ("level_ptr", _i64p), ("n_em", C.c_int64), ("em_line", _i32p), ("em_cum", _dp),
                ("nu_min", C.c_double), ("nu_max", C.c_double), ("n_bins", C.c_int32),
                ("seed", C.c_uint64)]


class smc_tune(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("long_waves_per_cu", C.c_int32),
                ("long_budget", C.c_uint32), ("long_lanes", C.c_uint32)]


class smc_iter_params(C.Structure):
    _fields_ = [("n_packets", C.c_uint64), ("iteration", C.c_uint32), ("flags", C.c_uint32),
                ("T_inner", C.c_double), ("L_requested", C.c_double), ("damping", C.c_double),
                ("max_segments", C.c_uint64), ("packet_ids", C.c_void_p), ("n_ids", C.c_uint64),
                ("n_virtual", C.c_uint32), ("reserved", C.c_uint32)]


ION_LTE, ION_NEBULAR = 0, 1
EXC_LTE, EXC_DILUTE_LTE = 0, 1
JB_DILUTE_BLACKBODY, JB_DETAILED = 0, 1
_u8p = C.POINTER(C.c_uint8)


class smc_plasma_desc(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("n_ions", C.c_int32), ("n_levels", C.c_int32),
                ("n_nlte_ions", C.c_int32), ("element_ion_ptr", _i32p), ("ion_chi", _dp),
                ("ion_zeta", _dp), ("ion_level_ptr", _i32p), ("level_energy", _dp),
                ("level_g", _dp), ("level_metastable", _u8p), ("line_lower", _i32p),
                ("line_upper", _i32p), ("line_f", _dp), ("number_density", _dp),
                ("nlte_ions", _i32p), ("line_upsilon", _dp)]


class smc_plasma_params(C.Structure):
    _fields_ = [("ionization", C.c_int32), ("excitation", C.c_int32), ("delta", C.c_double),
                ("T_R", _dp), ("W", _dp), ("nlte", C.c_int32), ("jblue_mode", C.c_int32)]


PACKET_DTYPE = np.dtype([("id", np.uint64), ("status", np.int32), ("shell", np.int32),
                         ("nu", np.float64), ("energy", np.float64), ("mu", np.float64),
                         ("r", np.float64), ("mu0", np.float64), ("nu_cmf0", np.float64),
                         ("n_segments", np.uint64), ("n_escatter", np.uint64),
                         ("n_line", np.uint64), ("n_passes", np.uint64), ("hash", np.uint64),
                         ("last_line", np.int64)], align=True)

EXPORTS = ("smc_ctx_create", "smc_ctx_destroy", "smc_last_error", "smc_model_workspace_bytes",
           "smc_model_load", "smc_model_free", "smc_run_iteration", "smc_read_estimators",
           "smc_read_spectrum", "smc_read_counters", "smc_read_packets", "smc_read_timing",
           "smc_model_set_tune", "smc_model_get_tune", "smc_batch_run", "smc_batch_read_timing",
           "smc_batch_autotune", "smc_graph_capture", "smc_graph_launch", "smc_graph_destroy",
           "smc_read_virtual_spectrum", "smc_plasma_workspace_bytes", "smc_plasma_load",
           "smc_plasma_update", "smc_plasma_read", "smc_plasma_free", "smc_graph_capture_plasma",
           "smc_batch_run_static", "smc_measure_atomic_rate", "smc_model_read_macroatom")


class SmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsmc error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsmc.so (after torch, so that both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime libsmc links against)

    if not os.path.exists(path):
        raise RuntimeError(f"libsmc.so is not built ({path}); run python -m paper_1401_5469_amd.build")
    L = C.CDLL(path)
    vp = C.c_void_p
    L.smc_ctx_create.argtypes = [C.POINTER(vp), C.c_int]
    L.smc_ctx_destroy.argtypes = [vp]
    L.smc_last_error.restype = C.c_char_p
    L.smc_model_workspace_bytes.argtypes = [C.POINTER(smc_model_desc), C.c_uint64, C.c_uint32,
                                            C.POINTER(C.c_uint64)]
    L.smc_model_load.argtypes = [vp, C.POINTER(smc_model_desc), C.c_uint64, C.c_uint32, vp,
                                 C.c_uint64, vp, C.POINTER(vp)]
    L.smc_model_free.argtypes = [vp]
    L.smc_model_read_macroatom.argtypes = [vp, _i64p, _i32p, _dp, vp]
    L.smc_run_iteration.argtypes = [vp, C.POINTER(smc_iter_params), vp]
    L.smc_read_estimators.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, vp]
    L.smc_read_spectrum.argtypes = [vp, _dp, _dp, vp]
    L.smc_read_counters.argtypes = [vp, _u64p, vp]
    L.smc_read_virtual_spectrum.argtypes = [vp, _dp, _dp, _u64p, vp]
    L.smc_read_packets.argtypes = [vp, vp, C.c_uint64, vp]
    L.smc_read_timing.argtypes = [vp, _dp]
    L.smc_model_set_tune.argtypes = [vp, C.POINTER(smc_tune)]
    L.smc_batch_run.argtypes = [vp, C.POINTER(vp), C.POINTER(smc_iter_params), C.c_int,
                                C.POINTER(smc_tune), C.c_uint32, vp]
    L.smc_batch_run_static.argtypes = [vp, C.POINTER(vp), C.POINTER(smc_iter_params), C.c_int,
                                       C.POINTER(smc_tune), C.c_uint32, vp]
    L.smc_measure_atomic_rate.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_int, C.c_int, vp, _dp]
    L.smc_batch_read_timing.argtypes = [vp, _dp]
    L.smc_batch_autotune.argtypes = [vp, C.POINTER(vp), C.POINTER(smc_iter_params), C.c_int,
                                     C.POINTER(smc_tune), C.c_int, C.POINTER(smc_tune), _dp, vp]
    L.smc_graph_capture.argtypes = [vp, C.POINTER(vp), C.POINTER(smc_iter_params), C.c_int,
                                    C.c_int, C.POINTER(smc_tune), vp, C.POINTER(vp)]
    L.smc_graph_launch.argtypes = [vp, vp]
    L.smc_graph_destroy.argtypes = [vp]
    L.smc_model_get_tune.argtypes = [vp, C.POINTER(smc_tune)]
    L.smc_plasma_workspace_bytes.argtypes = [C.POINTER(smc_plasma_desc), C.c_int32, C.c_int64,
                                             C.POINTER(C.c_uint64)]
    L.smc_plasma_load.argtypes = [vp, C.POINTER(smc_plasma_desc), vp, C.c_uint64, vp,
                                  C.POINTER(vp)]
    L.smc_plasma_update.argtypes = [vp, C.POINTER(smc_plasma_params), vp]
    L.smc_plasma_read.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _u64p, vp]
    L.smc_plasma_free.argtypes = [vp]
    L.smc_graph_capture_plasma.argtypes = [vp, C.POINTER(vp), C.POINTER(smc_iter_params), C.c_int,
                                           C.c_int, C.POINTER(smc_tune), C.POINTER(vp),
                                           C.POINTER(smc_plasma_params), vp, C.POINTER(vp)]
    for name in EXPORTS:
        if name != "smc_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != SMC_OK:
        raise SmcError(rc, _lib.smc_last_error().decode(errors="replace"))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _tune(d):
    return smc_tune(int(d.get("blocks_per_cu", 0)), int(d.get("long_waves_per_cu", 0)),
                    int(d.get("long_budget", 0)), int(d.get("long_lanes", 0)))


class Graph:
    """A captured sequence of iterations (smc_graph_*)."""

    def __init__(self, handle, models, keep):
        self.handle = handle
        self.models = list(models)  # the workspaces must outlive the graph
        self._keep = keep

    def launch(self, stream=None):
        _check(_lib.smc_graph_launch(self.handle, _stream_ptr(stream)))

    def destroy(self):
        if self.handle:
            _lib.smc_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0):
        lib = load_library()
        h = C.c_void_p()
        _check(lib.smc_ctx_create(C.byref(h), int(device)))
        self.handle = h
        self.device = int(device)

    def batch_run(self, models, params, tune=None, timing=False, stream=None):
        """One iteration of every model in one set of launches.  params: one
        dict per model with the keyword arguments of Model.run_iteration."""
        n = len(models)
        if len(params) != n:
            raise ValueError("one parameter set per model")
        arr = (smc_iter_params * n)()
        handles = (C.c_void_p * n)()
        for k, (m, p) in enumerate(zip(models, params)):
            arr[k] = m._params(**p)
            handles[k] = m.handle
        t = _tune(tune) if tune else None
        _check(_lib.smc_batch_run(self.handle, handles, arr, n, C.byref(t) if t else None,
                                  F_TIMING if timing else 0, _stream_ptr(stream)))

    def batch_run_static(self, models, params, tune=None, timing=False, stream=None):
        """batch_run with the launch-wide scratch in the library's static
        device array: no allocation (at most STATIC_MAX_MODELS models)."""
        n = len(models)
        if len(params) != n:
            raise ValueError("one parameter set per model")
        arr = (smc_iter_params * n)()
        handles = (C.c_void_p * n)()
        for k, (m, p) in enumerate(zip(models, params)):
            arr[k] = m._params(**p)
            handles[k] = m.handle
        t = _tune(tune) if tune else None
        _check(_lib.smc_batch_run_static(self.handle, handles, arr, n,
                                         C.byref(t) if t else None,
                                         F_TIMING if timing else 0, _stream_ptr(stream)))

    def batch_autotune(self, models, params, candidates=None, stream=None):
        """Time the batch under each candidate tuning (default: the library's
        coordinate search) and return (best tuning dict, its ms)."""
        n = len(models)
        arr = (smc_iter_params * n)()
        handles = (C.c_void_p * n)()
        for k, (m, p) in enumerate(zip(models, params)):
            arr[k] = m._params(**p)
            handles[k] = m.handle
        cands, nc = None, 0
        if candidates:
            nc = len(candidates)
            cands = (smc_tune * nc)()
            for i, c in enumerate(candidates):
                cands[i] = _tune(c)
        best = smc_tune()
        ms = C.c_double()
        _check(_lib.smc_batch_autotune(self.handle, handles, arr, n, cands, nc, C.byref(best),
                                       C.byref(ms), _stream_ptr(stream)))
        return (dict(blocks_per_cu=best.blocks_per_cu, long_waves_per_cu=best.long_waves_per_cu,
                     long_budget=best.long_budget, long_lanes=best.long_lanes), float(ms.value))

    def capture(self, models, params_per_iter, tune=None, plasmas=None, plasma_params=None,
                stream=None):
        """Record iterations (a list, one list of per-model parameter dicts per
        iteration) into a replayable HIP graph.  plasmas: per model a Plasma
        (or None) updated after each of its iterations with plasma_params
        (per model a dict of Plasma.update's mode arguments)."""
        n, n_iter = len(models), len(params_per_iter)
        arr = (smc_iter_params * (n * n_iter))()
        handles = (C.c_void_p * n)()
        for k, m in enumerate(models):
            handles[k] = m.handle
        keep = []
        for i, plist in enumerate(params_per_iter):
            for k, (m, p) in enumerate(zip(models, plist)):
                arr[i * n + k] = m._params(**p)
                keep.append(m._ids)
        h = C.c_void_p()
        t = _tune(tune) if tune else None
        if plasmas is None:
            _check(_lib.smc_graph_capture(self.handle, handles, arr, n, n_iter,
                                          C.byref(t) if t else None, _stream_ptr(stream),
                                          C.byref(h)))
            return Graph(h, models, keep)
        ph = (C.c_void_p * n)()
        pp = (smc_plasma_params * n)()
        for k, pl in enumerate(plasmas):
            ph[k] = pl.handle if pl is not None else None
            q = dict((plasma_params or [{}] * n)[k] or {})
            pp[k].ionization = int(q.get("ionization", ION_NEBULAR))
            pp[k].excitation = int(q.get("excitation", EXC_DILUTE_LTE))
            pp[k].delta = float(q.get("delta", 1.0))
            pp[k].nlte = 1 if q.get("nlte", False) else 0
            pp[k].jblue_mode = int(q.get("jblue_mode", JB_DILUTE_BLACKBODY))
        _check(_lib.smc_graph_capture_plasma(self.handle, handles, arr, n, n_iter,
                                             C.byref(t) if t else None, ph, pp,
                                             _stream_ptr(stream), C.byref(h)))
        keep.append([pl for pl in plasmas if pl is not None])
        return Graph(h, models, keep)

    def batch_read_timing(self):
        ms = C.c_double()
        _check(_lib.smc_batch_read_timing(self.handle, C.byref(ms)))
        return float(ms.value)

    def close(self):
        if self.handle:
            _lib.smc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _need(a, n: int, what: str, at_least: bool = False):
    """The C descriptions carry counts, not array lengths: an array shorter
    than its count would be read past its end, so every length is checked
    here, before a pointer crosses the boundary."""
    got = -1 if a is None else int(np.size(a))
    if got < int(n) or (got != int(n) and not at_least):
        raise ValueError(f"{what} has {'no' if a is None else got} entries where the "
                         f"description needs {n}")


def derived_tables(model) -> bool:
    """A macroatom model without tables: a plasma object derives them."""
    return (model.line_mode == MACROATOM and model.level_ptr is None and model.em_line is None
            and model.em_cum is None)


def _desc(model, keep: list) -> smc_model_desc:
    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    d = smc_model_desc()
    S, L = model.n_shells, model.n_lines
    _need(model.n_e, S, "n_e")
    _need(model.tau_sobolev, S * L, "tau_sobolev")
    if L and np.ndim(model.tau_sobolev) == 2 and np.shape(model.tau_sobolev) != (S, L):
        raise ValueError(f"tau_sobolev must be [{S}, {L}], not {np.shape(model.tau_sobolev)}")
    derived = derived_tables(model)
    if model.line_mode in (DOWNBRANCH, MACROATOM) and not derived:
        n_em = int(np.size(model.em_line))
        _need(model.line_upper, L, "line_upper")
        _need(model.level_ptr, int(model.n_levels) + 1, "level_ptr")
        _need(model.em_cum, S * n_em if model.line_mode == MACROATOM else n_em, "em_cum")
    if derived:
        _need(model.line_upper, L, "line_upper")
    d.n_shells = S
    d.v_bounds = _ptr(arr(model.v_bounds, np.float64), _dp)
    d.t_exp = float(model.t_exp)
    d.n_e = _ptr(arr(model.n_e, np.float64), _dp)
    d.n_lines = L
    d.line_nu = _ptr(arr(model.line_nu if L else np.zeros(1), np.float64), _dp)
    d.tau_sobolev = _ptr(arr(model.tau_sobolev if L else np.zeros(1), np.float64), _dp)
    d.line_mode = int(model.line_mode)
    if derived:
        # the plasma object lays out the rows and derives the probabilities
        d.line_upper = _ptr(arr(model.line_upper, np.int32), _i32p)
        d.n_levels = int(model.n_levels)
    elif model.line_mode in (DOWNBRANCH, MACROATOM):
        d.line_upper = _ptr(arr(model.line_upper, np.int32), _i32p)
        d.n_levels = int(model.n_levels)
        d.level_ptr = _ptr(arr(model.level_ptr, np.int64), _i64p)
        d.n_em = int(model.em_line.shape[0])
        d.em_line = _ptr(arr(model.em_line, np.int32), _i32p)
        d.em_cum = _ptr(arr(model.em_cum, np.float64), _dp)
    d.nu_min = float(model.nu_min)
    d.nu_max = float(model.nu_max)
    d.n_bins = int(model.n_bins)
    d.seed = int(model.seed)
    return d


def workspace_bytes(model, n_packets_max: int, flags: int) -> int:
    lib = load_library()
    keep = []
    d = _desc(model, keep)
    out = C.c_uint64()
    _check(lib.smc_model_workspace_bytes(C.byref(d), int(n_packets_max), int(flags), C.byref(out)))
    return int(out.value)


class Model:
    """A model resident in device memory (section 2.1 shells, 2.5 lines)."""

    def __init__(self, ctx: Context, model, n_packets_max: int, flags: int = F_JBLUE,
                 workspace=None, stream=None):
        import torch
        lib = load_library()
        keep = []
        d = _desc(model, keep)
        need = workspace_bytes(model, n_packets_max, flags)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.workspace = workspace
        h = C.c_void_p()
        _check(lib.smc_model_load(ctx.handle, C.byref(d), int(n_packets_max), int(flags),
                                  C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                                  _stream_ptr(stream), C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.S, self.L, self.n_bins = model.n_shells, model.n_lines, model.n_bins
        self.line_mode = int(model.line_mode)
        self.n_levels = int(model.n_levels) if model.line_mode != SCATTER else 0
        self.n_em = (3 * model.n_lines if derived_tables(model) else
                     int(np.size(model.em_line)) if model.line_mode != SCATTER else 0)
        self.flags = flags
        self.n_packets_max = n_packets_max
        self._ids = None

    def free(self):
        if self.handle:
            _lib.smc_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def _params(self, n_packets: int, T_inner: float, iteration: int = 0,
                flags: Optional[int] = None, L_requested: float = 0.0, damping: float = 1.0,
                max_segments: int = 10**7, packet_ids=None, n_virtual: int = 0):
        import torch
        p = smc_iter_params()
        p.n_packets = int(n_packets)
        p.iteration = int(iteration)
        p.flags = int(self.flags if flags is None else flags)
        p.T_inner = float(T_inner)
        p.L_requested = float(L_requested)
        p.damping = float(damping)
        p.max_segments = int(max_segments)
        p.n_virtual = int(n_virtual)
        if packet_ids is not None:
            if not isinstance(packet_ids, torch.Tensor):
                packet_ids = torch.as_tensor(np.asarray(packet_ids, dtype=np.int64))
            ids = packet_ids.to(device=self.workspace.device, dtype=torch.int64).contiguous()
            self._ids = ids  # keep alive until the next iteration
            p.packet_ids = ids.data_ptr()
            p.n_ids = int(ids.numel())
        return p

    def run_iteration(self, n_packets: int, T_inner: float, iteration: int = 0,
                      flags: Optional[int] = None, L_requested: float = 0.0,
                      damping: float = 1.0, max_segments: int = 10**7, packet_ids=None,
                      n_virtual: int = 0, stream=None):
        """Enqueue one iteration.  packet_ids: optional torch int64/uint64
        CUDA tensor or numpy array of ids (copied to the device); n_virtual:
        virtual packets per packet launch (section 2.9)."""
        p = self._params(n_packets, T_inner, iteration, flags, L_requested, damping,
                         max_segments, packet_ids, n_virtual)
        _check(_lib.smc_run_iteration(self.handle, C.byref(p), _stream_ptr(stream)))

    def read_estimators(self, jblue: bool = True, stream=None):
        S, L = self.S, self.L
        out = dict(J=np.zeros(S), nubar=np.zeros(S), T_R=np.zeros(S), W=np.zeros(S),
                   jblue=np.zeros((S, L)) if jblue else None)
        _check(_lib.smc_read_estimators(self.handle, _ptr(out["J"], _dp), _ptr(out["nubar"], _dp),
                                        _ptr(out["jblue"], _dp), _ptr(out["T_R"], _dp),
                                        _ptr(out["W"], _dp), _stream_ptr(stream)))
        return out

    def read_spectrum(self, stream=None):
        L_nu = np.zeros(self.n_bins + 2)
        sc = np.zeros(6)
        _check(_lib.smc_read_spectrum(self.handle, _ptr(L_nu, _dp), _ptr(sc, _dp),
                                      _stream_ptr(stream)))
        return dict(L_nu=L_nu, L_emitted=sc[0], L_reabsorbed=sc[1], L_capped=sc[2],
                    L_inner=sc[3], T_inner=sc[4], T_inner_next=sc[5])

    def read_virtual_spectrum(self, stream=None):
        """v-packet spectrum of the last iteration: L_nu [n_bins + 2], the
        summed luminosity and the counts (launched, counted, passes)."""
        L_nu = np.zeros(self.n_bins + 2)
        tot = np.zeros(1)
        c = np.zeros(3, dtype=np.uint64)
        _check(_lib.smc_read_virtual_spectrum(self.handle, _ptr(L_nu, _dp), _ptr(tot, _dp),
                                              _ptr(c, _u64p), _stream_ptr(stream)))
        return dict(L_nu=L_nu, L_total=float(tot[0]),
                    counts=dict(launched=int(c[0]), counted=int(c[1]), passes=int(c[2])))

    def read_macroatom(self, stream=None):
        """The model's downbranch or macroatom tables: level_ptr, em_line and
        em_cum ([S, n_em] in macroatom mode)."""
        ptr = np.zeros(self.n_levels + 1, dtype=np.int64)
        line = np.zeros(self.n_em, dtype=np.int32)
        cum = np.zeros((self.S, self.n_em) if self.line_mode == MACROATOM else self.n_em)
        _check(_lib.smc_model_read_macroatom(self.handle, _ptr(ptr, _i64p), _ptr(line, _i32p),
                                             _ptr(cum, _dp), _stream_ptr(stream)))
        return ptr, line, cum

    def read_counters(self, stream=None):
        c = np.zeros(8, dtype=np.uint64)
        _check(_lib.smc_read_counters(self.handle, _ptr(c, _u64p), _stream_ptr(stream)))
        return {k: int(v) for k, v in zip(COUNTER_NAMES, c)}

    def set_tune(self, blocks_per_cu=0, long_waves_per_cu=0, long_budget=0, long_lanes=0):
        """Launch tuning (0 = library default; long_budget=2**32-1 disables
        the hand-off to the group-per-packet kernel; long_lanes = 16, 32 or
        64 lanes per handed-off history)."""
        t = smc_tune(int(blocks_per_cu), int(long_waves_per_cu), int(long_budget),
                     int(long_lanes))
        _check(_lib.smc_model_set_tune(self.handle, C.byref(t)))

    def get_tune(self):
        t = smc_tune()
        _check(_lib.smc_model_get_tune(self.handle, C.byref(t)))
        return dict(blocks_per_cu=t.blocks_per_cu, long_waves_per_cu=t.long_waves_per_cu,
                    long_budget=t.long_budget, long_lanes=t.long_lanes)

    def read_timing(self):
        """Transport-kernel duration of the last (timed) iteration in ms."""
        ms = C.c_double()
        _check(_lib.smc_read_timing(self.handle, C.byref(ms)))
        return float(ms.value)

    def read_packets(self, n: int, stream=None):
        out = np.zeros(int(n), dtype=PACKET_DTYPE)
        _check(_lib.smc_read_packets(self.handle, C.c_void_p(out.ctypes.data), int(n),
                                     _stream_ptr(stream)))
        return out


def _plasma_desc(spec, keep: list, n_shells: int, n_lines: int) -> smc_plasma_desc:
    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    atom = spec.atom
    E, NI, NL = atom.n_elements, atom.n_ions, atom.n_levels
    _need(atom.ion_zeta, NI, "ion_zeta")
    _need(atom.ion_level_ptr, NI + 1, "ion_level_ptr")
    _need(atom.level_g, NL, "level_g")
    _need(atom.level_metastable, NL, "level_metastable")
    # the library reads the first n_lines line records (none for a model
    # without lines)
    for name in ("line_lower", "line_upper", "line_f"):
        _need(getattr(atom, name), n_lines, name, at_least=True)
    _need(spec.number_density, int(n_shells) * E, "number_density")
    if getattr(spec, "nlte_ions", ()) and n_lines and atom.line_upsilon is not None:
        _need(atom.line_upsilon, n_lines, "line_upsilon", at_least=True)
    d = smc_plasma_desc()
    d.n_elements = atom.n_elements
    d.n_ions = atom.n_ions
    d.n_levels = atom.n_levels
    d.element_ion_ptr = _ptr(arr(atom.element_ion_ptr, np.int32), _i32p)
    d.ion_chi = _ptr(arr(atom.ion_chi, np.float64), _dp)
    d.ion_zeta = _ptr(arr(atom.ion_zeta, np.float64), _dp)
    d.ion_level_ptr = _ptr(arr(atom.ion_level_ptr, np.int32), _i32p)
    d.level_energy = _ptr(arr(atom.level_energy, np.float64), _dp)
    d.level_g = _ptr(arr(atom.level_g, np.float64), _dp)
    d.level_metastable = _ptr(arr(atom.level_metastable, np.uint8), _u8p)
    n_lines = atom.line_lower.shape[0]
    d.line_lower = _ptr(arr(atom.line_lower if n_lines else np.zeros(1), np.int32), _i32p)
    d.line_upper = _ptr(arr(atom.line_upper if n_lines else np.zeros(1), np.int32), _i32p)
    d.line_f = _ptr(arr(atom.line_f if n_lines else np.zeros(1), np.float64), _dp)
    d.number_density = _ptr(arr(spec.number_density, np.float64), _dp)
    nlte = tuple(getattr(spec, "nlte_ions", ()) or ())
    d.n_nlte_ions = len(nlte)
    if nlte:
        d.nlte_ions = _ptr(arr(np.asarray(nlte), np.int32), _i32p)
        ups = atom.line_upsilon if atom.line_upsilon is not None else np.zeros(max(n_lines, 1))
        d.line_upsilon = _ptr(arr(ups if n_lines else np.zeros(1), np.float64), _dp)
    return d


def plasma_workspace_bytes(spec, n_shells: int, n_lines: int) -> int:
    lib = load_library()
    keep = []
    d = _plasma_desc(spec, keep, n_shells, n_lines)
    out = C.c_uint64()
    _check(lib.smc_plasma_workspace_bytes(C.byref(d), int(n_shells), int(n_lines), C.byref(out)))
    return int(out.value)


class Plasma:
    """Plasma state of a loaded model (section 2.3) that rewrites its Sobolev
    depths and electron densities on the device (section 2.5)."""

    def __init__(self, model: Model, spec, workspace=None, stream=None):
        import torch
        lib = load_library()
        # the C description carries no array lengths: check them here
        if spec.atom.line_lower.shape[0] != model.L:
            raise ValueError(f"the atom lists {spec.atom.line_lower.shape[0]} lines, "
                             f"the model {model.L}")
        if np.shape(spec.number_density) != (model.S, spec.atom.n_elements):
            raise ValueError("number_density must be [n_shells, n_elements]")
        keep = []
        d = _plasma_desc(spec, keep, model.S, model.L)
        need = plasma_workspace_bytes(spec, model.S, model.L)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=model.workspace.device)
        self.workspace = workspace
        h = C.c_void_p()
        _check(lib.smc_plasma_load(model.handle, C.byref(d), C.c_void_p(workspace.data_ptr()),
                                   int(workspace.numel()), _stream_ptr(stream), C.byref(h)))
        self.handle = h
        self.model = model  # must outlive the plasma object
        self.S, self.L = model.S, model.L
        self.n_ions, self.n_levels = spec.atom.n_ions, spec.atom.n_levels

    def update(self, ionization: int = ION_NEBULAR, excitation: int = EXC_DILUTE_LTE,
               delta: float = 1.0, T_R=None, W=None, nlte: bool = False,
               jblue_mode: int = JB_DILUTE_BLACKBODY, stream=None):
        """Recompute the model's tau_sobolev and n_e from T_R, W (host arrays)
        or, when both are None, from the model's current radiation field;
        nlte: statistical equilibrium for the spec's NLTE ions, with J_b
        from jblue_mode."""
        p = smc_plasma_params()
        p.ionization = int(ionization)
        p.excitation = int(excitation)
        p.delta = float(delta)
        p.nlte = 1 if nlte else 0
        p.jblue_mode = int(jblue_mode)
        keep = []
        if T_R is not None or W is not None:
            t = np.ascontiguousarray(T_R, dtype=np.float64) if T_R is not None else None
            w = np.ascontiguousarray(W, dtype=np.float64) if W is not None else None
            for a in (t, w):
                if a is not None and a.shape != (self.S,):
                    raise ValueError("T_R and W need one value per shell")
            keep += [t, w]
            p.T_R = _ptr(t, _dp)
            p.W = _ptr(w, _dp)
        _check(_lib.smc_plasma_update(self.handle, C.byref(p), _stream_ptr(stream)))

    def read(self, tau: bool = True, level_pop: bool = True, stream=None):
        S, NI, NL, L = self.S, self.n_ions, self.n_levels, self.L
        out = dict(n_e=np.zeros(S), N_ion=np.zeros((S, NI)), Z=np.zeros((S, NI)),
                   level_pop=np.zeros((S, NL)) if level_pop else None,
                   tau=np.zeros((S, L)) if tau else None)
        c = np.zeros(2, dtype=np.uint64)
        _check(_lib.smc_plasma_read(self.handle, _ptr(out["n_e"], _dp), _ptr(out["N_ion"], _dp),
                                    _ptr(out["Z"], _dp), _ptr(out["level_pop"], _dp),
                                    _ptr(out["tau"], _dp), _ptr(c, _u64p), _stream_ptr(stream)))
        out["n_clamped"] = int(c[0])
        out["n_singular"] = int(c[1])
        return out

    def free(self):
        if self.handle:
            _lib.smc_plasma_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def measure_atomic_rate(table, n_rounds: int = 256, scattered: bool = False, stream=None) -> float:
    """FP64 atomic adds per second in a tally pattern (a wavefront's 64
    consecutive doubles, or with `scattered` a place per lane), on a caller's
    float64 CUDA tensor (overwritten); see smc_measure_atomic_rate."""
    import torch
    lib = load_library()
    if table.dtype != torch.float64 or not table.is_cuda or not table.is_contiguous():
        raise ValueError("table must be a contiguous float64 CUDA tensor")
    n_cu = torch.cuda.get_device_properties(table.device).multi_processor_count
    out = C.c_double()
    _check(lib.smc_measure_atomic_rate(C.c_void_p(table.data_ptr()), table.numel(), int(n_rounds),
                                       1 if scattered else 0, int(n_cu), _stream_ptr(stream),
                                       C.byref(out)))
    return float(out.value)
