"""Thin ctypes binding of libragsnn.so (include/ragsnn.h): argument marshalling
only.  Every computation runs in the HIP library; there is no fallback path.

Device buffers handed to the library (the input raster) are torch tensors on
the GPU; host snapshots are numpy arrays."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

from . import build as _build

RS_OK, RS_EINVAL, RS_ENOMEM, RS_ECAPACITY, RS_ESTATE, RS_EDEVICE = 0, -1, -2, -3, -4, -5
RS_LEARN, RS_AUTO_UPDATE, RS_AUTO_RESET = 1, 2, 4
NUM_PHASES = 5
PHASES = ("forward", "eprop", "update", "rewire", "reset")

# variable ids (include/ragsnn.h)
V, A, Y, XBAR, ZBAR, PSI, LSIG, DELTA, Z = range(1, 10)
WOUT, BOUT, GOUT, GB, MOUT, VOUT, MB, VB = range(0x0A, 0x12)
ZCOUNT = 0x12
ZBITS = 0x13
P_LEN, P_IND, P_W, P_M, P_V, P_G, P_EPS, P_EBAR, P_CONN, P_SIGN, P_DORMANT = range(1, 12)


def PROJ(p: int, f: int) -> int:
    return 0x100 * (p + 1) + f


class RagsnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ragsnn error {code}: {msg}")
        self.code = code


class _EpropParams(C.Structure):
    _fields_ = [("n_in", C.c_uint32), ("n_rec", C.c_uint32), ("n_out", C.c_uint32), ("batch", C.c_uint32),
                ("alif", C.c_int32),
                ("dt_ms", C.c_float), ("tau_mem_ms", C.c_float), ("tau_adapt_ms", C.c_float),
                ("v_thr", C.c_float), ("beta", C.c_float),
                ("p_in", C.c_float), ("p_rec", C.c_float),
                ("sigma_in", C.c_float), ("sigma_rec", C.c_float), ("sigma_out", C.c_float),
                ("cap_in", C.c_uint32), ("cap_rec", C.c_uint32),
                ("deepr_mask", C.c_uint32), ("l1", C.c_float),
                ("lr", C.c_float), ("adam_b1", C.c_float), ("adam_b2", C.c_float), ("adam_eps", C.c_float),
                ("update_interval", C.c_uint32), ("sample_steps", C.c_uint32), ("seed", C.c_uint64),
                ("trace_block", C.c_uint32), ("reserved", C.c_uint32)]


class _Stats(C.Structure):
    _fields_ = [("eliminated", C.c_int64), ("formed", C.c_int64), ("blocked", C.c_int64),
                ("attempts", C.c_int64)]


class _Info(C.Structure):
    _fields_ = [("cap_in", C.c_uint32), ("cap_rec", C.c_uint32), ("words_in", C.c_uint32),
                ("words_rec", C.c_uint32), ("step", C.c_uint64), ("adam_step", C.c_uint32),
                ("last_block", C.c_uint32), ("synaptic_events", C.c_uint64), ("spikes", C.c_uint64),
                ("device_bytes", C.c_uint64), ("eliminated", C.c_uint64), ("formed", C.c_uint64),
                ("trace_block", C.c_uint32), ("first_block", C.c_uint32)]


class _TopoParams(C.Structure):
    _fields_ = [("L", C.c_uint32), ("cap", C.c_uint32), ("n_attempts", C.c_uint32), ("proj_id", C.c_uint32),
                ("p_form", C.c_float), ("sigma_form", C.c_float), ("g_theta", C.c_float),
                ("p_elim_dep", C.c_float), ("p_elim_pot", C.c_float), ("g_new", C.c_float),
                ("g_init", C.c_float), ("seed", C.c_uint64)]


class _TopoModel(C.Structure):
    _fields_ = [("h", C.c_float), ("C_m", C.c_float), ("tau_m", C.c_float), ("V_rest", C.c_float),
                ("E_exc", C.c_float), ("V_th", C.c_float), ("V_reset", C.c_float), ("tau_s", C.c_float),
                ("ref_steps", C.c_uint32), ("f_base", C.c_float), ("f_peak", C.c_float),
                ("sigma_stim", C.c_float), ("stim_steps", C.c_uint32), ("stim_kind", C.c_int32),
                ("stdp", C.c_int32), ("g_max", C.c_float), ("A_plus", C.c_float), ("A_minus", C.c_float),
                ("tau_plus", C.c_float), ("tau_minus", C.c_float), ("rewire_steps", C.c_uint32),
                ("stim_tile", C.c_uint32)]


EXPORTS = [
    "rs_last_error", "rs_eprop_create", "rs_eprop_set_input", "rs_eprop_set_input_poisson",
    "rs_eprop_step", "rs_eprop_update",
    "rs_eprop_rewire", "rs_eprop_reset", "rs_eprop_get", "rs_eprop_set", "rs_eprop_info_get",
    "rs_eprop_timing", "rs_eprop_phase_times", "rs_eprop_destroy",
    "rs_topo_create", "rs_topo_rewire", "rs_topo_get_rows", "rs_topo_set_rows", "rs_topo_get_bits",
    "rs_topo_last_ms", "rs_topo_destroy", "rs_topo_sim_init", "rs_topo_run", "rs_topo_run_stats",
    "rs_topo_sim_get", "rs_topo_sim_set", "rs_topo_sim_timing", "rs_topo_sim_phase_ms", "rs_calib_copy",
    "rs_multi_create", "rs_multi_set_input", "rs_multi_set_input_poisson", "rs_multi_train",
    "rs_multi_schedule_get", "rs_multi_schedule_set", "rs_multi_get", "rs_multi_set", "rs_multi_info_get",
    "rs_multi_destroy",
    "rs_serve_create", "rs_serve_submit", "rs_serve_step", "rs_serve_poll", "rs_serve_stats_get",
    "rs_serve_replay", "rs_serve_destroy",
    "rs_create", "rs_add_pop", "rs_add_proj", "rs_build", "rs_eprop_of", "rs_topo_of", "rs_step", "rs_update",
    "rs_rewire", "rs_get_rows", "rs_get_var", "rs_set_var", "rs_sync", "rs_step_counter", "rs_destroy",
    "rs_deepr_rewire_noalloc", "rs_eprop_custom_update", "rs_topo_custom_update",
    "rs_topo_add_lateral", "rs_topo_lat_rewire", "rs_topo_lat_get_rows", "rs_topo_lat_set_rows",
    "rs_topo_lat_get_bits", "rs_topo_lat_run_stats", "rs_topo_sim_kernel",
]

_lib = None


def lib_path() -> str:
    return _build.LIB


def lib():
    """Load libragsnn.so, building it first only if no build exists."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        vp, st = C.c_void_p, C.c_int32
        L.rs_last_error.restype = C.c_char_p
        L.rs_eprop_create.argtypes = [C.POINTER(_EpropParams), vp, C.POINTER(vp)]
        L.rs_eprop_set_input.argtypes = [vp, vp, vp, C.c_size_t, vp]
        L.rs_eprop_set_input_poisson.argtypes = [vp, C.POINTER(C.c_double), C.c_size_t, vp]
        L.rs_eprop_step.argtypes = [vp, C.c_uint32, C.c_uint32]
        L.rs_eprop_update.argtypes = [vp]
        L.rs_eprop_rewire.argtypes = [vp, C.c_uint32, C.POINTER(_Stats)]
        L.rs_eprop_reset.argtypes = [vp]
        L.rs_eprop_get.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_eprop_set.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_eprop_info_get.argtypes = [vp, C.POINTER(_Info)]
        L.rs_eprop_timing.argtypes = [vp, C.c_int32]
        L.rs_eprop_phase_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
        L.rs_eprop_destroy.argtypes = [vp]
        L.rs_eprop_destroy.restype = None
        L.rs_topo_create.argtypes = [C.POINTER(_TopoParams), vp, C.POINTER(vp)]
        L.rs_topo_rewire.argtypes = [vp, C.c_uint64, C.POINTER(_Stats)]
        L.rs_topo_get_rows.argtypes = [vp, vp, vp, vp]
        L.rs_topo_set_rows.argtypes = [vp, vp, vp, vp]
        L.rs_topo_get_bits.argtypes = [vp, vp]
        L.rs_topo_last_ms.argtypes = [vp, C.POINTER(C.c_double)]
        L.rs_topo_destroy.argtypes = [vp]
        L.rs_topo_destroy.restype = None
        L.rs_topo_sim_init.argtypes = [vp, C.POINTER(_TopoModel)]
        L.rs_topo_run.argtypes = [vp, C.c_uint64]
        L.rs_topo_run_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.rs_topo_sim_get.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_topo_sim_set.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_topo_sim_timing.argtypes = [vp, C.c_int32]
        L.rs_topo_sim_phase_ms.argtypes = [vp, C.POINTER(C.c_double)]
        L.rs_topo_add_lateral.argtypes = [vp, C.POINTER(_TopoParams)]
        L.rs_topo_lat_rewire.argtypes = [vp, C.c_uint64, C.POINTER(_Stats)]
        L.rs_topo_lat_get_rows.argtypes = [vp, vp, vp, vp]
        L.rs_topo_lat_set_rows.argtypes = [vp, vp, vp, vp]
        L.rs_topo_lat_get_bits.argtypes = [vp, vp]
        L.rs_topo_lat_run_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.rs_topo_sim_kernel.argtypes = [vp, C.c_int32]
        L.rs_calib_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.rs_multi_create.argtypes = [C.POINTER(_EpropParams), C.c_uint32, vp, C.POINTER(vp)]
        L.rs_multi_set_input.argtypes = [vp, C.c_uint32, vp, vp, C.c_size_t, vp]
        L.rs_multi_set_input_poisson.argtypes = [vp, C.c_uint32, C.POINTER(C.c_double), C.c_size_t, vp]
        L.rs_multi_train.argtypes = [vp, C.c_uint32]
        L.rs_multi_schedule_get.argtypes = [vp, C.POINTER(_MultiSchedule)]
        L.rs_multi_schedule_set.argtypes = [vp, C.c_int32, C.c_int32]
        L.rs_multi_get.argtypes = [vp, C.c_uint32, C.c_int32, vp, C.c_size_t]
        L.rs_multi_set.argtypes = [vp, C.c_uint32, C.c_int32, vp, C.c_size_t]
        L.rs_multi_info_get.argtypes = [vp, C.c_uint32, C.POINTER(_Info)]
        L.rs_multi_destroy.argtypes = [vp]
        L.rs_multi_destroy.restype = None
        L.rs_serve_create.argtypes = [C.POINTER(vp), C.c_uint32, C.POINTER(_ServeParams), vp, C.POINTER(vp)]
        L.rs_serve_submit.argtypes = [vp, C.c_uint32, vp, vp, C.c_size_t, C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_uint64)]
        L.rs_serve_step.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.rs_serve_poll.argtypes = [vp, C.POINTER(_ServeResult), C.POINTER(C.c_double), C.c_uint32,
                                    C.POINTER(C.c_uint32)]
        L.rs_serve_stats_get.argtypes = [vp, C.POINTER(_ServeStats)]
        L.rs_serve_replay.argtypes = [vp, C.POINTER(_ServeRequest), C.c_uint32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]
        L.rs_serve_destroy.argtypes = [vp]
        L.rs_serve_destroy.restype = None
        L.rs_create.argtypes = [vp, _ALLOC_FN, _FREE_FN, vp, C.c_uint64, C.POINTER(vp)]
        L.rs_add_pop.argtypes = [vp, C.c_int32, C.c_uint32, C.POINTER(_PopParams), C.POINTER(C.c_uint32)]
        L.rs_add_proj.argtypes = [vp, C.c_uint32, C.c_uint32, C.POINTER(_ProjDesc), C.POINTER(C.c_uint32)]
        L.rs_build.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint32]
        L.rs_eprop_of.argtypes = [vp, C.POINTER(vp)]
        L.rs_topo_of.argtypes = [vp, C.POINTER(vp)]
        L.rs_step.argtypes = [vp, C.c_uint32, C.c_uint32]
        L.rs_update.argtypes = [vp]
        L.rs_rewire.argtypes = [vp, C.c_uint32, C.POINTER(_Stats)]
        L.rs_get_rows.argtypes = [vp, C.c_uint32, vp, vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.rs_get_var.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_set_var.argtypes = [vp, C.c_int32, vp, C.c_size_t]
        L.rs_sync.argtypes = [vp]
        L.rs_step_counter.argtypes = [vp]
        L.rs_step_counter.restype = C.c_uint64
        L.rs_destroy.argtypes = [vp]
        L.rs_destroy.restype = None
        L.rs_deepr_rewire_noalloc.argtypes = [C.POINTER(_DeeprRows), C.c_uint64, C.c_uint32, C.c_uint64, vp,
                                              C.POINTER(_Stats)]
        L.rs_eprop_custom_update.argtypes = [vp, C.c_uint32, C.c_int32, C.c_uint64, _HOST_FN, vp, C.POINTER(_Stats)]
        L.rs_topo_custom_update.argtypes = [vp, C.c_int32, C.c_uint64, _HOST_FN, vp, C.POINTER(_Stats)]
        for name in EXPORTS:
            f = getattr(L, name)
            if name not in ("rs_last_error", "rs_eprop_destroy", "rs_topo_destroy", "rs_multi_destroy",
                            "rs_serve_destroy", "rs_destroy", "rs_step_counter"):
                f.restype = st
        _lib = L
    return _lib


def _check(code: int):
    if code != RS_OK:
        raise RagsnnError(code, lib().rs_last_error().decode())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class EpropConfig:
    n_in: int
    n_rec: int
    n_out: int
    batch: int
    alif: bool = True
    dt_ms: float = 1.0
    tau_mem_ms: float = 20.0
    tau_adapt_ms: float = 2000.0
    v_thr: float = 0.6
    beta: float = 0.0174
    p_in: float = 0.1
    p_rec: float = 0.1
    sigma_in: float = 0.0
    sigma_rec: float = 0.0
    sigma_out: float = 0.0
    cap_in: int = 0
    cap_rec: int = 0
    deepr_mask: int = 3
    l1: float = 0.005
    lr: float = 1e-3
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8
    update_interval: int = 100
    sample_steps: int = 1000
    seed: int = 1
    trace_block: int = 0

    def c(self) -> _EpropParams:
        p = _EpropParams()
        for f in fields(self):
            setattr(p, f.name, int(getattr(self, f.name)) if isinstance(getattr(self, f.name), bool)
                    else getattr(self, f.name))
        return p


@dataclass
class RewireStats:
    eliminated: int
    formed: int
    blocked: int
    attempts: int


class EpropNet:
    """e-prop classifier network held on the GPU (rs_eprop_*)."""

    def __init__(self, cfg: EpropConfig, stream=None):
        self.cfg = cfg
        self._h = C.c_void_p()
        self._stream = _stream_ptr(stream)
        self._input_refs = None
        _check(lib().rs_eprop_create(C.byref(cfg.c()), self._stream, C.byref(self._h)))
        self.info()

    @classmethod
    def _view(cls, handle, cfg, owner):
        """A network owned by another object (it is not destroyed by close)."""
        v = cls.__new__(cls)
        v.cfg, v._h, v._owner, v._input_refs = cfg, handle, owner, None
        v._stream = None
        v.info()
        return v

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = C.c_void_p()
            return
        if self._h:
            lib().rs_eprop_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- input
    def set_input(self, off, idx, labels):
        """off/idx/labels: int32 CUDA tensors (kept alive by this object)."""
        import torch
        for t in (off, idx, labels):
            assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()
        self._input_refs = (off, idx, labels)
        _check(lib().rs_eprop_set_input(self._h, C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()),
                                        idx.numel(), C.c_void_p(labels.data_ptr())))

    def set_input_poisson(self, rates_hz, labels):
        """rates_hz: host float64 [n_in] or [batch][n_in]; labels: int32 CUDA
        tensor (kept alive by this object)."""
        import torch
        assert isinstance(labels, torch.Tensor) and labels.is_cuda and labels.dtype == torch.int32
        assert labels.is_contiguous()
        r = np.ascontiguousarray(rates_hz, np.float64)
        self._input_refs = (labels,)
        _check(lib().rs_eprop_set_input_poisson(self._h, r.ctypes.data_as(C.POINTER(C.c_double)), r.size,
                                                C.c_void_p(labels.data_ptr())))

    # ---- simulation
    def step(self, n: int = 1, flags: int = RS_LEARN):
        _check(lib().rs_eprop_step(self._h, n, flags))

    def update(self):
        _check(lib().rs_eprop_update(self._h))

    def rewire(self, proj: int) -> RewireStats:
        st = _Stats()
        _check(lib().rs_eprop_rewire(self._h, proj, C.byref(st)))
        return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts)

    def reset(self):
        _check(lib().rs_eprop_reset(self._h))

    def custom_update(self, proj: int, rule: int, step: int, host_fn=None) -> RewireStats:
        """A custom connectivity update (rs_eprop_custom_update); host_fn(len,
        pre_var, info) may change the rule's per-row variable in place."""
        st = _Stats()
        cb = _host_fn(host_fn)
        _check(lib().rs_eprop_custom_update(self._h, proj, rule, step, cb, None, C.byref(st)))
        return _custom_stats(st)

    # ---- snapshots
    def shape_of(self, var: int):
        return _shape_of(self.cfg, self._info, var)

    def get(self, var: int) -> np.ndarray:
        shape, dt = self.shape_of(var)
        a = np.empty(shape, dt)
        _check(lib().rs_eprop_get(self._h, var, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return a

    def set(self, var: int, value):
        shape, dt = self.shape_of(var)
        a = np.ascontiguousarray(np.asarray(value, dtype=dt).reshape(shape))
        _check(lib().rs_eprop_set(self._h, var, a.ctypes.data_as(C.c_void_p), a.nbytes))

    def info(self) -> _Info:
        inf = _Info()
        _check(lib().rs_eprop_info_get(self._h, C.byref(inf)))
        self._info = inf
        return inf

    def timing(self, enable=True):
        """enable: True (all phases), False, or a bit mask of phases to time."""
        mask = (1 << NUM_PHASES) - 1 if enable is True else (0 if enable is False else int(enable))
        _check(lib().rs_eprop_timing(self._h, mask))

    def phase_times(self):
        ms = (C.c_double * NUM_PHASES)()
        cnt = (C.c_uint64 * NUM_PHASES)()
        _check(lib().rs_eprop_phase_times(self._h, ms, cnt))
        return {PHASES[q]: (ms[q], cnt[q]) for q in range(NUM_PHASES)}


def _shape_of(c, inf, var: int):
    """Shape and dtype of variable `var` of a network with config c and info inf."""
    B, NR, NI, K = c.batch, c.n_rec, c.n_in, c.n_out
    net = {V: ((B, NR), np.float64), A: ((B, NR), np.float64), Y: ((B, K), np.float64),
           XBAR: ((B, NI), np.float32), ZBAR: ((B, NR), np.float32), PSI: ((NR, B), np.float32),
           LSIG: ((NR, B), np.float32), DELTA: ((K, B), np.float32), Z: ((B, NR), np.uint8),
           WOUT: ((K, NR), np.float32), BOUT: ((K,), np.float32), GOUT: ((K, NR), np.float32),
           GB: ((K,), np.float32), MOUT: ((K, NR), np.float32), VOUT: ((K, NR), np.float32),
           MB: ((K,), np.float32), VB: ((K,), np.float32), ZCOUNT: ((B, NR), np.uint32),
           ZBITS: ((NR, B), np.uint32)}
    if var in net:
        return net[var]
    p, f = var // 0x100 - 1, var % 0x100
    n_pre = NI if p == 0 else NR
    cap = inf.cap_in if p == 0 else inf.cap_rec
    words = inf.words_in if p == 0 else inf.words_rec
    return {P_LEN: ((n_pre,), np.int32), P_IND: ((n_pre, cap), np.int32), P_W: ((n_pre, cap), np.float32),
            P_M: ((n_pre, cap), np.float32), P_V: ((n_pre, cap), np.float32), P_G: ((n_pre, cap), np.float32),
            P_EPS: ((n_pre, cap, B), np.float32), P_EBAR: ((n_pre, cap, B), np.float32),
            P_CONN: ((n_pre, words), np.uint32), P_SIGN: ((n_pre, words), np.uint32),
            P_DORMANT: ((n_pre,), np.int32)}[f]


RULE_ADD_DIAGONAL, RULE_REMOVE_RANDOM, RULE_DEEPR, RULE_TOPO = 1, 2, 3, 4


class _CustomHost(C.Structure):
    _fields_ = [("n_pre", C.c_int32), ("n_post", C.c_int32), ("cap", C.c_int32), ("recurrent", C.c_int32),
                ("len", C.POINTER(C.c_int32)), ("pre_var", C.POINTER(C.c_uint32)), ("seed", C.c_uint64),
                ("step", C.c_uint64), ("proj_id", C.c_uint32), ("rule", C.c_int32)]


_HOST_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(_CustomHost))


def _host_fn(fn):
    """Wrap fn(len: np.ndarray, pre_var: np.ndarray (writable), info: dict) as
    a host function of a custom connectivity update."""
    if fn is None:
        return _HOST_FN()

    def call(user, hp):
        h = hp.contents
        ln = np.ctypeslib.as_array(h.len, shape=(h.n_pre,))
        var = np.ctypeslib.as_array(h.pre_var, shape=(h.n_pre,))
        fn(ln, var, dict(n_pre=h.n_pre, n_post=h.n_post, cap=h.cap, recurrent=bool(h.recurrent), seed=h.seed,
                         step=h.step, proj_id=h.proj_id, rule=h.rule))
    return _HOST_FN(call)


def _custom_stats(st):
    return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts)


class _DeeprRows(C.Structure):
    _fields_ = [("n_pre", C.c_int32), ("n_post", C.c_int32), ("cap", C.c_int32), ("words", C.c_int32),
                ("recurrent", C.c_int32), ("batch", C.c_int32)] + \
               [(f, C.c_void_p) for f in ("len", "ind", "w", "m", "v", "G", "eps", "ebar", "conn", "sign")]


def deepr_rewire_noalloc(arrays: dict, n_post: int, recurrent: bool, seed: int, proj_id: int, step: int,
                         stream=None) -> RewireStats:
    """DEEP R of caller-owned rows (rs_deepr_rewire_noalloc): arrays maps len,
    ind, w, m, v, G, eps (optional), ebar, conn, sign to contiguous CUDA
    tensors in the rs_eprop_get layout."""
    n_pre, cap = arrays["ind"].shape
    batch = arrays["ebar"].shape[2]
    r = _DeeprRows(n_pre, n_post, cap, (n_post + 31) // 32, int(recurrent), batch,
                   *[C.c_void_p(arrays[f].data_ptr()) if arrays.get(f) is not None else None
                     for f in ("len", "ind", "w", "m", "v", "G", "eps", "ebar", "conn", "sign")])
    st = _Stats()
    _check(lib().rs_deepr_rewire_noalloc(C.byref(r), seed, proj_id, step, _stream_ptr(stream), C.byref(st)))
    return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts)


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

POP_SPIKE_SOURCE, POP_LIF, POP_ALIF, POP_READOUT, POP_POISSON_SHEET, POP_COND_LIF_SHEET = range(6)
INIT_FIXED_PROB, INIT_GAUSS_TORUS, INIT_DENSE = range(3)
LEARN_NONE, LEARN_EPROP, LEARN_STDP = range(3)
REWIRE_NONE, REWIRE_DEEPR, REWIRE_TOPO = range(3)


class _PopParams(C.Structure):
    _fields_ = [("dt_ms", C.c_float), ("tau_mem_ms", C.c_float), ("tau_adapt_ms", C.c_float), ("v_thr", C.c_float),
                ("beta", C.c_float), ("L", C.c_uint32), ("model", _TopoModel)]


class _ProjDesc(C.Structure):
    _fields_ = [("init", C.c_int32), ("p", C.c_float), ("sigma_w", C.c_float), ("p_form", C.c_float),
                ("sigma_form", C.c_float), ("g_init", C.c_float), ("cap", C.c_uint32), ("learn", C.c_int32),
                ("lr", C.c_float), ("adam_b1", C.c_float), ("adam_b2", C.c_float), ("adam_eps", C.c_float),
                ("rewire", C.c_int32), ("l1", C.c_float), ("n_attempts", C.c_uint32), ("g_theta", C.c_float),
                ("p_elim_dep", C.c_float), ("p_elim_pot", C.c_float), ("g_new", C.c_float),
                ("update_interval", C.c_uint32)]


def torch_allocator():
    """Allocator callbacks bound to torch's caching allocator (on the current
    device and stream)."""
    import torch

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    return _ALLOC_FN(alloc), _FREE_FN(free)


class ComposedNet:
    """A network declared population by population and projection by
    projection (rs_create / rs_add_pop / rs_add_proj / rs_build).  With
    allocator=True its device memory comes from torch's caching allocator."""

    def __init__(self, seed=1, allocator=True, stream=None):
        self._h = C.c_void_p()
        self._fns = torch_allocator() if allocator else (_ALLOC_FN(), _FREE_FN())
        _check(lib().rs_create(_stream_ptr(stream), self._fns[0], self._fns[1], None, seed, C.byref(self._h)))
        self.pops, self.projs = [], []

    def close(self):
        if self._h:
            lib().rs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_pop(self, kind, n, dt_ms=1.0, tau_mem_ms=20.0, tau_adapt_ms=2000.0, v_thr=0.6, beta=0.0174, L=0,
                model=None):
        p = _PopParams(dt_ms, tau_mem_ms, tau_adapt_ms, v_thr, beta, L, (model or TopoModel()).c())
        q = C.c_uint32()
        _check(lib().rs_add_pop(self._h, kind, n, C.byref(p), C.byref(q)))
        self.pops.append((kind, n))
        return q.value

    def add_proj(self, pre, post, **kw):
        d = _ProjDesc()
        d.adam_b1, d.adam_b2, d.adam_eps, d.lr = 0.9, 0.999, 1e-8, 1e-3
        for k, v in kw.items():
            setattr(d, k, v)
        q = C.c_uint32()
        _check(lib().rs_add_proj(self._h, pre, post, C.byref(d), C.byref(q)))
        self.projs.append(kw)
        return q.value

    def build(self, batch=1, sample_steps=1000, trace_block=0):
        _check(lib().rs_build(self._h, batch, sample_steps, trace_block))

    def eprop(self, cfg):
        """The built classifier as an EpropNet view (owned by this network)."""
        h = C.c_void_p()
        _check(lib().rs_eprop_of(self._h, C.byref(h)))
        return EpropNet._view(h, cfg, self)

    def topo(self, cfg, lat_cfg=None):
        """The built map's rs_topo object (cfg, lat_cfg: its projections' shapes)."""
        h = C.c_void_p()
        _check(lib().rs_topo_of(self._h, C.byref(h)))
        v = TopoNet._view(h, cfg, self)
        if lat_cfg is not None:
            v.lat_cfg = lat_cfg
        return v

    def step(self, n, flags=RS_LEARN):
        _check(lib().rs_step(self._h, n, flags))

    def rewire(self, proj) -> RewireStats:
        st = _Stats()
        _check(lib().rs_rewire(self._h, proj, C.byref(st)))
        return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts)

    def step_counter(self) -> int:
        return int(lib().rs_step_counter(self._h))


class _ServeParams(C.Structure):
    _fields_ = [("slots_per_model", C.c_uint32), ("block_steps", C.c_uint32), ("max_running", C.c_uint32),
                ("max_queue", C.c_uint32), ("state_budget_bytes", C.c_uint64)]


class _ServeResult(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("model", C.c_uint32), ("steps", C.c_uint32), ("decision", C.c_int32),
                ("reserved", C.c_uint32), ("spikes", C.c_uint64), ("events", C.c_uint64),
                ("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double)]


class _ServeStats(C.Structure):
    _fields_ = [("admitted", C.c_uint64), ("rejected", C.c_uint64), ("completed", C.c_uint64),
                ("blocks", C.c_uint64), ("queued", C.c_uint64), ("running", C.c_uint32),
                ("n_out_max", C.c_uint32), ("state_bytes_used", C.c_uint64), ("state_budget_bytes", C.c_uint64),
                ("clock_s", C.c_double)]


class _ServeRequest(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("model", C.c_uint32), ("n_steps", C.c_uint32),
                ("raster_steps", C.c_uint32), ("reserved", C.c_uint32), ("off_dev", C.c_void_p),
                ("idx_dev", C.c_void_p), ("n_idx", C.c_size_t)]


class Server:
    """Served inference with continuous batching over trained networks (rs_serve_*).
    `models` are EpropNet objects, kept alive by the server."""

    def __init__(self, models, slots_per_model=256, block_steps=20, max_running=1024, max_queue=1 << 20,
                 state_budget_bytes=1 << 30, stream=None):
        self.models = list(models)
        arr = (C.c_void_p * len(self.models))(*[m._h.value for m in self.models])
        prm = _ServeParams(slots_per_model, block_steps, max_running, max_queue, state_budget_bytes)
        self._h = C.c_void_p()
        self._refs = []
        _check(lib().rs_serve_create(arr, len(self.models), C.byref(prm), _stream_ptr(stream), C.byref(self._h)))
        self.n_out_max = max(m.cfg.n_out for m in self.models)

    def close(self):
        if self._h:
            lib().rs_serve_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, model, off, idx, raster_steps, n_steps):
        """off/idx: int32 CUDA tensors of a batch-1 raster (kept alive by the server).
        Returns the ticket, or None if the request was rejected."""
        self._refs.append((off, idx))
        t = C.c_uint64()
        code = lib().rs_serve_submit(self._h, model, C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()),
                                     idx.numel(), raster_steps, n_steps, C.byref(t))
        if code == RS_ECAPACITY:
            return None
        _check(code)
        return t.value

    def step(self) -> int:
        n = C.c_uint32()
        _check(lib().rs_serve_step(self._h, C.byref(n)))
        return n.value

    def poll(self, max_results=4096):
        out = (_ServeResult * max_results)()
        sc = np.zeros((max_results, self.n_out_max), np.float64)
        n = C.c_uint32()
        _check(lib().rs_serve_poll(self._h, out, sc.ctypes.data_as(C.POINTER(C.c_double)), max_results,
                                   C.byref(n)))
        res = []
        for q in range(n.value):
            r = out[q]
            res.append(dict(ticket=r.ticket, model=r.model, steps=r.steps, decision=r.decision, spikes=r.spikes,
                            events=r.events, submit_s=r.submit_s, admit_s=r.admit_s, done_s=r.done_s,
                            scores=sc[q].copy()))
        return res

    def stats(self) -> dict:
        st = _ServeStats()
        _check(lib().rs_serve_stats_get(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServeStats._fields_}

    def replay(self, arrivals_s, models, n_steps, rasters):
        """rasters: list of (off, idx, raster_steps) device inputs, one per request.
        Returns latency_ms, decision, spikes arrays (latency -1 if rejected)."""
        n = len(arrivals_s)
        reqs = (_ServeRequest * n)()
        for q in range(n):
            off, idx, T = rasters[q]
            self._refs.append((off, idx))
            reqs[q] = _ServeRequest(float(arrivals_s[q]), int(models[q]), int(n_steps[q]), int(T), 0,
                                    C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()), idx.numel())
        lat = np.zeros(n, np.float64)
        dec = np.zeros(n, np.int32)
        spk = np.zeros(n, np.uint64)
        _check(lib().rs_serve_replay(self._h, reqs, n, lat.ctypes.data_as(C.POINTER(C.c_double)),
                                     dec.ctypes.data_as(C.POINTER(C.c_int32)),
                                     spk.ctypes.data_as(C.POINTER(C.c_uint64))))
        return lat, dec, spk


class _MultiSchedule(C.Structure):
    _fields_ = [("tuned", C.c_uint32), ("schedule", C.c_uint32), ("threads_per_row", C.c_uint32),
                ("rows_per_tile", C.c_uint32), ("workgroups", C.c_uint32), ("graph", C.c_uint32),
                ("trace_block", C.c_uint32), ("reserved", C.c_uint32), ("sample_ms", C.c_double * 8),
                ("samples", C.c_uint64)]


class MultiNet:
    """A set of e-prop networks of different sizes trained together (rs_multi_*)."""

    def __init__(self, cfgs, stream=None):
        self.cfgs = list(cfgs)
        arr = (_EpropParams * len(self.cfgs))(*[c.c() for c in self.cfgs])
        self._h = C.c_void_p()
        self._stream = _stream_ptr(stream)
        self._input_refs = [None] * len(self.cfgs)
        _check(lib().rs_multi_create(arr, len(self.cfgs), self._stream, C.byref(self._h)))
        self._infos = [None] * len(self.cfgs)
        for i in range(len(self.cfgs)):
            self.info(i)

    def close(self):
        if self._h:
            lib().rs_multi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.cfgs)

    def set_input(self, i, off, idx, labels):
        import torch
        for t in (off, idx, labels):
            assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()
        self._input_refs[i] = (off, idx, labels)
        _check(lib().rs_multi_set_input(self._h, i, C.c_void_p(off.data_ptr()), C.c_void_p(idx.data_ptr()),
                                        idx.numel(), C.c_void_p(labels.data_ptr())))

    def set_input_poisson(self, i, rates_hz, labels):
        import torch
        assert isinstance(labels, torch.Tensor) and labels.is_cuda and labels.dtype == torch.int32
        r = np.ascontiguousarray(rates_hz, np.float64)
        self._input_refs[i] = (labels,)
        _check(lib().rs_multi_set_input_poisson(self._h, i, r.ctypes.data_as(C.POINTER(C.c_double)), r.size,
                                                C.c_void_p(labels.data_ptr())))

    def train(self, n_samples: int = 1):
        _check(lib().rs_multi_train(self._h, n_samples))

    def schedule(self) -> dict:
        s = _MultiSchedule()
        _check(lib().rs_multi_schedule_get(self._h, C.byref(s)))
        return dict(tuned=bool(s.tuned), schedule=s.schedule, threads_per_row=s.threads_per_row,
                    rows_per_tile=s.rows_per_tile, workgroups=s.workgroups, graph=bool(s.graph),
                    trace_block=s.trace_block, sample_ms=list(s.sample_ms)[:5], samples=s.samples)

    def set_schedule(self, schedule: int, use_graph: bool = True):
        _check(lib().rs_multi_schedule_set(self._h, schedule, int(use_graph)))

    def get(self, i: int, var: int) -> np.ndarray:
        shape, dt = _shape_of(self.cfgs[i], self._infos[i], var)
        a = np.empty(shape, dt)
        _check(lib().rs_multi_get(self._h, i, var, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return a

    def set(self, i: int, var: int, value):
        shape, dt = _shape_of(self.cfgs[i], self._infos[i], var)
        a = np.ascontiguousarray(np.asarray(value, dtype=dt).reshape(shape))
        _check(lib().rs_multi_set(self._h, i, var, a.ctypes.data_as(C.c_void_p), a.nbytes))

    def info(self, i: int) -> _Info:
        inf = _Info()
        _check(lib().rs_multi_info_get(self._h, i, C.byref(inf)))
        self._infos[i] = inf
        return inf


@dataclass
class TopoConfig:
    L: int = 64
    cap: int = 32
    n_attempts: int = 160
    proj_id: int = 0
    p_form: float = 0.16
    sigma_form: float = 2.5
    g_theta: float = 0.1
    p_elim_dep: float = 2.45e-2 * 50
    p_elim_pot: float = 1.36e-4 * 50
    g_new: float = 0.2
    g_init: float = 0.2
    seed: int = 1

    def c(self) -> _TopoParams:
        p = _TopoParams()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


class TopoNet:
    """Topographic-map projection held on the GPU (rs_topo_*)."""

    def __init__(self, cfg: TopoConfig, stream=None):
        self.cfg = cfg
        self._h = C.c_void_p()
        _check(lib().rs_topo_create(C.byref(cfg.c()), _stream_ptr(stream), C.byref(self._h)))
        self.n = cfg.L * cfg.L
        self.words = (self.n + 31) // 32

    @classmethod
    def _view(cls, handle, cfg, owner):
        v = cls.__new__(cls)
        v.cfg, v._h, v._owner = cfg, handle, owner
        v.n = cfg.L * cfg.L
        v.words = (v.n + 31) // 32
        return v

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = C.c_void_p()
            return
        if self._h:
            lib().rs_topo_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rewire(self, step: int, stats: bool = True, lateral: bool = False):
        st = _Stats()
        fn = lib().rs_topo_lat_rewire if lateral else lib().rs_topo_rewire
        _check(fn(self._h, step, C.byref(st) if stats else None))
        return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts) if stats else None

    def add_lateral(self, cfg: "TopoConfig"):
        """Target -> target projection (rs_topo_add_lateral); before sim_init."""
        _check(lib().rs_topo_add_lateral(self._h, C.byref(cfg.c())))
        self.lat_cfg = cfg

    def sim_kernel(self, kind: int):
        _check(lib().rs_topo_sim_kernel(self._h, kind))

    def get_rows(self, lateral: bool = False):
        n, cap = self.n, (self.lat_cfg.cap if lateral else self.cfg.cap)
        ln = np.empty(n, np.int32)
        ind = np.empty((n, cap), np.int32)
        w = np.empty((n, cap), np.float32)
        fn = lib().rs_topo_lat_get_rows if lateral else lib().rs_topo_get_rows
        _check(fn(self._h, ln.ctypes.data_as(C.c_void_p), ind.ctypes.data_as(C.c_void_p),
                  w.ctypes.data_as(C.c_void_p)))
        return ln, ind, w

    def set_rows(self, ln, ind, w, lateral: bool = False):
        ln = np.ascontiguousarray(ln, np.int32)
        ind = np.ascontiguousarray(ind, np.int32)
        w = np.ascontiguousarray(w, np.float32)
        fn = lib().rs_topo_lat_set_rows if lateral else lib().rs_topo_set_rows
        _check(fn(self._h, ln.ctypes.data_as(C.c_void_p), ind.ctypes.data_as(C.c_void_p),
                  w.ctypes.data_as(C.c_void_p)))

    def custom_update(self, rule: int, step: int, host_fn=None) -> RewireStats:
        st = _Stats()
        cb = _host_fn(host_fn)
        _check(lib().rs_topo_custom_update(self._h, rule, step, cb, None, C.byref(st)))
        return _custom_stats(st)

    def get_bits(self, lateral: bool = False):
        b = np.empty((self.n, self.words), np.uint32)
        fn = lib().rs_topo_lat_get_bits if lateral else lib().rs_topo_get_bits
        _check(fn(self._h, b.ctypes.data_as(C.c_void_p)))
        return b

    def last_ms(self) -> float:
        ms = C.c_double()
        _check(lib().rs_topo_last_ms(self._h, C.byref(ms)))
        return ms.value


    # ---- simulation (rs_topo_sim_*): conductance LIF, STDP, Poisson stimulus
    def sim_init(self, model: "TopoModel"):
        _check(lib().rs_topo_sim_init(self._h, C.byref(model.c())))
        self.model = model

    def run(self, n_steps: int):
        _check(lib().rs_topo_run(self._h, n_steps))

    def run_stats(self, lateral: bool = False) -> RewireStats:
        st = _Stats()
        fn = lib().rs_topo_lat_run_stats if lateral else lib().rs_topo_run_stats
        _check(fn(self._h, C.byref(st)))
        return RewireStats(st.eliminated, st.formed, st.blocked, st.attempts)

    def sim_timing(self, on: bool):
        _check(lib().rs_topo_sim_timing(self._h, 1 if on else 0))

    def sim_phase_ms(self) -> dict:
        ms = (C.c_double * 4)()
        _check(lib().rs_topo_sim_phase_ms(self._h, ms))
        return dict(zip(TOPO_PHASES, ms))

    def _var(self, var: int):
        if var == TV_STEP:
            return np.empty(1, np.uint64)
        if var in (TV_ZIN, TV_ZOUT):
            return np.empty(self.words, np.uint32)
        if var == TV_REF:
            return np.empty(self.n, np.int32)
        if var == TV_COUNT:
            return np.empty(self.n, np.uint32)
        return np.empty(self.n, np.float32)

    def sim_get(self, var: int) -> np.ndarray:
        a = self._var(var)
        _check(lib().rs_topo_sim_get(self._h, var, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return a

    def sim_set(self, var: int, value):
        a = self._var(var)
        a[...] = np.asarray(value).reshape(a.shape)
        _check(lib().rs_topo_sim_set(self._h, var, a.ctypes.data_as(C.c_void_p), a.nbytes))


STIM_BLOB, STIM_BAR = 0, 1
TOPO_PHASES = ("delivery_and_source", "neurons", "potentiation", "launch_prologue")
TV_V, TV_G, TV_Y, TV_X, TV_REF, TV_COUNT, TV_ZIN, TV_ZOUT, TV_STEP, TV_XLAT = range(10)
TOPO_KERNEL_AUTO, TOPO_KERNEL_ONE_WG, TOPO_KERNEL_TILED = 0, 1, 2


@dataclass
class TopoModel:
    """Topographic-map model (Tab. D-H), GeNN units: ms, mV, nF, uS, Hz."""
    h: float = 0.1
    C_m: float = 20.0
    tau_m: float = 20.0
    V_rest: float = -70.0
    E_exc: float = 0.0
    V_th: float = -54.0
    V_reset: float = -70.0
    tau_s: float = 5.0
    ref_steps: int = 50
    f_base: float = 5.0
    f_peak: float = 152.8
    sigma_stim: float = 2.0
    stim_steps: int = 200
    stim_kind: int = STIM_BLOB
    stdp: int = 1
    g_max: float = 0.2
    A_plus: float = 0.1 * 0.2
    A_minus: float = 1.2 * 0.1 * 0.2 * 20.0 / 64.0
    tau_plus: float = 20.0
    tau_minus: float = 64.0
    rewire_steps: int = 10
    stim_tile: int = 0  # side of the square the input is replicated over (scaled maps); 0: whole sheet

    def c(self) -> _TopoModel:
        m = _TopoModel()
        for f in fields(self):
            setattr(m, f.name, getattr(self, f.name))
        return m


def calib_copy(dst, src, nbytes: int, stream=None):
    _check(lib().rs_calib_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, _stream_ptr(stream)))
