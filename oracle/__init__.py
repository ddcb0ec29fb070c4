"""Reference CPU oracle for ragged-row SNN simulation, e-prop, DEEP R and
topographic-map rewiring.

TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded fp64 C implementation
of the paper's method (Knight, Senk, Nowotny et al., arXiv 2510.19764), wrapped
with ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  It shares no code with the HIP library in
``paper_2510_19764_amd``.

Per-function citations live in the C sources:
  philox.c   counter-based generator (Salmon et al. SC'11)
  build.c    fixed-probability / pairwise-Bernoulli rows, DEEP R bitfield init
  eprop.c    ALIF/LIF step, leaky readout, e-prop eligibility and gradients
  update.c   L1 term for DEEP R projections + Adam
  deepr.c    DEEP R elimination and formation
  topomap.c  topographic-map rewiring
  topo_sim.c topographic-map simulation: conductance LIF, STDP, stimulus
  input.c    Poisson input spikes on the counter-based generator
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = ["philox.c", "build.c", "eprop.c", "update.c", "deepr.c", "topomap.c", "input.c", "topo_sim.c", "custom.c"]
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

TAG_CONN, TAG_WINIT, TAG_SIGN = 1, 2, 3
TAG_DR_ROW, TAG_DR_TGT = 4, 5
TAG_TP_ROW, TAG_TP_TGT, TAG_TP_ELIM, TAG_TP_FORM = 6, 7, 8, 9
TAG_INPUT = 10
TAG_CUSTOM = 13
MAX_TRIES = 64


_OMP_LIB_PATH = os.path.join(_HERE, "_build", "liboracle_omp.so")


def build(force: bool = True, omp: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so (the
    single-threaded parity build), or with omp into liboracle_omp.so (the
    multi-core timing build: the same sources with OpenMP enabled)."""
    path = _OMP_LIB_PATH if omp else _LIB_PATH
    if not force and os.path.exists(path):
        return path
    os.makedirs(os.path.dirname(path), exist_ok=True)
    srcs = [os.path.join(_HERE, s) for s in _SRCS]
    tmp = path + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-ffp-contract=off"] + (["-fopenmp"] if omp else ["-Wno-unknown-pragmas"]) + \
        ["-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    return path


_lib = None
_omp_lib = None


def _load(path, omp):
    newest_src = max(os.path.getmtime(os.path.join(_HERE, s)) for s in _SRCS + ["oracle.h"])
    if not os.path.exists(path) or os.path.getmtime(path) < newest_src:
        build(omp=omp)
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _load(_LIB_PATH, False)
    return _lib


def use_multicore(on: bool = True) -> int:
    """Route the calls below to the multi-core timing build (on) or back to
    the parity build; returns the threads the build runs on."""
    global _lib, _omp_lib
    if on:
        if _omp_lib is None:
            _omp_lib = _load(_OMP_LIB_PATH, True)
        _lib = _omp_lib
    else:
        _lib = None
    return int(lib().orc_threads())


P_i32 = C.POINTER(C.c_int32)
P_u32 = C.POINTER(C.c_uint32)
P_u8 = C.POINTER(C.c_uint8)
P_f64 = C.POINTER(C.c_double)
P_u64 = C.POINTER(C.c_uint64)


class _CProj(C.Structure):
    _fields_ = [("n_pre", C.c_int32), ("n_post", C.c_int32), ("cap", C.c_int32),
                ("recurrent", C.c_int32), ("proj_id", C.c_int32),
                ("len", P_i32), ("ind", P_i32),
                ("w", P_f64), ("m", P_f64), ("v", P_f64), ("G", P_f64),
                ("eps", P_f64), ("ebar", P_f64),
                ("conn", P_u32), ("sign", P_u32), ("words", C.c_int32), ("Gabs", P_f64)]


class _CNet(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_rec", C.c_int32), ("n_out", C.c_int32),
                ("batch", C.c_int32), ("alif", C.c_int32),
                ("alpha", C.c_double), ("rho", C.c_double), ("v_thr", C.c_double),
                ("beta", C.c_double), ("alpha_trace", C.c_double),
                ("inp", C.POINTER(_CProj)), ("rec", C.POINTER(_CProj)),
                ("v", P_f64), ("a", P_f64), ("y", P_f64), ("xbar", P_f64), ("zbar", P_f64),
                ("Wout", P_f64), ("bout", P_f64), ("Gout", P_f64), ("Gb", P_f64),
                ("Mout", P_f64), ("Vout", P_f64), ("Mb", P_f64), ("Vb", P_f64),
                ("psi", P_f64), ("L", P_f64), ("z", P_u8), ("delta", P_f64),
                ("Labs", P_f64), ("Goutabs", P_f64), ("Gbabs", P_f64)]


class _CTopoParams(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_attempts", C.c_int32),
                ("p_form", C.c_double), ("sigma_form", C.c_double), ("g_theta", C.c_double),
                ("p_elim_dep", C.c_double), ("p_elim_pot", C.c_double), ("g_new", C.c_double)]


class _CTopoModel(C.Structure):
    _fields_ = [("L", C.c_int32), ("h", C.c_double),
                ("C_m", C.c_double), ("tau_m", C.c_double), ("V_rest", C.c_double),
                ("E_exc", C.c_double), ("V_th", C.c_double), ("V_reset", C.c_double),
                ("tau_s", C.c_double), ("ref_steps", C.c_int32),
                ("f_base", C.c_double), ("f_peak", C.c_double), ("sigma_stim", C.c_double),
                ("stim_steps", C.c_int32), ("stim_kind", C.c_int32), ("stdp", C.c_int32),
                ("g_max", C.c_double), ("A_plus", C.c_double), ("A_minus", C.c_double),
                ("tau_plus", C.c_double), ("tau_minus", C.c_double), ("rewire_steps", C.c_int32),
                ("stim_tile", C.c_int32)]


class _CTopoState(C.Structure):
    _fields_ = [("V", P_f64), ("g", P_f64), ("y", P_f64), ("ref", P_i32), ("count", P_i32),
                ("zout", P_u8), ("x", P_f64), ("zin", P_u8), ("xl", P_f64)]


_ROW_FN = C.CFUNCTYPE(C.c_uint32, C.c_void_p, C.c_int32)
_TGT_FN = C.CFUNCTYPE(C.c_uint32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32)
_RS_FN = C.CFUNCTYPE(C.c_uint32, C.c_void_p, C.c_int32, C.c_int32)


class _CTopoDraws(C.Structure):
    _fields_ = [("attempt_row", _ROW_FN), ("target", _TGT_FN), ("elim_u32", _RS_FN),
                ("form_u32", _RS_FN), ("ctx", C.c_void_p)]


def _declare(L):
    L.orc_threads.restype = C.c_int32
    L.orc_philox4x64_10.argtypes = [C.c_uint64, C.c_uint64, P_u64, P_u64]
    L.orc_u32.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32] + [C.c_uint64] * 4
    L.orc_u32.restype = C.c_uint32
    L.orc_below.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_below.restype = C.c_uint32
    L.orc_threshold.argtypes = [C.c_double]
    L.orc_threshold.restype = C.c_uint64
    L.orc_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32] + [C.c_uint64] * 4
    L.orc_normal.restype = C.c_double
    L.orc_rate_threshold.argtypes = [C.c_double, C.c_double]
    L.orc_rate_threshold.restype = C.c_uint64
    L.orc_poisson_input.argtypes = [C.c_uint64, C.c_uint64, C.c_int32, C.c_int32, P_u64, C.c_int32,
                                    P_i32, P_i32]
    L.orc_poisson_input.restype = C.c_int64
    L.orc_fixed_prob_rows.argtypes = [C.c_uint64, C.POINTER(_CProj), C.c_double, C.c_double]
    L.orc_fixed_prob_rows.restype = C.c_int32
    L.orc_gauss_rows.argtypes = [C.c_uint64, C.POINTER(_CProj), C.c_int32, C.c_double,
                                 C.c_double, C.c_double]
    L.orc_gauss_rows.restype = C.c_int32
    L.orc_dense_init.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, P_f64]
    L.orc_deepr_init_bits.argtypes = [C.c_uint64, C.POINTER(_CProj)]
    L.orc_eprop_step.argtypes = [C.POINTER(_CNet), P_i32, P_i32, P_i32, P_u8, C.c_int32]
    L.orc_eprop_spikes.argtypes = [C.POINTER(_CNet), P_u8, P_f64]
    L.orc_eprop_reset.argtypes = [C.POINTER(_CNet)]
    L.orc_adam_update.argtypes = [C.POINTER(_CNet), C.c_int32, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_int32]
    L.orc_deepr_rewire.argtypes = [C.c_uint64, C.POINTER(_CProj), C.c_int32, C.c_uint64,
                                   P_i32, P_i32]
    L.orc_topo_rewire_with.argtypes = [C.POINTER(_CProj), C.POINTER(_CTopoParams),
                                       C.POINTER(_CTopoDraws), P_u32, P_i32]
    L.orc_topo_rewire.argtypes = [C.c_uint64, C.POINTER(_CProj), C.POINTER(_CTopoParams),
                                  C.c_uint64, P_u32, P_i32]
    L.orc_torus_d2.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.orc_topo_stimulus.argtypes = [C.c_uint64, C.POINTER(_CTopoModel), C.c_uint64, P_i32, P_i32, P_i32]
    L.orc_topo_stim_d2.argtypes = [C.POINTER(_CTopoModel), C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.orc_topo_stim_d2.restype = C.c_int32
    L.orc_topo_input_u32.argtypes = [C.c_uint64, C.c_uint64, C.c_int32]
    L.orc_topo_input_u32.restype = C.c_uint32
    L.orc_topo_rate.argtypes = [C.POINTER(_CTopoModel), C.c_int32]
    L.orc_topo_rate.restype = C.c_double
    L.orc_topo_sim_step.argtypes = [C.c_uint64, C.POINTER(_CTopoModel), C.POINTER(_CProj),
                                    C.POINTER(_CTopoState), C.c_uint64]
    L.orc_topo_sim_step_lat.argtypes = [C.c_uint64, C.POINTER(_CTopoModel), C.POINTER(_CProj),
                                        C.POINTER(_CProj), C.POINTER(_CTopoState), C.c_uint64]
    L.orc_topo_run_lat.argtypes = [C.c_uint64, C.POINTER(_CTopoModel), C.POINTER(_CProj),
                                   C.POINTER(_CTopoParams), C.POINTER(_CProj), C.POINTER(_CTopoParams),
                                   C.POINTER(_CTopoState), C.c_uint64, C.c_uint64, P_u32, P_u32, P_i32, P_i32]
    L.orc_topo_run.argtypes = [C.c_uint64, C.POINTER(_CTopoModel), C.POINTER(_CProj),
                               C.POINTER(_CTopoParams), C.POINTER(_CTopoState), C.c_uint64,
                               C.c_uint64, P_u32, P_i32]
    L.orc_torus_d2.restype = C.c_int32
    L.orc_add_diagonal.argtypes = [C.POINTER(_CProj), C.c_int32]
    L.orc_add_diagonal.restype = C.c_int32
    L.orc_remove_random_targets.argtypes = [C.c_uint64, C.POINTER(_CProj), C.c_uint64, P_u32]
    L.orc_remove_targets.argtypes = [C.POINTER(_CProj), C.c_int32, P_u32]
    L.orc_remove_targets.restype = C.c_int32


def _ptr(a, t):
    if a is None:
        return C.cast(None, t)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------- generator
def philox4x64_10(key0: int, key1: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(C.c_uint64(key0), C.c_uint64(key1), _ptr(c, P_u64), _ptr(out, P_u64))
    return out


def u32(seed, tag, proj, c0, c1, c2, c3=0) -> int:
    return int(lib().orc_u32(seed, tag, proj, c0, c1, c2, c3))


def below(u: int, n: int) -> int:
    return int(lib().orc_below(u, n))


def threshold(p: float) -> int:
    return int(lib().orc_threshold(p))


def rate_thresholds(rates_hz, dt_ms: float = 1.0) -> np.ndarray:
    """Per-step Bernoulli thresholds floor(rate*dt*2^32) of Poisson channels."""
    r = np.ascontiguousarray(rates_hz, np.float64)
    return np.array([lib().orc_rate_threshold(float(x), float(dt_ms)) for x in r.ravel()],
                    np.uint64).reshape(r.shape)


def poisson_input(seed: int, step: int, B: int, thr: np.ndarray):
    """Input spike lists (idx, off[B+1]) of one step; thr is [n_in] (shared by
    the instances) or [B][n_in]."""
    thr = np.ascontiguousarray(thr, np.uint64)
    n_in = thr.shape[-1]
    per_instance = 1 if thr.ndim == 2 else 0
    assert not per_instance or thr.shape[0] == B
    idx = np.zeros(max(B * n_in, 1), np.int32)
    off = np.zeros(B + 1, np.int32)
    n = lib().orc_poisson_input(seed, step, B, n_in, _ptr(thr, P_u64), per_instance,
                                _ptr(idx, P_i32), _ptr(off, P_i32))
    return idx[:n].copy(), off


def normal(seed, tag, proj, c0, c1, c2, c3=0) -> float:
    return float(lib().orc_normal(seed, tag, proj, c0, c1, c2, c3))


def torus_d2(L: int, i: int, j: int) -> int:
    return int(lib().orc_torus_d2(L, i, j))


# ---------------------------------------------------------------- projections
@dataclass
class Proj:
    n_pre: int
    n_post: int
    cap: int
    recurrent: bool
    proj_id: int
    batch: int = 1
    trained: bool = False
    traces: str = "none"  # "none" | "lif" | "alif"
    bitfields: bool = False
    # error-bound bookkeeping for tests: Gabs accumulates sum |L ebar| beside G
    abs_sums: bool = False
    len: np.ndarray = field(init=False)
    ind: np.ndarray = field(init=False)
    w: np.ndarray = field(init=False)
    m: np.ndarray | None = field(init=False, default=None)
    v: np.ndarray | None = field(init=False, default=None)
    G: np.ndarray | None = field(init=False, default=None)
    eps: np.ndarray | None = field(init=False, default=None)
    ebar: np.ndarray | None = field(init=False, default=None)
    conn: np.ndarray | None = field(init=False, default=None)
    sign: np.ndarray | None = field(init=False, default=None)
    Gabs: np.ndarray | None = field(init=False, default=None)

    def __post_init__(self):
        n = self.n_pre * max(self.cap, 1)
        self.words = (self.n_post + 31) // 32
        self.len = np.zeros(self.n_pre, np.int32)
        self.ind = np.zeros(n, np.int32)
        self.w = np.zeros(n, np.float64)
        if self.trained:
            self.m = np.zeros(n)
            self.v = np.zeros(n)
            self.G = np.zeros(n)
            if self.abs_sums:
                self.Gabs = np.zeros(n)
        if self.traces != "none":
            self.ebar = np.zeros(n * self.batch)
            if self.traces == "alif":
                self.eps = np.zeros(n * self.batch)
        if self.bitfields:
            self.conn = np.zeros(self.n_pre * self.words, np.uint32)
            self.sign = np.zeros(self.n_pre * self.words, np.uint32)

    def c(self, rows_only: bool = False) -> _CProj:
        s = _CProj()
        s.n_pre, s.n_post, s.cap = self.n_pre, self.n_post, self.cap
        s.recurrent, s.proj_id, s.words = int(self.recurrent), self.proj_id, self.words
        s.len = _ptr(self.len, P_i32)
        s.ind = _ptr(None if rows_only else self.ind, P_i32)
        s.w = _ptr(None if rows_only else self.w, P_f64)
        s.m, s.v, s.G = _ptr(self.m, P_f64), _ptr(self.v, P_f64), _ptr(self.G, P_f64)
        s.eps, s.ebar = _ptr(self.eps, P_f64), _ptr(self.ebar, P_f64)
        s.conn, s.sign = _ptr(self.conn, P_u32), _ptr(self.sign, P_u32)
        s.Gabs = _ptr(self.Gabs, P_f64)
        self._c = s  # keep alive
        return s

    # convenience views
    def rows(self):
        """List of (targets, weights) per row, in slot order."""
        out = []
        for i in range(self.n_pre):
            n = int(self.len[i])
            out.append((self.ind[i * self.cap:i * self.cap + n].copy(),
                        self.w[i * self.cap:i * self.cap + n].copy()))
        return out

    def slot_view(self, a: np.ndarray, width: int = 1):
        return a.reshape(self.n_pre, self.cap, width) if width > 1 else a.reshape(self.n_pre, self.cap)


def fixed_prob_count(seed: int, n_pre: int, n_post: int, p: float, recurrent: bool, proj_id: int):
    P = Proj(n_pre, n_post, 0, recurrent, proj_id)
    mx = lib().orc_fixed_prob_rows(seed, C.byref(P.c(rows_only=True)), p, 1.0)
    return P.len.copy(), int(mx)


def fixed_prob_rows(seed: int, P: Proj, p: float, sigma: float) -> int:
    return int(lib().orc_fixed_prob_rows(seed, C.byref(P.c()), p, sigma))


def gauss_count(seed: int, L: int, p_form: float, sigma: float, proj_id: int):
    P = Proj(L * L, L * L, 0, False, proj_id)
    mx = lib().orc_gauss_rows(seed, C.byref(P.c(rows_only=True)), L, p_form, sigma, 0.0)
    return P.len.copy(), int(mx)


def gauss_rows(seed: int, P: Proj, L: int, p_form: float, sigma: float, g_init: float) -> int:
    return int(lib().orc_gauss_rows(seed, C.byref(P.c()), L, p_form, sigma, g_init))


def dense_init(seed: int, proj_id: int, rows: int, cols: int, sigma: float) -> np.ndarray:
    W = np.zeros(rows * cols)
    lib().orc_dense_init(seed, proj_id, rows, cols, sigma, _ptr(W, P_f64))
    return W.reshape(rows, cols)


def deepr_init_bits(seed: int, P: Proj):
    lib().orc_deepr_init_bits(seed, C.byref(P.c()))


def deepr_rewire(seed: int, P: Proj, step: int):
    dormant = np.zeros(P.n_pre, np.int32)
    stats = np.zeros(2, np.int32)
    lib().orc_deepr_rewire(seed, C.byref(P.c()), P.batch, step, _ptr(dormant, P_i32), _ptr(stats, P_i32))
    return dormant, stats


def add_diagonal(P: Proj) -> int:
    """The paper's add_diagonal example (custom connectivity update)."""
    return int(lib().orc_add_diagonal(C.byref(P.c()), P.batch))


def remove_random_targets(seed: int, P: Proj, step: int) -> np.ndarray:
    """Host part of the paper's remove_random example: one target per row."""
    out = np.zeros(P.n_pre, np.uint32)
    lib().orc_remove_random_targets(seed, C.byref(P.c()), step, _ptr(out, P_u32))
    return out


def remove_targets(P: Proj, post_ind) -> int:
    """Row part of remove_random: remove each row's first synapse onto post_ind[row]."""
    a = np.ascontiguousarray(post_ind, np.uint32)
    return int(lib().orc_remove_targets(C.byref(P.c()), P.batch, _ptr(a, P_u32)))


# ---------------------------------------------------------------- e-prop network
@dataclass
class EpropParams:
    n_in: int
    n_rec: int
    n_out: int
    batch: int
    alif: bool
    dt_ms: float = 1.0
    tau_mem_ms: float = 20.0
    tau_adapt_ms: float = 2000.0
    v_thr: float = 0.6
    beta: float = 0.0174
    # explicit decay factors; None derives them from dt and the time constants
    alpha_value: float | None = None
    rho_value: float | None = None
    # decay of the presynaptic traces; None uses alpha
    alpha_trace_value: float | None = None

    @property
    def alpha(self):
        if self.alpha_value is not None:
            return float(self.alpha_value)
        return float(np.exp(-self.dt_ms / self.tau_mem_ms))

    @property
    def alpha_trace(self):
        if self.alpha_trace_value is not None:
            return float(self.alpha_trace_value)
        return self.alpha

    @property
    def rho(self):
        if not self.alif:
            return 0.0
        if self.rho_value is not None:
            return float(self.rho_value)
        return float(np.exp(-self.dt_ms / self.tau_adapt_ms))

    @property
    def beta_eff(self):
        return self.beta if self.alif else 0.0


class Net:
    """fp64 e-prop network state; arrays are numpy views the C code updates in place.
    With abs_sums, Labs / Goutabs / Gbabs hold the magnitude sums of the terms of
    L, Gout and Gb (error-bound bookkeeping for tests)."""

    def __init__(self, prm: EpropParams, inp: Proj, rec: Proj, abs_sums: bool = False):
        self.prm = prm
        B, NR, NI, K = prm.batch, prm.n_rec, prm.n_in, prm.n_out
        self.inp, self.rec = inp, rec
        self.v = np.zeros((B, NR))
        self.a = np.zeros((B, NR))
        self.y = np.zeros((B, K))
        self.xbar = np.zeros((B, NI))
        self.zbar = np.zeros((B, NR))
        self.Wout = np.zeros((K, NR))
        self.bout = np.zeros(K)
        self.Gout = np.zeros((K, NR))
        self.Gb = np.zeros(K)
        self.Mout = np.zeros((K, NR))
        self.Vout = np.zeros((K, NR))
        self.Mb = np.zeros(K)
        self.Vb = np.zeros(K)
        self.psi = np.zeros((B, NR))
        self.L = np.zeros((B, NR))
        self.z = np.zeros((B, NR), np.uint8)
        self.delta = np.zeros((B, K))
        self.Labs = np.zeros((B, NR)) if abs_sums else None
        self.Goutabs = np.zeros((K, NR)) if abs_sums else None
        self.Gbabs = np.zeros(K) if abs_sums else None

    def c(self) -> _CNet:
        p = self.prm
        s = _CNet()
        s.n_in, s.n_rec, s.n_out, s.batch, s.alif = p.n_in, p.n_rec, p.n_out, p.batch, int(p.alif)
        s.alpha, s.rho, s.v_thr, s.beta = p.alpha, p.rho, p.v_thr, p.beta_eff
        s.alpha_trace = p.alpha_trace
        self._ci, self._cr = self.inp.c(), self.rec.c()
        s.inp, s.rec = C.pointer(self._ci), C.pointer(self._cr)
        for name in ["v", "a", "y", "xbar", "zbar", "Wout", "bout", "Gout", "Gb",
                     "Mout", "Vout", "Mb", "Vb", "psi", "L", "delta"]:
            setattr(s, name, _ptr(getattr(self, name), P_f64))
        s.z = _ptr(self.z, P_u8)
        s.Labs, s.Goutabs, s.Gbabs = (_ptr(self.Labs, P_f64), _ptr(self.Goutabs, P_f64),
                                      _ptr(self.Gbabs, P_f64))
        self._c = s
        return s

    def step(self, x_idx, x_off, labels, z_force=None, learn=True):
        x_idx = np.ascontiguousarray(x_idx, np.int32)
        if x_idx.size == 0:
            x_idx = np.zeros(1, np.int32)
        x_off = np.ascontiguousarray(x_off, np.int32)
        labels = np.ascontiguousarray(labels, np.int32)
        zf = None if z_force is None else np.ascontiguousarray(z_force, np.uint8)
        lib().orc_eprop_step(C.byref(self.c()), _ptr(x_idx, P_i32), _ptr(x_off, P_i32),
                             _ptr(labels, P_i32), _ptr(zf, P_u8), int(learn))

    def spikes(self):
        z = np.zeros(self.v.shape, np.uint8)
        margin = np.zeros(self.v.shape)
        lib().orc_eprop_spikes(C.byref(self.c()), _ptr(z, P_u8), _ptr(margin, P_f64))
        return z, margin

    def reset(self):
        lib().orc_eprop_reset(C.byref(self.c()))

    def adam_update(self, k, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, l1=0.0, deepr_mask=0):
        lib().orc_adam_update(C.byref(self.c()), k, lr, b1, b2, eps, l1, deepr_mask)


# ---------------------------------------------------------------- topographic map
@dataclass
class TopoParams:
    L: int
    n_attempts: int
    p_form: float
    sigma_form: float
    g_theta: float
    p_elim_dep: float
    p_elim_pot: float
    g_new: float

    def c(self):
        return _CTopoParams(self.L, self.n_attempts, self.p_form, self.sigma_form, self.g_theta,
                            self.p_elim_dep, self.p_elim_pot, self.g_new)


def topo_rewire(seed: int, P: Proj, tp: TopoParams, step: int, bits: np.ndarray | None = None):
    if bits is None:
        bits = np.zeros(P.n_pre * P.words, np.uint32)
    stats = np.zeros(4, np.int32)
    ctp = tp.c()
    lib().orc_topo_rewire(seed, C.byref(P.c()), C.byref(ctp), step, _ptr(bits, P_u32), _ptr(stats, P_i32))
    return stats, bits


def topo_rewire_scripted(P: Proj, tp: TopoParams, attempt_row, target, elim_u32, form_u32,
                         bits: np.ndarray | None = None):
    """Topomap rewiring with every random outcome supplied by Python callables."""
    if bits is None:
        bits = np.zeros(P.n_pre * P.words, np.uint32)
    stats = np.zeros(4, np.int32)
    fns = (_ROW_FN(lambda _c, a: attempt_row(a)),
           _TGT_FN(lambda _c, r, q, t: target(r, q, t)),
           _RS_FN(lambda _c, r, s: elim_u32(r, s)),
           _RS_FN(lambda _c, r, j: form_u32(r, j)))
    d = _CTopoDraws(fns[0], fns[1], fns[2], fns[3], None)
    ctp = tp.c()
    lib().orc_topo_rewire_with(C.byref(P.c()), C.byref(ctp), C.byref(d), _ptr(bits, P_u32), _ptr(stats, P_i32))
    return stats, bits


# ---------------------------------------------------------------- topographic-map simulation
STIM_BLOB, STIM_BAR = 0, 1


@dataclass
class TopoModel:
    """Topographic-map model parameters (Tab. D, E, F, G, H), GeNN units: ms, mV, nF, uS, Hz."""
    L: int
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
    A_plus: float = 0.02
    A_minus: float = 0.2 * 0.1 * 1.2 * 20.0 / 64.0
    tau_plus: float = 20.0
    tau_minus: float = 64.0
    rewire_steps: int = 10
    stim_tile: int = 0  # side of the square the stimulus is replicated over (scaled maps); 0: L

    def c(self):
        return _CTopoModel(*[getattr(self, f) for f, _ in _CTopoModel._fields_])


class TopoState:
    """Both sheets' state; V starts at V_rest, everything else at zero."""

    def __init__(self, M: TopoModel):
        N = M.L * M.L
        self.V = np.full(N, M.V_rest, np.float64)
        self.g = np.zeros(N, np.float64)
        self.y = np.zeros(N, np.float64)
        self.ref = np.zeros(N, np.int32)
        self.count = np.zeros(N, np.int32)
        self.zout = np.zeros(N, np.uint8)
        self.x = np.zeros(N, np.float64)
        self.zin = np.zeros(N, np.uint8)
        self.xl = np.zeros(N, np.float64)  # lateral pre trace of the targets

    def c(self):
        return _CTopoState(_ptr(self.V, P_f64), _ptr(self.g, P_f64), _ptr(self.y, P_f64),
                           _ptr(self.ref, P_i32), _ptr(self.count, P_i32), _ptr(self.zout, P_u8),
                           _ptr(self.x, P_f64), _ptr(self.zin, P_u8), _ptr(self.xl, P_f64))


def topo_stimulus(seed: int, M: TopoModel, step: int):
    cx, cy, o = C.c_int32(), C.c_int32(), C.c_int32()
    lib().orc_topo_stimulus(seed, C.byref(M.c()), step, C.byref(cx), C.byref(cy), C.byref(o))
    return cx.value, cy.value, o.value


def topo_stim_d2(M: TopoModel, i: int, cx: int, cy: int, orient: int) -> int:
    return lib().orc_topo_stim_d2(C.byref(M.c()), i, cx, cy, orient)


def topo_input_u32(seed: int, t: int, i: int) -> int:
    return lib().orc_topo_input_u32(seed, t, i)


def topo_rate(M: TopoModel, d2: int) -> float:
    return lib().orc_topo_rate(C.byref(M.c()), d2)


def topo_sim_step(seed: int, M: TopoModel, P: Proj, S: TopoState, t: int, PL: Proj | None = None):
    """One step; PL is the lateral (target -> target) projection or None."""
    cm, cs = M.c(), S.c()
    if PL is None:
        lib().orc_topo_sim_step(seed, C.byref(cm), C.byref(P.c()), C.byref(cs), t)
    else:
        lib().orc_topo_sim_step_lat(seed, C.byref(cm), C.byref(P.c()), C.byref(PL.c()), C.byref(cs), t)


def topo_run(seed: int, M: TopoModel, P: Proj, tp: TopoParams, S: TopoState, t0: int, n: int,
             bits: np.ndarray | None = None, PL: Proj | None = None, tpl: TopoParams | None = None,
             bits_l: np.ndarray | None = None):
    """Steps t0 .. t0+n-1 with a rewire after every rewire_steps; returns summed rewire stats
    (a pair, feed-forward and lateral, when PL is given)."""
    if bits is None:
        bits = np.zeros(P.n_pre * P.words, np.uint32)
    stats = np.zeros(4, np.int32)
    cm, cs, ctp = M.c(), S.c(), tp.c()
    if PL is None:
        lib().orc_topo_run(seed, C.byref(cm), C.byref(P.c()), C.byref(ctp), C.byref(cs), t0, n,
                           _ptr(bits, P_u32), _ptr(stats, P_i32))
        return stats
    if bits_l is None:
        bits_l = np.zeros(PL.n_pre * PL.words, np.uint32)
    stats_l = np.zeros(4, np.int32)
    ctpl = tpl.c()
    lib().orc_topo_run_lat(seed, C.byref(cm), C.byref(P.c()), C.byref(ctp), C.byref(PL.c()), C.byref(ctpl),
                           C.byref(cs), t0, n, _ptr(bits, P_u32), _ptr(bits_l, P_u32), _ptr(stats, P_i32),
                           _ptr(stats_l, P_i32))
    return stats, stats_l
