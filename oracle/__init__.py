"""RACIPE CPU oracle -- test infrastructure only.

A ctypes wrapper around ``liboracle.so`` (plain FP64 C, see ``oracle.c``).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU library never does.

Functions follow the GRiNS paper (arXiv 2503.18356): Eq. 1-2 for the RHS,
Table 1 and Sec. 2.1.2 for sampling, Sec. 2.1.3 for the simulation controls.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CONVERGED, T_END, MAX_STEPS, STEP_UNDERFLOW, NONFINITE = range(5)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (portable x86-64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Ranges(C.Structure):
    _fields_ = [("g_min", C.c_double), ("g_max", C.c_double), ("k_min", C.c_double),
                ("k_max", C.c_double), ("lam_act_min", C.c_double), ("lam_act_max", C.c_double),
                ("lam_inh_min", C.c_double), ("lam_inh_max", C.c_double),
                ("n_min", C.c_int32), ("n_max", C.c_int32), ("t_lo", C.c_double),
                ("t_hi", C.c_double), ("t_median", C.c_double), ("method", C.c_int32),
                ("threshold_rule", C.c_int32), ("hf_samples", C.c_int32),
                ("hf_act_over_lambda", C.c_int32), ("lhs_total", C.c_int64),
                ("n_continuous", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("t0", C.c_double), ("t_end", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("ss_atol", C.c_double), ("ss_rtol", C.c_double),
                ("h0", C.c_double), ("max_steps", C.c_int64),
                ("divide_act_by_lambda", C.c_int32), ("stop_at_steady", C.c_int32),
                ("ic_absolute", C.c_int32), ("method", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("n_genes", C.c_int32), ("n_edges", C.c_int32),
                ("src", C.c_void_p), ("dst", C.c_void_p), ("sign", C.c_void_p),
                ("G", C.c_void_p), ("k", C.c_void_p), ("T", C.c_void_p), ("lam", C.c_void_p),
                ("n", C.c_void_p), ("n_sets", C.c_int64), ("ic", C.c_void_p), ("n_ic", C.c_int32),
                ("nf", C.c_void_p)]


_lib = None


def load(path: str):
    """Load and type an oracle shared library from ``path``."""
    L = C.CDLL(path)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    L.orc_philox4x64_10.argtypes = [vp, vp, vp]
    L.orc_canonicalize.argtypes = [C.c_int, C.c_int, vp, vp, vp, vp, vp, vp]
    L.orc_canonicalize.restype = C.c_int
    L.orc_default_ranges.argtypes = [C.POINTER(_Ranges)]
    L.orc_gk_median.argtypes = [C.POINTER(_Ranges)]
    L.orc_gk_median.restype = C.c_double
    L.orc_sample.argtypes = [C.c_int, C.c_int, vp, vp, vp, C.POINTER(_Ranges), u64, i64, i64, i32,
                             vp, vp, vp, vp, vp, vp, vp]
    L.orc_sample.restype = C.c_int
    L.orc_hf_median.argtypes = [C.POINTER(_Ranges), i32, i32]
    L.orc_hf_median.restype = C.c_double
    L.orc_sobol_u32.argtypes = [i64, i32, C.POINTER(C.c_uint32)]
    L.orc_sobol_u32.restype = C.c_int
    L.orc_primitive_count.argtypes = [i32]
    L.orc_primitive_count.restype = C.c_int
    L.orc_lhs_perm.argtypes = [u64, i32, i32, i64, i64]
    L.orc_lhs_perm.restype = i64
    L.orc_default_opts.argtypes = [C.POINTER(_Opts)]
    L.orc_rhs.argtypes = [C.POINTER(_Problem), i64, i32, vp, vp]
    L.orc_steady_states.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), vp, i64, i32,
                                    vp, vp, vp, vp, vp]
    L.orc_steady_states.restype = C.c_int
    L.orc_time_series.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), vp, i32, vp, i64,
                                  i32, vp, vp, vp, vp, vp]
    L.orc_time_series.restype = C.c_int
    L.orc_rk4.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_double, vp, i32, vp,
                          i64, i32, vp]
    L.orc_rk4.restype = C.c_int
    L.orc_dp5_fixed.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), i64, i64, vp, vp]
    L.orc_dp5_fixed.restype = C.c_int
    L.orc_tableau.argtypes = [i32, vp, vp, vp, vp]
    L.orc_tableau.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = load(_LIB_PATH)
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


@dataclass
class Network:
    """Canonical (dst, src)-sorted signed edge list."""
    n_genes: int
    src: np.ndarray
    dst: np.ndarray
    sign: np.ndarray

    @property
    def n_edges(self) -> int:
        return int(self.src.size)


def canonicalize(n_genes: int, src, dst, sign) -> Network:
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    g = np.ascontiguousarray(sign, dtype=np.int8)
    E = s.size
    os_, od, og = np.zeros(E, np.int32), np.zeros(E, np.int32), np.zeros(E, np.int8)
    rc = lib().orc_canonicalize(n_genes, E, _ptr(s), _ptr(d), _ptr(g), _ptr(os_), _ptr(od), _ptr(og))
    if rc != 0:
        raise ValueError("invalid topology")
    return Network(n_genes, os_, od, og)


@dataclass
class Ranges:
    g_min: float = 1.0
    g_max: float = 100.0
    k_min: float = 0.1
    k_max: float = 1.0
    lam_act_min: float = 1.0
    lam_act_max: float = 100.0
    lam_inh_min: float = 0.01
    lam_inh_max: float = 1.0
    n_min: int = 1
    n_max: int = 6
    t_lo: float = 0.02
    t_hi: float = 1.98
    t_median: float = 0.0
    method: int = 0           # UNIFORM, SOBOL, LHS
    threshold_rule: int = 0   # PRIOR_MEDIAN, HALF_FUNCTIONAL
    hf_samples: int = 65536
    hf_act_over_lambda: int = 1
    lhs_total: int = 0
    n_continuous: int = 0     # 1: real Hill coefficients on [n_min, n_max] (in Params.nf)

    def c(self) -> _Ranges:
        return _Ranges(*[getattr(self, f[0]) for f in _Ranges._fields_])


def gk_median(r: Ranges | None = None) -> float:
    rr = (r or Ranges()).c()
    return lib().orc_gk_median(C.byref(rr))


@dataclass
class Params:
    G: np.ndarray    # [N][P] f32
    k: np.ndarray    # [N][P] f32
    T: np.ndarray    # [E][P] f32
    lam: np.ndarray  # [E][P] f32
    n: np.ndarray    # [E][P] u8
    ic: np.ndarray   # [n_ic][N] f32
    nf: np.ndarray | None = None  # [E][P] f32 real Hill coefficients, used instead of n

    @property
    def n_sets(self) -> int:
        return int(self.G.shape[1])


def sample(net: Network, seed: int, n_sets: int, n_ic: int, set_begin: int = 0,
           ranges: Ranges | None = None) -> Params:
    N, E, P = net.n_genes, net.n_edges, n_sets
    G = np.zeros((N, P), np.float32); k = np.zeros((N, P), np.float32)
    T = np.zeros((E, P), np.float32); lam = np.zeros((E, P), np.float32)
    n = np.zeros((E, P), np.uint8); ic = np.zeros((n_ic, N), np.float32)
    rg = ranges or Ranges()
    nf = np.zeros((E, P), np.float32) if rg.n_continuous else None
    rr = rg.c()
    rc = lib().orc_sample(N, E, _ptr(net.src), _ptr(net.dst), _ptr(net.sign), C.byref(rr),
                          C.c_uint64(seed & (2**64 - 1)),
                          set_begin, P, n_ic, _ptr(G), _ptr(k), _ptr(T), _ptr(lam), _ptr(n), _ptr(ic),
                          _ptr(nf))
    if rc != 0:
        raise ValueError("orc_sample failed")
    return Params(G, k, T, lam, n, ic, nf)


DP5, TSIT5 = 0, 1
UNIFORM, SOBOL, LHS = 0, 1, 2
PRIOR_MEDIAN, HALF_FUNCTIONAL = 0, 1


def hf_median(n_act: int, n_inh: int, ranges: "Ranges | None" = None) -> float:
    rr = (ranges or Ranges()).c()
    return lib().orc_hf_median(C.byref(rr), n_act, n_inh)


def sobol_u32(i: int, q: int) -> int:
    v = C.c_uint32(0)
    if lib().orc_sobol_u32(i, q, C.byref(v)) != 0:
        raise ValueError("Sobol index or dimension out of range")
    return v.value


def primitive_count(s: int) -> int:
    return lib().orc_primitive_count(s)


def lhs_perm(seed: int, domain: int, q: int, n: int, i: int) -> int:
    return lib().orc_lhs_perm(C.c_uint64(seed & (2**64 - 1)), domain, q, n, i)


def tableau(method: int):
    """(A[7][7], b, bh, c) of the oracle's 5(4) pair for a method."""
    a = np.zeros((7, 7)); b = np.zeros(7); bh = np.zeros(7); c = np.zeros(7)
    if lib().orc_tableau(method, _ptr(a), _ptr(b), _ptr(bh), _ptr(c)) != 0:
        raise ValueError(f"unknown method {method}")
    return a, b, bh, c


@dataclass
class Opts:
    t0: float = 0.0
    t_end: float = 200.0
    rtol: float = 1e-6
    atol: float = 1e-9
    ss_atol: float = 1e-6
    ss_rtol: float = 0.0
    h0: float = 0.0
    max_steps: int = 100000
    divide_act_by_lambda: int = 1
    stop_at_steady: int = 0
    ic_absolute: int = 0
    method: int = 0  # DP5 or TSIT5

    def c(self) -> _Opts:
        return _Opts(*[getattr(self, f[0]) for f in _Opts._fields_])


class _Keep:
    """Holds the arrays a _Problem points at."""

    def __init__(self, net: Network, prm: Params):
        self.arrs = [np.ascontiguousarray(a) for a in
                     (net.src, net.dst, net.sign, prm.G, prm.k, prm.T, prm.lam, prm.n, prm.ic)]
        s, d, g, G, k, T, lam, n, ic = self.arrs
        assert G.dtype == np.float32 and T.dtype == np.float32 and n.dtype == np.uint8
        assert ic.dtype == np.float32
        nf = None if prm.nf is None else np.ascontiguousarray(prm.nf, dtype=np.float32)
        self.arrs.append(nf)
        self.pb = _Problem(net.n_genes, net.n_edges, _ptr(s), _ptr(d), _ptr(g), _ptr(G), _ptr(k),
                           _ptr(T), _ptr(lam), _ptr(n), prm.n_sets, _ptr(ic), ic.shape[0], _ptr(nf))


@dataclass
class Result:
    x: np.ndarray
    t_final: np.ndarray = field(default=None)
    status: np.ndarray = field(default=None)
    n_acc: np.ndarray = field(default=None)
    n_rej: np.ndarray = field(default=None)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def rhs(net: Network, prm: Params, p: int, x, divide: int = 1) -> np.ndarray:
    keep = _Keep(net, prm)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros(net.n_genes, np.float64)
    lib().orc_rhs(C.byref(keep.pb), p, divide, _ptr(xx), _ptr(f))
    return f


def _ids(traj_ids, total):
    if traj_ids is None:
        return None, total
    ids = np.ascontiguousarray(traj_ids, dtype=np.int64)
    return ids, ids.size


def steady_states(net: Network, prm: Params, opts: Opts | None = None, traj_ids=None,
                  n_threads: int | None = None) -> Result:
    keep = _Keep(net, prm)
    o = (opts or Opts()).c()
    ids, nt = _ids(traj_ids, prm.n_sets * prm.ic.shape[0])
    x = np.zeros((nt, net.n_genes), np.float64)
    tf = np.zeros(nt, np.float64); st = np.zeros(nt, np.int8)
    na = np.zeros(nt, np.int32); nr = np.zeros(nt, np.int32)
    rc = lib().orc_steady_states(C.byref(keep.pb), C.byref(o), _ptr(ids), nt,
                                 n_threads or default_threads(), _ptr(x), _ptr(tf), _ptr(st),
                                 _ptr(na), _ptr(nr))
    if rc != 0:
        raise ValueError("orc_steady_states failed")
    return Result(x, tf, st, na, nr)


def time_series(net: Network, prm: Params, t_out, opts: Opts | None = None, traj_ids=None,
                n_threads: int | None = None) -> Result:
    keep = _Keep(net, prm)
    o = (opts or Opts()).c()
    t = np.ascontiguousarray(t_out, dtype=np.float64)
    ids, nt = _ids(traj_ids, prm.n_sets * prm.ic.shape[0])
    x = np.zeros((nt, t.size, net.n_genes), np.float64)
    tf = np.zeros(nt, np.float64); st = np.zeros(nt, np.int8)
    na = np.zeros(nt, np.int32); nr = np.zeros(nt, np.int32)
    rc = lib().orc_time_series(C.byref(keep.pb), C.byref(o), _ptr(t), t.size, _ptr(ids), nt,
                               n_threads or default_threads(), _ptr(x), _ptr(tf), _ptr(st),
                               _ptr(na), _ptr(nr))
    if rc != 0:
        raise ValueError("orc_time_series failed")
    return Result(x, tf, st, na, nr)


def rk4(net: Network, prm: Params, h: float, t_out, opts: Opts | None = None, traj_ids=None,
        n_threads: int | None = None) -> np.ndarray:
    keep = _Keep(net, prm)
    o = (opts or Opts()).c()
    t = np.ascontiguousarray(t_out, dtype=np.float64)
    ids, nt = _ids(traj_ids, prm.n_sets * prm.ic.shape[0])
    x = np.zeros((nt, t.size, net.n_genes), np.float64)
    rc = lib().orc_rk4(C.byref(keep.pb), C.byref(o), h, _ptr(t), t.size, _ptr(ids), nt,
                       n_threads or default_threads(), _ptr(x))
    if rc != 0:
        raise ValueError("orc_rk4 failed")
    return x


def dp5_fixed(net: Network, prm: Params, traj: int, n_steps: int, opts: Opts | None = None):
    keep = _Keep(net, prm)
    o = (opts or Opts()).c()
    x = np.zeros(net.n_genes, np.float64)
    err = C.c_double(0.0)
    rc = lib().orc_dp5_fixed(C.byref(keep.pb), C.byref(o), traj, n_steps, _ptr(x), C.byref(err))
    if rc != 0:
        raise ValueError("orc_dp5_fixed failed")
    return x, err.value
