"""Python binding of librac.so (the C ABI in include/rac.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory and streams.  The
binding fails loudly when the native library is missing; there is no CPU
fallback.

Names follow rac.h: ``create_topology``, ``sample_params``, ``steady_states``,
``integrate`` and ``steady_states_batch``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librac.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
CONVERGED, T_END, MAX_STEPS, STEP_UNDERFLOW, NONFINITE = range(5)
FP32, FP64 = 0, 1
DP5, TSIT5 = 0, 1  # rac_method
SAMPLE_UNIFORM, SAMPLE_SOBOL, SAMPLE_LHS = 0, 1, 2  # rac_sample_method
PRIOR_MEDIAN, HALF_FUNCTIONAL = 0, 1  # rac_threshold_rule
STATUS_NAMES = ["CONVERGED", "T_END", "MAX_STEPS", "STEP_UNDERFLOW", "NONFINITE"]


class RacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rac error {code}: {msg}")
        self.code = code


class _Ranges(C.Structure):
    _fields_ = [("g_min", C.c_double), ("g_max", C.c_double), ("k_min", C.c_double),
                ("k_max", C.c_double), ("lam_act_min", C.c_double), ("lam_act_max", C.c_double),
                ("lam_inh_min", C.c_double), ("lam_inh_max", C.c_double), ("n_min", C.c_int32),
                ("n_max", C.c_int32), ("t_lo", C.c_double), ("t_hi", C.c_double),
                ("t_median", C.c_double), ("method", C.c_int32), ("threshold_rule", C.c_int32),
                ("hf_samples", C.c_int32), ("hf_act_over_lambda", C.c_int32),
                ("lhs_total", C.c_int64), ("n_continuous", C.c_int32)]


class _ParamsView(C.Structure):
    _fields_ = [("G", C.c_void_p), ("k", C.c_void_p), ("T", C.c_void_p), ("lam", C.c_void_p),
                ("n", C.c_void_p), ("n_sets", C.c_int64), ("nf", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("t0", C.c_double), ("t_end", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("ss_atol", C.c_double), ("ss_rtol", C.c_double),
                ("h0", C.c_double), ("max_steps", C.c_int64), ("precision", C.c_int32),
                ("activation_divides_by_lambda", C.c_int32), ("stop_at_steady", C.c_int32),
                ("ic_absolute", C.c_int32), ("lanes_per_traj", C.c_int32),
                ("refill_min", C.c_int32), ("method", C.c_int32)]


class _IsingOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("low", C.c_int32), ("max_steps", C.c_int32),
                ("check_every", C.c_int32), ("seed", C.c_uint64), ("order", C.c_void_p),
                ("order_len", C.c_int32), ("dev_evals", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("t_final", C.c_void_p), ("status", C.c_void_p), ("n_accepted", C.c_void_p),
                ("n_rejected", C.c_void_p)]


class _BatchItem(C.Structure):
    _fields_ = [("topo", C.c_void_p), ("params", _ParamsView), ("ic", C.c_void_p),
                ("n_ic", C.c_int32), ("x_out", C.c_void_p), ("info", _Info),
                ("lanes_per_traj", C.c_int32), ("refill_min", C.c_int32)]


_lib = None


def lib():
    """The loaded librac.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.rac_last_error.restype = C.c_char_p
        L.rac_version.restype = C.c_char_p
        L.rac_create_topology.argtypes = [i32, i32, vp, vp, vp, C.POINTER(vp)]
        L.rac_create_topology.restype = C.c_int
        L.rac_destroy_topology.argtypes = [vp]
        L.rac_topology_size.argtypes = [vp, vp, vp]
        L.rac_topology_size.restype = C.c_int
        L.rac_topology_edges.argtypes = [vp, vp, vp, vp]
        L.rac_topology_edges.restype = C.c_int
        L.rac_default_ranges.argtypes = [C.POINTER(_Ranges)]
        L.rac_sample_params.argtypes = [vp, C.POINTER(_Ranges), C.c_uint64, i64, i64, i32,
                                        C.POINTER(_ParamsView), vp]
        L.rac_sample_params.restype = C.c_int
        L.rac_default_opts.argtypes = [C.POINTER(_Opts), i32]
        L.rac_steady_states.argtypes = [vp, C.POINTER(_ParamsView), vp, i32, C.POINTER(_Opts),
                                        vp, C.POINTER(_Info), vp]
        L.rac_steady_states.restype = C.c_int
        L.rac_steady_states_noalloc.argtypes = [vp, C.POINTER(_ParamsView), vp, i32, C.POINTER(_Opts),
                                                vp, C.POINTER(_Info), vp]
        L.rac_steady_states_noalloc.restype = C.c_int
        L.rac_integrate.argtypes = [vp, C.POINTER(_ParamsView), vp, i32, C.POINTER(_Opts), vp,
                                    i32, vp, C.POINTER(_Info), vp]
        L.rac_integrate.restype = C.c_int
        L.rac_steady_states_batch.argtypes = [C.POINTER(_BatchItem), i32, C.POINTER(_Opts), vp]
        L.rac_steady_states_batch.restype = C.c_int
        L.rac_auto_lanes.argtypes = [vp, i32]
        L.rac_auto_lanes.restype = i32
        L.rac_auto_lanes_for.argtypes = [vp, i32, i64]
        L.rac_auto_lanes_for.restype = i32
        L.rac_lanes_supported.argtypes = [vp, i32, i32]
        L.rac_lanes_supported.restype = i32
        L.rac_plan_shape.argtypes = [vp, i32, i32, vp, vp]
        L.rac_plan_shape.restype = C.c_int
        L.rac_factor_form.argtypes = [i32, i32]
        L.rac_factor_form.restype = i32
        L.rac_valu_ceilings.argtypes = [vp, i32]
        L.rac_valu_ceilings.restype = C.c_int
        L.rac_sample_params_device.argtypes = [vp, C.POINTER(_Ranges), C.c_uint64, i64, i64, i32,
                                               C.POINTER(_ParamsView), vp, vp]
        L.rac_sample_params_device.restype = C.c_int
        L.rac_server_create.argtypes = [C.POINTER(_Opts), i32, i32, i32, i32, C.POINTER(vp)]
        L.rac_server_create.restype = C.c_int
        L.rac_server_destroy.argtypes = [vp]
        L.rac_server_submit.argtypes = [vp, vp, C.POINTER(_ParamsView), vp, i32, vp,
                                        C.POINTER(_Info), vp, C.POINTER(i32)]
        L.rac_server_submit.restype = C.c_int
        L.rac_server_step.argtypes = [vp, vp]
        L.rac_server_step.restype = C.c_int
        L.rac_server_done_counts.argtypes = [vp, i32, i32, vp, vp]
        L.rac_server_done_counts.restype = C.c_int
        L.rac_server_info.argtypes = [vp, vp, vp, vp, vp]
        L.rac_server_info.restype = C.c_int
        L.rac_not_steady_flag.argtypes = [i32]
        L.rac_not_steady_flag.restype = i32
        L.rac_steady_flags.argtypes = [vp, i64, vp, vp]
        L.rac_steady_flags.restype = C.c_int
        L.rac_normalize.argtypes = [vp, C.POINTER(_ParamsView), i32, i32, vp, vp, vp]
        L.rac_normalize.restype = C.c_int
        L.rac_level_thresholds.argtypes = [vp, i64, i32, vp, i32, i32, vp, vp, vp]
        L.rac_level_thresholds.restype = C.c_int
        L.rac_discretize.argtypes = [vp, i64, i32, vp, i32, i32, vp, vp, vp, vp]
        L.rac_discretize.restype = C.c_int
        L.rac_multistability.argtypes = [vp, i64, i32, vp, vp, vp]
        L.rac_multistability.restype = C.c_int
        L.rac_state_counts.argtypes = [vp, i64, i64, vp, vp, vp, vp]
        L.rac_state_counts.restype = C.c_int
        L.rac_default_ising_opts.argtypes = [C.POINTER(_IsingOpts)]
        L.rac_ising.argtypes = [vp, C.POINTER(_IsingOpts), i64, vp, vp, vp, vp, vp]
        L.rac_ising.restype = C.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise RacError(code, lib().rac_last_error().decode())


def last_error() -> str:
    return lib().rac_last_error().decode()


CEILING_NAMES = ("fp32_fma", "v_exp_f32", "v_log_f32", "v_rcp_f32", "fp64_fma", "fp32_fma_literal")


def valu_ceilings() -> dict:
    """Measured sustained lane-operation rates (per second, all lanes) of the
    current device for FP32 FMA (register operands), v_exp/v_log/v_rcp, FP64
    FMA and FP32 FMA with a literal multiplier."""
    out = (C.c_double * len(CEILING_NAMES))()
    _check(lib().rac_valu_ceilings(out, len(CEILING_NAMES)))
    return dict(zip(CEILING_NAMES, list(out)))


def factor_form(precision: int, epl: int) -> int:
    """Hill-factor form of the kernels with this precision and edge-slot count
    (1: 1 + D / (1 + 2^z); 0: symmetric sqrt(lam) form).  Kernels of one form
    and lane count give bit-identical results whatever their slot counts."""
    f = int(lib().rac_factor_form(precision, epl))
    if f < 0:
        raise ValueError(f"bad precision {precision} or epl {epl}")
    return f


class Topology:
    """Owns a rac_topology handle; edges are kept in canonical (dst, src) order."""

    def __init__(self, n_genes: int, src, dst, sign):
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        g = np.ascontiguousarray(sign, dtype=np.int8)
        h = C.c_void_p()
        _check(lib().rac_create_topology(int(n_genes), int(s.size), s.ctypes.data, d.ctypes.data,
                                         g.ctypes.data, C.byref(h)))
        self._h = h
        self.n_genes = int(n_genes)
        self.n_edges = int(s.size)
        self.src = np.zeros(self.n_edges, np.int32)
        self.dst = np.zeros(self.n_edges, np.int32)
        self.sign = np.zeros(self.n_edges, np.int8)
        _check(lib().rac_topology_edges(h, self.src.ctypes.data, self.dst.ctypes.data,
                                        self.sign.ctypes.data))

    @classmethod
    def from_inputs(cls, t) -> "Topology":
        return cls(t.n_genes, t.src, t.dst, t.sign)

    @property
    def handle(self):
        return self._h

    def auto_lanes(self, precision: int = FP32, n_traj: int | None = None) -> int:
        """The library's lane count: the cost model's, or, given the call's
        trajectory count, the one a call of that size takes."""
        if n_traj is None:
            return int(lib().rac_auto_lanes(self._h, precision))
        return int(lib().rac_auto_lanes_for(self._h, precision, int(n_traj)))

    def lanes_supported(self, lanes: int, precision: int = FP32) -> bool:
        return bool(lib().rac_lanes_supported(self._h, precision, lanes))

    def shape(self, lanes: int, precision: int = FP32) -> tuple[int, int]:
        """Compiled (edge slots, gene slots) per lane at this lane count."""
        e, g = C.c_int32(), C.c_int32()
        _check(lib().rac_plan_shape(self._h, precision, lanes, C.byref(e), C.byref(g)))
        return e.value, g.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rac_destroy_topology(h)
            self._h = None


def create_topology(n_genes: int, src, dst, sign) -> Topology:
    return Topology(n_genes, src, dst, sign)


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
    method: int = 0             # SAMPLE_UNIFORM, SAMPLE_SOBOL, SAMPLE_LHS
    threshold_rule: int = 0     # PRIOR_MEDIAN, HALF_FUNCTIONAL
    hf_samples: int = 65536
    hf_act_over_lambda: int = 1
    lhs_total: int = 0
    n_continuous: int = 0       # 1: real Hill coefficients on [n_min, n_max], in nf

    def c(self) -> _Ranges:
        return _Ranges(*[getattr(self, f[0]) for f in _Ranges._fields_])


@dataclass
class HostParams:
    """Host arrays in the layout of rac_params_view (set index fastest)."""
    G: np.ndarray
    k: np.ndarray
    T: np.ndarray
    lam: np.ndarray
    n: np.ndarray
    ic: np.ndarray
    nf: np.ndarray | None = None   # real Hill coefficients (f32), used instead of n

    @property
    def n_sets(self) -> int:
        return int(self.G.shape[1])

    def to_device(self, device="cuda"):
        import torch
        return DeviceParams(*[None if getattr(self, f.name) is None else
                              torch.from_numpy(np.ascontiguousarray(getattr(self, f.name))).to(device)
                              for f in fields(self)])


@dataclass
class DeviceParams:
    """torch tensors on the GPU: G, k [N][P]; T, lam [E][P] f32; n [E][P] u8; ic [n_ic][N];
    nf [E][P] f32 real Hill coefficients or None."""
    G: object
    k: object
    T: object
    lam: object
    n: object
    ic: object
    nf: object = None

    @property
    def n_sets(self) -> int:
        return int(self.G.shape[1])

    @property
    def n_ic(self) -> int:
        return int(self.ic.shape[0])

    def view(self) -> _ParamsView:
        return _ParamsView(self.G.data_ptr(), self.k.data_ptr(), self.T.data_ptr(),
                           self.lam.data_ptr(), None if self.n is None else self.n.data_ptr(), self.n_sets,
                           None if self.nf is None else self.nf.data_ptr())


def sample_params(topo: Topology, seed: int, n_sets: int, n_ic: int, set_begin: int = 0,
                  ranges: Ranges | None = None) -> HostParams:
    N, E, P = topo.n_genes, topo.n_edges, int(n_sets)
    G = np.zeros((N, P), np.float32)
    k = np.zeros((N, P), np.float32)
    T = np.zeros((E, P), np.float32)
    lam = np.zeros((E, P), np.float32)
    n = np.zeros((E, P), np.uint8)
    ic = np.zeros((n_ic, N), np.float32)
    rg = ranges or Ranges()
    nf = np.zeros((E, P), np.float32) if rg.n_continuous else None
    v = _ParamsView(G.ctypes.data, k.ctypes.data, T.ctypes.data, lam.ctypes.data, n.ctypes.data, P,
                    None if nf is None else nf.ctypes.data)
    rr = rg.c()
    _check(lib().rac_sample_params(topo.handle, C.byref(rr), C.c_uint64(seed & (2**64 - 1)),
                                   set_begin, P, n_ic, C.byref(v), ic.ctypes.data))
    return HostParams(G, k, T, lam, n, ic, nf)


def alloc_params(topo: Topology, n_sets: int, n_ic: int, device="cuda",
                 n_continuous: bool = False) -> DeviceParams:
    import torch
    N, E, P = topo.n_genes, topo.n_edges, int(n_sets)
    f = lambda *sh: torch.empty(sh, dtype=torch.float32, device=device)
    return DeviceParams(f(N, P), f(N, P), f(E, P), f(E, P),
                        torch.empty((E, P), dtype=torch.uint8, device=device), f(n_ic, N),
                        f(E, P) if n_continuous else None)


def sample_params_device(topo: Topology, seed: int, n_sets: int, n_ic: int, set_begin: int = 0,
                         ranges: Ranges | None = None, out: DeviceParams | None = None,
                         stream=None) -> DeviceParams:
    """rac_sample_params_device: the same draws as sample_params, on the GPU."""
    rg = ranges or Ranges()
    out = out or alloc_params(topo, n_sets, n_ic, n_continuous=bool(rg.n_continuous))
    v = out.view()
    rr = rg.c()
    _check(lib().rac_sample_params_device(topo.handle, C.byref(rr), C.c_uint64(seed & (2**64 - 1)),
                                          set_begin, int(n_sets), n_ic, C.byref(v),
                                          out.ic.data_ptr(), _stream_ptr(stream)))
    return out


@dataclass
class Opts:
    t0: float = 0.0
    t_end: float = 200.0
    rtol: float = 1e-6
    atol: float = 1e-9
    ss_atol: float = 1e-6
    ss_rtol: float | None = None   # None: 1e-5 for FP32, 0 for FP64
    h0: float = 0.0
    max_steps: int = 100000
    precision: int = FP32
    activation_divides_by_lambda: int = 1
    stop_at_steady: int = 0
    ic_absolute: int = 0
    lanes_per_traj: int = 0
    refill_min: int = 0
    method: int = 0  # DP5 or TSIT5

    def c(self) -> _Opts:
        o = _Opts()
        lib().rac_default_opts(C.byref(o), self.precision)
        for f in fields(self):
            v = getattr(self, f.name)
            if v is not None:
                setattr(o, f.name, v)
        return o


@dataclass
class Result:
    x: object          # torch tensor [n_traj][N] (or [n_traj][n_t][N])
    t_final: object    # f64 [n_traj]
    status: object     # i8 [n_traj]
    n_acc: object      # i32 [n_traj]
    n_rej: object      # i32 [n_traj]


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def alloc_result(n_traj: int, n_genes: int, precision: int, n_t: int = 0, device="cuda") -> Result:
    import torch
    dt = torch.float32 if precision == FP32 else torch.float64
    shape = (n_traj, n_t, n_genes) if n_t else (n_traj, n_genes)
    return Result(torch.empty(shape, dtype=dt, device=device),
                  torch.empty(n_traj, dtype=torch.float64, device=device),
                  torch.empty(n_traj, dtype=torch.int8, device=device),
                  torch.empty(n_traj, dtype=torch.int32, device=device),
                  torch.empty(n_traj, dtype=torch.int32, device=device))


def fill_sentinels(res: Result) -> Result:
    """Mark every output as not written (x NaN, t_final NaN, status -1, step
    counts -1), so that a trajectory a solve never finished is visible."""
    res.x.fill_(float("nan"))
    res.t_final.fill_(float("nan"))
    res.status.fill_(-1)
    res.n_acc.fill_(-1)
    res.n_rej.fill_(-1)
    return res


def unfinished(res: Result) -> int:
    """Trajectories whose outputs still hold a sentinel after a solve: a
    status outside 0..4, a negative step count, a NaN end time or a
    non-finite state (a finished trajectory with NaN state has status
    NONFINITE and is not counted)."""
    import torch
    st = res.status
    bad = (st < 0) | (st > 4) | (res.n_acc < 0) | (res.n_rej < 0) | torch.isnan(res.t_final)
    xbad = ~torch.isfinite(res.x.reshape(res.x.shape[0], -1)).all(dim=1)
    bad |= xbad & (st != NONFINITE)
    return int(bad.sum().item())


def _info(res: Result) -> _Info:
    return _Info(res.t_final.data_ptr(), res.status.data_ptr(), res.n_acc.data_ptr(),
                 res.n_rej.data_ptr())


def steady_states(topo: Topology, params: DeviceParams, opts: Opts | None = None,
                  out: Result | None = None, stream=None) -> Result:
    """Enqueue rac_steady_states on the stream (asynchronous)."""
    opts = opts or Opts()
    n_traj = params.n_sets * params.n_ic
    out = out or alloc_result(n_traj, topo.n_genes, opts.precision, device=params.G.device)
    v = params.view()
    info = _info(out)
    o = opts.c()
    _check(lib().rac_steady_states(topo.handle, C.byref(v), params.ic.data_ptr(), params.n_ic,
                                   C.byref(o), out.x.data_ptr(), C.byref(info), _stream_ptr(stream)))
    return out


def steady_states_noalloc(topo: Topology, params: DeviceParams, opts: Opts, out: Result,
                          stream=None) -> Result:
    """Enqueue rac_steady_states_noalloc: as steady_states into the caller's
    `out`, with no device allocation (the network must have been solved once
    with the same options on this device)."""
    v = params.view()
    info = _info(out)
    o = opts.c()
    _check(lib().rac_steady_states_noalloc(topo.handle, C.byref(v), params.ic.data_ptr(), params.n_ic,
                                           C.byref(o), out.x.data_ptr(), C.byref(info),
                                           _stream_ptr(stream)))
    return out


def integrate(topo: Topology, params: DeviceParams, t_out, opts: Opts | None = None,
              out: Result | None = None, stream=None) -> Result:
    """Enqueue rac_integrate (time series at t_out) on the stream."""
    opts = opts or Opts()
    t = np.ascontiguousarray(t_out, dtype=np.float64)
    n_traj = params.n_sets * params.n_ic
    out = out or alloc_result(n_traj, topo.n_genes, opts.precision, n_t=t.size,
                              device=params.G.device)
    v = params.view()
    info = _info(out)
    o = opts.c()
    _check(lib().rac_integrate(topo.handle, C.byref(v), params.ic.data_ptr(), params.n_ic,
                               C.byref(o), t.ctypes.data, int(t.size), out.x.data_ptr(),
                               C.byref(info), _stream_ptr(stream)))
    return out


def steady_states_batch(items, opts: Opts | None = None, stream=None) -> list[Result]:
    """items: list of (Topology, DeviceParams[, Result[, (lanes, refill_min)]]).
    One fused launch per lane count and kernel shape; returns the Results.
    The optional pair overrides the options' lane count and refill batch for
    that network (0 keeps the options')."""
    opts = opts or Opts()
    outs, arr = [], (_BatchItem * max(len(items), 1))()
    for i, it in enumerate(items):
        topo, prm = it[0], it[1]
        out = it[2] if len(it) > 2 and it[2] is not None else alloc_result(
            prm.n_sets * prm.n_ic, topo.n_genes, opts.precision, device=prm.G.device)
        lanes, refill = it[3] if len(it) > 3 and it[3] is not None else (0, 0)
        outs.append(out)
        arr[i] = _BatchItem(topo.handle.value, prm.view(), prm.ic.data_ptr(), prm.n_ic,
                            out.x.data_ptr(), _info(out), int(lanes), int(refill))
    o = opts.c()
    _check(lib().rac_steady_states_batch(arr, len(items), C.byref(o), _stream_ptr(stream)))
    return outs


class StepServer:
    """One rac_server: step batches of the bounded kernel for networks that fit
    (lanes, epl, gpl)."""

    def __init__(self, opts: Opts, lanes: int, epl: int, gpl: int, max_requests: int = 65536,
                 batch_steps: int = 256):
        o = Opts(**{f.name: getattr(opts, f.name) for f in fields(opts)})
        o.lanes_per_traj = lanes
        h = C.c_void_p()
        _check(lib().rac_server_create(C.byref(o.c()), epl, gpl, max_requests, batch_steps,
                                       C.byref(h)))
        self._h = h
        self.lanes, self.epl, self.gpl = lanes, epl, gpl
        self.n_requests = 0

    def submit(self, topo: Topology, params: DeviceParams, out: Result, stream=None) -> int:
        v = params.view()
        info = _info(out)
        rid = C.c_int32()
        _check(lib().rac_server_submit(self._h, topo.handle, C.byref(v), params.ic.data_ptr(),
                                       params.n_ic, out.x.data_ptr(), C.byref(info),
                                       _stream_ptr(stream), C.byref(rid)))
        self.n_requests = rid.value + 1
        return rid.value

    def step(self, stream=None):
        _check(lib().rac_server_step(self._h, _stream_ptr(stream)))

    def done_counts(self, first: int, count: int, out: np.ndarray, stream=None):
        """Enqueue the copy of finished counts into out[:count] (int32, host)."""
        _check(lib().rac_server_done_counts(self._h, first, count, out.ctypes.data,
                                            _stream_ptr(stream)))

    def info(self) -> dict:
        n, tot, waves, sb = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib().rac_server_info(self._h, C.byref(n), C.byref(tot), C.byref(waves), C.byref(sb)))
        return dict(n_requests=n.value, total=tot.value, waves=waves.value, slot_bytes=sb.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rac_server_destroy(h)
            self._h = None


# --------------------------------------------------------------------------
# Post-processing (rac_normalize ... rac_state_counts).  State codes travel
# as int64 tensors holding the u64 bits; RAC_NO_STATE reads as -1.
# --------------------------------------------------------------------------
NO_STATE = -1


def _ptr(t):
    return None if t is None else t.data_ptr()


def not_steady_flag(status: int) -> int:
    """The paper's steady-state flag of one status: 0 if CONVERGED, else 1."""
    return int(lib().rac_not_steady_flag(int(status)))


def steady_flags(status, out=None, stream=None):
    """rac_steady_flags: the paper's flag (u8, 1 = no steady state) for every
    trajectory of a device status array."""
    import torch
    out = out if out is not None else torch.empty(status.numel(), dtype=torch.uint8, device=status.device)
    _check(lib().rac_steady_flags(status.data_ptr(), status.numel(), out.data_ptr(), _stream_ptr(stream)))
    return out


def normalize(topo: Topology, params: DeviceParams, x, n_t: int = 1, out=None, stream=None):
    """G/k-normalised copy of a float32 result x ([P*n_ic*n_t][N] or any shape
    with that many elements)."""
    import torch
    assert x.dtype == torch.float32 and x.is_contiguous()
    y = out if out is not None else torch.empty_like(x)
    v = params.view()
    _check(lib().rac_normalize(topo.handle, C.byref(v), params.n_ic, n_t, x.data_ptr(), y.data_ptr(),
                               _stream_ptr(stream)))
    return y


def level_thresholds(y, n_genes: int, status=None, n_bins: int = 64, n_levels: int = 2, stream=None):
    """(hist int64[n_bins], thresholds int32[n_levels-1]) on the device."""
    import torch
    n_rows = y.numel() // n_genes
    hist = torch.empty(n_bins, dtype=torch.int64, device=y.device)
    thr = torch.empty(n_levels - 1, dtype=torch.int32, device=y.device)
    _check(lib().rac_level_thresholds(y.data_ptr(), n_rows, n_genes, _ptr(status), n_bins, n_levels,
                                      hist.data_ptr(), thr.data_ptr(), _stream_ptr(stream)))
    return hist, thr


def discretize(y, n_genes: int, thresholds, status=None, n_bins: int = 64, n_levels: int = 2,
               want_levels: bool = True, want_codes: bool = True, stream=None):
    """(levels uint8[rows][N] or None, codes int64[rows] or None)."""
    import torch
    n_rows = y.numel() // n_genes
    lv = torch.empty((n_rows, n_genes), dtype=torch.uint8, device=y.device) if want_levels else None
    cd = torch.empty(n_rows, dtype=torch.int64, device=y.device) if want_codes else None
    _check(lib().rac_discretize(y.data_ptr(), n_rows, n_genes, _ptr(status), n_bins, n_levels,
                                thresholds.data_ptr(), _ptr(lv), _ptr(cd), _stream_ptr(stream)))
    return lv, cd


def multistability(codes, n_sets: int, n_ic: int, stream=None):
    """(n_states int32[n_sets], states int64[n_sets][n_ic])."""
    import torch
    n = torch.empty(n_sets, dtype=torch.int32, device=codes.device)
    st = torch.empty((n_sets, n_ic), dtype=torch.int64, device=codes.device)
    _check(lib().rac_multistability(codes.data_ptr(), n_sets, n_ic, n.data_ptr(), st.data_ptr(),
                                    _stream_ptr(stream)))
    return n, st


def state_counts(codes, capacity: int = 1 << 16, stream=None):
    """(keys int64[capacity], counts int64[capacity], n_unique int64[1]) on the
    device; the first n_unique entries are the distinct states in ascending
    unsigned order."""
    import torch
    keys = torch.empty(capacity, dtype=torch.int64, device=codes.device)
    counts = torch.empty(capacity, dtype=torch.int64, device=codes.device)
    nu = torch.empty(1, dtype=torch.int64, device=codes.device)
    _check(lib().rac_state_counts(codes.data_ptr(), codes.numel(), capacity, keys.data_ptr(),
                                  counts.data_ptr(), nu.data_ptr(), _stream_ptr(stream)))
    return keys, counts, nu


def state_table_size(n_rows: int, n_genes: int, n_levels: int, capacity: int = 1 << 16) -> int:
    """The state-frequency table analyse_steady_states allocates: no more
    distinct states can occur than rows or than n_levels^N codes, so the
    smallest power of two (at least 2) holding that many, capped at capacity."""
    bound = min(n_rows, n_levels ** n_genes)
    cap = 2
    while cap < bound and cap < capacity:
        cap <<= 1
    return min(cap, capacity)


def analyse_steady_states(topo: Topology, params: DeviceParams, result: Result, n_bins: int = 64,
                          n_levels: int = 2, capacity: int = 1 << 16, stream=None) -> dict:
    """The whole chain on a steady-state result, all on the device: normalised
    states, histogram and thresholds, levels and state codes, multistability
    per parameter set and global state frequencies (in a table of
    state_table_size(rows, N, n_levels, capacity) entries)."""
    N = topo.n_genes
    y = normalize(topo, params, result.x, 1, stream=stream)
    hist, thr = level_thresholds(y, N, result.status, n_bins, n_levels, stream=stream)
    lv, cd = discretize(y, N, thr, result.status, n_bins, n_levels, stream=stream)
    n_states, states = multistability(cd, params.n_sets, params.n_ic, stream=stream)
    cap = state_table_size(params.n_sets * params.n_ic, N, n_levels, capacity)
    keys, counts, nu = state_counts(cd, cap, stream=stream)
    return dict(y=y, hist=hist, thresholds=thr, levels=lv, codes=cd, n_states=n_states,
                states=states, keys=keys, counts=counts, n_unique=nu)


# --------------------------------------------------------------------------
# Boolean Ising formalism (rac_ising).  States travel as int64 tensors of
# shape [n_traj][W] holding the bit-packed u64 words (gene i: bit i % 64 of
# word i // 64).
# --------------------------------------------------------------------------
ISING_SYNC, ISING_ASYNC = 0, 1


def ising(topo: Topology, n_traj: int, mode: int = ISING_SYNC, low: int = 0, max_steps: int = 1000,
          seed: int = 0, init=None, order=None, check_every: int = 0, device="cuda", stream=None,
          evals=None):
    """(final int64[n_traj][W], steps int32[n_traj], status int8[n_traj]);
    init: int64[n_traj][W] device tensor or None for seeded random states;
    evals: optional one-element int64 device tensor that the gene
    evaluations performed are added to."""
    import torch
    W = (topo.n_genes + 63) // 64
    fin = torch.empty((n_traj, W), dtype=torch.int64, device=device)
    steps = torch.empty(n_traj, dtype=torch.int32, device=device)
    status = torch.empty(n_traj, dtype=torch.int8, device=device)
    o = _IsingOpts()
    lib().rac_default_ising_opts(C.byref(o))
    o.mode, o.low, o.max_steps, o.check_every = mode, low, max_steps, check_every
    o.seed = seed & (2**64 - 1)
    ordr = None
    if order is not None:
        ordr = np.ascontiguousarray(order, np.int32)
        o.order, o.order_len = ordr.ctypes.data, ordr.size
    if evals is not None:
        o.dev_evals = evals.data_ptr()
    _check(lib().rac_ising(topo.handle, C.byref(o), n_traj, _ptr(init), fin.data_ptr(), steps.data_ptr(),
                           status.data_ptr(), _stream_ptr(stream)))
    return fin, steps, status
