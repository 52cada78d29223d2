"""CPU checks of the C ABI: exported symbols, topology validation, the host
sampler (bit-exact against the oracle's independent sampler), and argument
errors that integration calls report before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "rac.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rac_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "rac_steady_states" in names and "rac_integrate" in names
    assert "rac_create_topology" in names and "rac_sample_params" in names
    L = rp.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _topo(n, src, dst, sign):
    h = C.c_void_p()
    s, d, g = (np.ascontiguousarray(v, dt) for v, dt in
               ((src, np.int32), (dst, np.int32), (sign, np.int8)))
    code = rp.lib().rac_create_topology(n, s.size, s.ctypes.data, d.ctypes.data, g.ctypes.data,
                                        C.byref(h))
    return code, h


@pytest.mark.parametrize("args", [
    (0, [], [], []),                 # no genes
    (2, [0], [2], [1]),              # index out of range
    (2, [-1], [0], [1]),
    (2, [0], [1], [0]),              # sign not +-1
    (2, [0, 0], [1, 1], [1, -1]),    # duplicate edge
])
def test_topology_rejects_bad_input(args):
    code, h = _topo(*args)
    assert code == rp.EINVAL and not h.value
    assert rp.last_error()


def test_topology_too_large_is_unsupported():
    code, _ = _topo(5000, [], [], [])
    assert code == rp.EUNSUPPORTED


def test_topology_canonical_order_and_self_loops():
    t = rp.Topology(3, [2, 0, 1, 1], [0, 1, 1, 0], [1, -1, 1, -1])
    assert list(zip(t.dst, t.src)) == sorted(zip([0, 1, 1, 0], [2, 0, 1, 1]))
    assert t.n_edges == 4


CASES = [
    (inputs.toggle_switch(), 2001),
    (inputs.toggle_switch_self_activation(), 7),
    (inputs.erdos_renyi(10, 25, 1002), 2002),
    (inputs.dense_core(1004), 2004),
    (inputs.unregulated(3), 3),
]


@pytest.mark.parametrize("topo,seed", CASES, ids=[c[0].name for c in CASES])
def test_sampler_matches_oracle_bit_exact(topo, seed):
    t = rp.Topology.from_inputs(topo)
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    assert np.array_equal(t.src, net.src) and np.array_equal(t.dst, net.dst)
    for begin, P, n_ic in [(0, 257, 7), (12345, 31, 1)]:
        a = rp.sample_params(t, seed, P, n_ic, set_begin=begin)
        b = oracle.sample(net, seed, P, n_ic, set_begin=begin)
        for f in ("G", "k", "T", "lam", "n", "ic"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_sampler_custom_ranges_match_oracle():
    topo = inputs.erdos_renyi(6, 10, 3)
    t = rp.Topology.from_inputs(topo)
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    kw = dict(g_min=1, g_max=10, k_min=0.01, k_max=1, lam_act_min=2, lam_act_max=5,
              lam_inh_min=0.1, lam_inh_max=0.5, n_min=2, n_max=3, t_lo=0.5, t_hi=1.5)
    a = rp.sample_params(t, 9, 100, 3, ranges=rp.Ranges(**kw))
    b = oracle.sample(net, 9, 100, 3, ranges=oracle.Ranges(**kw))
    for f in ("G", "k", "T", "lam", "n", "ic"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_sampler_rejects_bad_ranges():
    t = rp.Topology.from_inputs(inputs.toggle_switch())
    with pytest.raises(rp.RacError) as e:
        rp.sample_params(t, 1, 10, 1, ranges=rp.Ranges(k_min=0.0))
    assert e.value.code == rp.EINVAL
    with pytest.raises(rp.RacError):
        rp.sample_params(t, 1, 10, 1, ranges=rp.Ranges(g_min=5, g_max=1))


class _FakeTensor:
    """Stands in for a device tensor: a non-NULL address that is never touched
    because the call fails its argument checks first."""

    def __init__(self, shape):
        self.shape = shape

    def data_ptr(self):
        return 0x1000

    @property
    def device(self):
        return "cuda"


def _fake_params(N, E, P, n_ic):
    return rp.DeviceParams(_FakeTensor((N, P)), _FakeTensor((N, P)), _FakeTensor((E, P)),
                           _FakeTensor((E, P)), _FakeTensor((E, P)), _FakeTensor((n_ic, N)))


def _fake_result():
    return rp.Result(*[_FakeTensor((1,)) for _ in range(5)])


@pytest.mark.parametrize("bad", [
    dict(t_end=0.0), dict(rtol=0.0, atol=0.0), dict(rtol=-1.0), dict(max_steps=0),
    dict(precision=7), dict(lanes_per_traj=3), dict(ss_atol=-1.0), dict(t0=float("nan")),
    dict(method=2), dict(method=-1),
])
def test_steady_states_rejects_bad_options_before_enqueue(bad):
    t = rp.Topology.from_inputs(inputs.toggle_switch())
    with pytest.raises(rp.RacError) as e:
        rp.steady_states(t, _fake_params(2, 2, 4, 2), rp.Opts(**bad), out=_fake_result(),
                         stream=type("S", (), {"cuda_stream": 0})())
    assert e.value.code == rp.EINVAL


def test_integrate_rejects_unordered_times():
    t = rp.Topology.from_inputs(inputs.toggle_switch())
    s = type("S", (), {"cuda_stream": 0})()
    for times in ([0.0, 2.0, 1.0], [-1.0, 1.0], [], [1.0, 1.0]):
        with pytest.raises(rp.RacError) as e:
            rp.integrate(t, _fake_params(2, 2, 4, 2), times, out=_fake_result(), stream=s)
        assert e.value.code == rp.EINVAL


def test_lane_choices():
    ts = rp.Topology.from_inputs(inputs.toggle_switch())
    assert ts.auto_lanes() >= 1 and ts.lanes_supported(1)
    big = rp.Topology.from_inputs(inputs.erdos_renyi(100, 250, 5))
    assert big.auto_lanes() >= 8
    assert not big.lanes_supported(1)
    assert not ts.lanes_supported(3)


def test_lane_choice_follows_the_call_size():
    # A call that fills the GPU keeps the cost model's lane count; a small
    # one takes more lanes per trajectory, never fewer, and only supported
    # counts.  The figures are the choices that the timings of these
    # networks at 10^3 to 10^6 trajectories favoured.
    er10 = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    base = er10.auto_lanes(rp.FP32)
    assert base == 4
    assert er10.auto_lanes(rp.FP32, 10**6) == base and er10.auto_lanes(rp.FP32, 10**8) == base
    assert er10.auto_lanes(rp.FP32, 10**5) == 8 and er10.auto_lanes(rp.FP32, 10**4) == 16
    ts = rp.Topology.from_inputs(inputs.toggle_switch())
    assert ts.auto_lanes(rp.FP32, 10**4) == 2 * ts.auto_lanes(rp.FP32)
    core = rp.Topology.from_inputs(inputs.dense_core(1004))
    assert core.auto_lanes(rp.FP32, 10**4) == core.auto_lanes(rp.FP32) == 8
    for topo in (er10, ts, core):
        prev = 64
        for n in (1, 10, 10**3, 10**4, 10**5, 10**6, 10**7):
            for prec in (rp.FP32, rp.FP64):
                lanes = topo.auto_lanes(prec, n)
                assert lanes >= topo.auto_lanes(prec) and topo.lanes_supported(lanes, prec)
            lanes = topo.auto_lanes(rp.FP32, n)
            assert lanes <= prev
            prev = lanes
    assert rp.lib().rac_auto_lanes_for(er10.handle, 7, 100) == 0
    assert rp.lib().rac_auto_lanes_for(er10.handle, rp.FP32, -1) == 0


def test_largest_supported_networks_and_one_past_them():
    # FP32: 64 lanes x 8 gene slots bound N at 512; 1,024 edges fit 16 edge
    # slots per lane.  FP64 kernels stop at 4 gene slots with 8 edge slots.
    big = rp.Topology.from_inputs(inputs.erdos_renyi(512, 1024, 7))
    assert big.auto_lanes(rp.FP32) == 64 and big.shape(64, rp.FP32) == (16, 8)
    assert big.auto_lanes(rp.FP64) == 0
    big64 = rp.Topology.from_inputs(inputs.erdos_renyi(256, 400, 7))
    assert big64.auto_lanes(rp.FP64) == 64 and big64.shape(64, rp.FP64) == (8, 4)
    # One gene more than 64 x 8: rejected before anything is enqueued.
    past = rp.Topology.from_inputs(inputs.erdos_renyi(513, 1000, 7))
    assert past.auto_lanes(rp.FP32) == 0
    with pytest.raises(rp.RacError) as e:
        rp.steady_states(past, _fake_params(513, 1000, 4, 2), rp.Opts(), out=_fake_result(),
                         stream=type("S", (), {"cuda_stream": 0})())
    assert e.value.code == rp.EUNSUPPORTED


def test_factor_form_switch_point():
    # FP32 kernels of up to 16 edge slots use the base-free Hill factor; wider
    # FP32 and all FP64 kernels the symmetric one.
    assert [rp.factor_form(rp.FP32, e) for e in (1, 7, 16, 17, 24, 32)] == [1, 1, 1, 0, 0, 0]
    assert [rp.factor_form(rp.FP64, e) for e in (1, 7, 16)] == [0, 0, 0]
    for bad in ((rp.FP32, 0), (5, 4)):
        with pytest.raises(ValueError):
            rp.factor_form(*bad)


def test_valu_ceilings_rejects_bad_arguments_before_touching_the_device():
    lib = rp.lib()
    assert lib.rac_valu_ceilings(None, 5) == rp.EINVAL
    out = (C.c_double * 1)()
    assert lib.rac_valu_ceilings(out, 0) == rp.EINVAL


def test_default_options_and_server_method_check():
    o = rp.Opts().c()
    assert o.method == rp.DP5 and o.rtol == 1e-6 and o.atol == 1e-9
    # Serving step batches are compiled for DP5 only: rejected before any
    # device call.
    with pytest.raises(rp.RacError) as e:
        rp.StepServer(rp.Opts(method=rp.TSIT5), 4, 8, 3)
    assert e.value.code == rp.EUNSUPPORTED


def test_postprocessing_rejects_bad_arguments_before_enqueue():
    L = rp.lib()
    s = None  # never reached: the checks fail first
    fake = 0x1000
    # n_bins / n_levels outside their ranges.
    for bins, levels in ((1, 2), (2000, 2), (64, 1), (64, 5), (3, 4)):
        assert L.rac_level_thresholds(fake, 10, 2, None, bins, levels, fake, fake, s) == rp.EINVAL
    assert L.rac_level_thresholds(fake, 10, 2, None, 512, 4, fake, fake, s) == rp.EUNSUPPORTED
    assert L.rac_level_thresholds(fake, 10, 2, None, 64, 2, None, fake, s) == rp.EINVAL
    # Codes that do not fit 64 bits: 2^64 states of 64 binary genes.
    assert L.rac_discretize(fake, 10, 64, None, 64, 2, fake, None, fake, s) == rp.EUNSUPPORTED
    assert L.rac_discretize(fake, 10, 40, None, 64, 4, fake, None, fake, s) == rp.EUNSUPPORTED
    assert L.rac_discretize(fake, 10, 4, None, 64, 2, fake, None, None, s) == rp.EINVAL
    # Per-set state lists are bounded; capacities are powers of two.
    assert L.rac_multistability(fake, 10, 5000, fake, fake, s) == rp.EUNSUPPORTED
    assert L.rac_multistability(fake, 10, 0, fake, fake, s) == rp.EINVAL
    for cap in (0, 1, 3, 1000, 1 << 31):
        assert L.rac_state_counts(fake, 10, cap, fake, fake, fake, s) == rp.EINVAL
    t = rp.Topology.from_inputs(inputs.toggle_switch())
    p = _fake_params(2, 2, 4, 2)
    v = p.view()
    assert L.rac_normalize(t.handle, C.byref(v), 0, 1, fake, fake, s) == rp.EINVAL
    assert L.rac_normalize(t.handle, C.byref(v), 2, 1, None, fake, s) == rp.EINVAL


def test_plain_c_caller_links_against_the_library():
    # tests/c_abi_demo.c is C99 that calls the ABI with no Python and no C++;
    # built with the library, it loads librac.so and, without arguments,
    # prints its usage before any device call.
    import subprocess
    from paper_2503_18356_amd import build
    exe = build.C_DEMO if os.path.exists(build.C_DEMO) else build.build_c_demo()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage:" in r.stderr, (r.returncode, r.stderr)
