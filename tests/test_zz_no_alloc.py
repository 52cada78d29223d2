"""The steady-state entry point without device allocation, through the C ABI,
against rac_steady_states on the same inputs: bit-identical results on two
calls in a row, the second with a smaller ensemble (the scratch keeps the
first call's counter and descriptor, which the second must clear and
replace)."""
import numpy as np
import pytest

from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _same(a, b):
    for f in ("x", "t_final", "status", "n_acc", "n_rej"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


def _filled(n_traj, n_genes, precision):
    # Sentinels: every output must be written by the call.
    r = rp.alloc_result(n_traj, n_genes, precision)
    r.x.fill_(float("nan"))
    r.t_final.fill_(-1.0)
    r.status.fill_(-1)
    r.n_acc.fill_(-1)
    r.n_rej.fill_(-1)
    return r


@pytest.mark.parametrize("prec", [rp.FP32, rp.FP64])
def test_noalloc_matches_steady_states_twice(prec):
    T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    opts = rp.Opts(precision=prec, ss_rtol=1e-5)
    print(f"[gpu] noalloc prec={prec}", flush=True)
    for n_sets, n_ic in ((3000, 20), (700, 3)):
        dp = rp.sample_params(T, 321 + n_sets, n_sets, n_ic).to_device()
        ref = rp.steady_states(T, dp, opts)
        torch.cuda.synchronize()
        out = _filled(n_sets * n_ic, T.n_genes, prec)
        rp.steady_states_noalloc(T, dp, opts, out)
        torch.cuda.synchronize()
        _same(ref, out)
        assert int((out.status < 0).sum()) == 0


def test_noalloc_with_the_four_wave_spilling_shape():
    # The (10, 4) steady-state kernel, asked for four waves per SIMD, keeps a
    # few registers in per-lane scratch: the entry point without allocation
    # still matches rac_steady_states on it, twice.
    T = rp.Topology.from_inputs(inputs.erdos_renyi(7, 17, 1))
    assert T.shape(2, rp.FP32) == (10, 4)
    opts = rp.Opts(precision=rp.FP32, ss_rtol=1e-5, lanes_per_traj=2)
    print("[gpu] noalloc shape (10, 4)", flush=True)
    for n_sets, n_ic in ((2000, 10), (300, 2)):
        dp = rp.sample_params(T, 55 + n_sets, n_sets, n_ic).to_device()
        ref = rp.steady_states(T, dp, opts)
        torch.cuda.synchronize()
        out = _filled(n_sets * n_ic, T.n_genes, rp.FP32)
        rp.steady_states_noalloc(T, dp, opts, out)
        torch.cuda.synchronize()
        _same(ref, out)
        assert int((out.status < 0).sum()) == 0


def test_noalloc_needs_a_prepared_lane_plan():
    T = rp.Topology.from_inputs(inputs.dense_core(1004))
    dp = rp.sample_params(T, 5, 10, 2).to_device()
    out = _filled(20, T.n_genes, rp.FP32)
    with pytest.raises(rp.RacError) as e:
        rp.steady_states_noalloc(T, dp, rp.Opts(precision=rp.FP32), out)
    assert e.value.code == rp.EINVAL
    rp.steady_states(T, dp, rp.Opts(precision=rp.FP32))
    torch.cuda.synchronize()
    rp.steady_states_noalloc(T, dp, rp.Opts(precision=rp.FP32), out)
    torch.cuda.synchronize()
    assert int((out.status < 0).sum()) == 0


def test_noalloc_replays_from_a_hip_graph():
    # A caller under graph capture: the call recorded once into a HIP graph
    # (torch's capture on its own stream) and replayed three times, with eager
    # solves and synchronisations between the replays; every replay must
    # equal the eager call bit for bit (the scratch counters are cleared by a
    # kernel inside the graph, not by a memset node).
    T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    opts = rp.Opts(precision=rp.FP32, ss_rtol=1e-5)
    dp = rp.sample_params(T, 777, 2000, 10).to_device()
    print("[gpu] noalloc under graph capture", flush=True)
    ref = rp.steady_states(T, dp, opts)  # also puts the lane plan on the device
    torch.cuda.synchronize()
    out = _filled(20000, T.n_genes, rp.FP32)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rp.steady_states_noalloc(T, dp, opts, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    _same(ref, out)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rp.steady_states_noalloc(T, dp, opts, out)
    other = rp.sample_params(T, 778, 500, 4).to_device()
    for rep in range(3):
        fresh = _filled(20000, T.n_genes, rp.FP32)
        for f in ("x", "t_final", "status", "n_acc", "n_rej"):
            getattr(out, f).copy_(getattr(fresh, f))
        eager = rp.steady_states(T, other, opts)
        torch.cuda.synchronize()
        assert int((eager.status < 0).sum()) == 0
        g.replay()
        torch.cuda.synchronize()
        _same(ref, out)
