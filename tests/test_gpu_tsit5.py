"""GPU parity of the Tsitouras 5(4) kernels against the oracle's Tsit5.

Same cases and metric as the Dormand-Prince parity tests: steady states of
the toggle switch (FP32 and FP64), a 1 %-style subsample of the 10-gene
network, every lane count of the 22-gene network, and the 22-gene time
series (cubic Hermite output between steps).
"""
import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp
from tests import parity
from tests.test_gpu_parity import THREADS, Case, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def tsit5(prec, **kw):
    return rp.Opts(precision=prec, method=rp.TSIT5, **kw)


@pytest.mark.parametrize("prec", [rp.FP64, rp.FP32])
def test_tsit5_toggle_switch(prec):
    case = Case(inputs.toggle_switch(), 2001, 1000, 10)
    out, ref, rep = case.check(tsit5(prec), label="TS tsit5")
    if prec == rp.FP64:
        assert rep.p99_rel < 1e-9 and rep.max_err < 1e-5


def test_tsit5_er10_subsample():
    case = Case(inputs.erdos_renyi(10, 25, 1002), 2002, 2000, 100)
    case.check(tsit5(rp.FP32), sample=4000, seed=2, label="ER10 tsit5")


def test_tsit5_every_lane_count_core22():
    case = Case(inputs.dense_core(1004), 78, 64, 5)
    for lanes in (1, 2, 4, 8, 16, 32, 64):
        if case.T.lanes_supported(lanes, rp.FP32):
            case.check(tsit5(rp.FP32, lanes_per_traj=lanes), label=f"tsit5 lanes={lanes}")


def test_tsit5_time_series_dense_core():
    case = Case(inputs.dense_core(1004), 2004, 300, 10)
    tk = np.linspace(0.0, 100.0, 101)
    opts = tsit5(rp.FP32)
    say("[gpu] tsit5 time series core22")
    out = rp.integrate(case.T, case.dp, tk, opts)
    torch.cuda.synchronize()
    traj = np.sort(np.random.default_rng(4).choice(case.n_traj, 300, replace=False))
    ref = oracle.time_series(case.net, case.op, tk, case.oracle_opts(opts), traj_ids=traj,
                             n_threads=THREADS)
    assert np.all(out.status.cpu().numpy()[traj] == rp.T_END)
    err, _ = parity.compare_series(case.op, traj, out.x.cpu().numpy()[traj], ref.x, case.n_ic)
    say("    max normalised error per time (every 10th):", np.array2string(err[::10], precision=1))
    assert err.max() <= parity.TOL, (err.argmax(), err.max())


def test_tsit5_and_dp5_reach_the_same_states():
    # Fixed points do not depend on the integrator: the two methods' FP32
    # steady states agree within the parity tolerance (basin flips aside).
    case = Case(inputs.erdos_renyi(10, 25, 1002), 31, 500, 4)
    a = case.gpu(rp.Opts(precision=rp.FP32))
    b = case.gpu(tsit5(rp.FP32))
    gk = (case.op.G / case.op.k).T.astype(np.float64)[np.arange(case.n_traj) // case.n_ic]
    d = np.abs(a.x.cpu().numpy() - b.x.cpu().numpy()) / gk
    flips = np.sum(d.max(axis=1) > 0.5)
    say(f"    tsit5 vs dp5: {flips} basin flips, p99 normalised diff "
        f"{np.percentile(d.max(axis=1), 99):.2e}")
    assert flips <= 0.005 * case.n_traj
    assert np.percentile(d.max(axis=1), 99) < 1e-4


def test_tsit5_uneven_batch():
    # The batch call with the Tsitouras pair: each network's results equal
    # its one-network solve at the batch's lane count, and match the
    # oracle's Tsit5.
    topos = inputs.uneven_batch(1005, n_networks=6, n_min=5, n_max=50)
    cases = [Case(t, 3100 + i, 50 + 9 * i, 3) for i, t in enumerate(topos)]
    opts = tsit5(rp.FP32)
    say("[gpu] tsit5 batch of", [t.n_genes for t in topos])
    outs = rp.steady_states_batch([(c.T, c.dp) for c in cases], opts)
    torch.cuda.synchronize()
    total = sum(c.n_traj for c in cases)
    for c, o in zip(cases, outs):
        single = c.gpu(tsit5(rp.FP32, lanes_per_traj=c.T.auto_lanes(rp.FP32, total)))
        assert torch.equal(single.x, o.x), c.topo.name
        traj = np.arange(min(c.n_traj, 60))
        ref = oracle.steady_states(c.net, c.op, c.oracle_opts(opts), traj_ids=traj, n_threads=THREADS)
        rep = parity.compare_steady(c.net, c.op, c.oracle_opts(opts), traj, o.x.cpu().numpy()[traj],
                                    ref.x, c.n_ic, o.status.cpu().numpy()[traj], ref.status)
        assert rep.ok(), (c.topo.name, rep)
