"""The parity adjudication itself (tests/parity.py), on the CPU.

Fake "device" results are built from oracle results with planted errors, and
the report must reject each error that the 1e-4 bar forbids and accept only
the three capped excuses it defines.
"""
import numpy as np

import oracle
from paper_2503_18356_amd import inputs
from tests import parity


def _case(n_sets=40, n_ic=5):
    topo = inputs.erdos_renyi(6, 12, 8)
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    prm = oracle.sample(net, 21, n_sets, n_ic)
    opts = oracle.Opts(ss_rtol=1e-5)
    ref = oracle.steady_states(net, prm, opts, n_threads=4)
    return net, prm, opts, ref, n_ic


def _report(net, prm, opts, ref, n_ic, x, st):
    traj = np.arange(ref.x.shape[0])
    return parity.compare_steady(net, prm, opts, traj, x, ref.x, n_ic, st, ref.status)


def test_identical_results_pass():
    net, prm, opts, ref, n_ic = _case()
    rep = _report(net, prm, opts, ref, n_ic, ref.x.copy(), ref.status.copy())
    assert rep.ok() and rep.max_err == 0.0 and rep.status_mismatch == 0


def test_error_above_tolerance_fails():
    net, prm, opts, ref, n_ic = _case()
    x = ref.x.copy()
    gk = parity.gk_of(prm, np.arange(x.shape[0]), n_ic)
    # 3e-4 of G/k on one gene of one converged trajectory: no excuse applies
    # (well-conditioned fixed point, same basin).
    i = int(np.flatnonzero(ref.status == oracle.CONVERGED)[0])
    x[i, 0] += 3e-4 * gk[i, 0]
    rep = _report(net, prm, opts, ref, n_ic, x, ref.status.copy())
    assert not rep.ok() and rep.unexcused


def test_unsolved_status_mismatch_fails():
    net, prm, opts, ref, n_ic = _case()
    st = ref.status.copy()
    st[3] = oracle.MAX_STEPS
    rep = _report(net, prm, opts, ref, n_ic, ref.x.copy(), st)
    assert not rep.ok() and rep.unexcused[0][2] == "status"


def test_status_mismatch_must_agree_with_the_state():
    # CONVERGED vs T_END is excused only where the claim agrees with the
    # claimed state in FP64.  Claiming T_END for a trajectory whose state is
    # steady (a steady test that never fires) fails; a trajectory that hovers
    # near its fixed point under the absolute criterion, whose status the
    # oracle itself changes when x0 moves by 1e-5, is excused.
    net, prm, opts, ref, n_ic = _case()
    st = ref.status.copy()
    early = np.flatnonzero((st == oracle.CONVERGED) & (ref.t_final < 50.0))
    # What a never-firing test returns: the state at t_end, deep in convergence.
    deep = oracle.steady_states(net, prm, oracle.Opts(ss_rtol=0.0, ss_atol=1e-13), n_threads=4)
    x = ref.x.copy()
    x[early[0]] = deep.x[early[0]]
    st[early[0]] = oracle.T_END
    rep = _report(net, prm, opts, ref, n_ic, x, st)
    assert not rep.ok() and rep.unexcused[0][2] == "status"
    # Absolute FP64 criterion on a 10-gene network: find a trajectory whose
    # oracle status changes with x0 * (1 + 1e-5), and claim the other status.
    topo = inputs.erdos_renyi(10, 25, 1002)
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    prm = oracle.sample(net, 77, 64, 5)
    n_ic = 5
    o0 = oracle.Opts(ss_rtol=0.0)
    base = oracle.steady_states(net, prm, o0, n_threads=4)
    pert = oracle.Params(prm.G, prm.k, prm.T, prm.lam, prm.n, (prm.ic * np.float32(1 + 1e-5)).astype(np.float32))
    moved = oracle.steady_states(net, pert, o0, n_threads=4)
    cand = np.flatnonzero((base.status != moved.status) & np.isin(base.status, (0, 1)) &
                          np.isin(moved.status, (0, 1)))
    assert cand.size > 0
    i = int(cand[0])
    st0 = base.status.copy()
    st0[i] = moved.status[i]
    x0 = base.x.copy()
    x0[i] = moved.x[i]
    traj = np.arange(base.x.shape[0])
    rep = parity.compare_steady(net, prm, o0, traj, x0, base.x, n_ic, st0, base.status)
    assert rep.ok() and rep.status_mismatch == 1, rep


def test_no_slow_excuse_without_convergence():
    # A large difference on a trajectory both sides ended at T_END is never
    # excused as a slow fixed point.
    net, prm, opts, ref, n_ic = _case()
    opts_short = oracle.Opts(ss_rtol=1e-5, t_end=0.5)
    short = oracle.steady_states(net, prm, opts_short, n_threads=4)
    assert np.all(short.status == oracle.T_END)
    x = short.x.copy()
    gk = parity.gk_of(prm, np.arange(x.shape[0]), n_ic)
    x[0, 1] += 1e-2 * gk[0, 1]
    traj = np.arange(x.shape[0])
    rep = parity.compare_steady(net, prm, opts_short, traj, x, short.x, n_ic, short.status, short.status)
    assert not rep.ok() and rep.slow == 0
