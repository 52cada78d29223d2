"""Pins of the oracle's Runge-Kutta tableaus and of its Tsitouras 5(4) solver.

The order conditions of explicit Runge-Kutta methods (Butcher trees up to
order 5) are checked directly on the oracle's own coefficients: the fifth-order
weights of each pair must satisfy all 17 conditions of order <= 5, the
embedded weights the 8 conditions of order <= 4 but not order 5.  Then the
Tsit5 integrator is pinned like DP5: fixed-step convergence order, the closed
form of an unregulated gene, fixed points and an independent RK4.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from tests.test_oracle_pins import _closed_free, hand_params, net_of

METHODS = [oracle.DP5, oracle.TSIT5]


def _order_conditions(A, b, c):
    """Residuals of the order conditions (rooted trees) of orders 1..5."""
    one = np.ones_like(b)
    Ac = A @ c
    by_order = {
        1: [b @ one - 1],
        2: [b @ c - 1 / 2],
        3: [b @ c**2 - 1 / 3, b @ Ac - 1 / 6],
        4: [b @ c**3 - 1 / 4, b @ (c * Ac) - 1 / 8, b @ (A @ c**2) - 1 / 12,
            b @ (A @ Ac) - 1 / 24],
        5: [b @ c**4 - 1 / 5, b @ (c**2 * Ac) - 1 / 10, b @ (c * (A @ c**2)) - 1 / 15,
            b @ (c * (A @ Ac)) - 1 / 30, b @ Ac**2 - 1 / 20, b @ (A @ c**3) - 1 / 20,
            b @ (A @ (c * Ac)) - 1 / 40, b @ (A @ (A @ c**2)) - 1 / 60,
            b @ (A @ (A @ Ac)) - 1 / 120],
    }
    return {k: np.abs(np.array(v)) for k, v in by_order.items()}


@pytest.mark.parametrize("method", METHODS)
def test_tableau_order_conditions(method):
    A, b, bh, c = oracle.tableau(method)
    assert np.allclose(c, A.sum(axis=1), atol=1e-15)          # row sums are the nodes
    assert np.array_equal(A[6, :6], b[:6]) and b[6] == 0      # first same as last
    assert np.all(np.triu(A) == 0)                            # explicit
    r5 = _order_conditions(A, b, c)
    assert max(v.max() for v in r5.values()) < 1e-13, r5
    r4 = _order_conditions(A, bh, c)
    assert max(r4[k].max() for k in (1, 2, 3, 4)) < 1e-13, r4
    assert r4[5].max() > 1e-5                                 # genuinely order 4


def test_tsit5_nodes():
    _, _, _, c = oracle.tableau(oracle.TSIT5)
    want = [0.0, 0.161, 0.327, 0.9, 0.9800255409045097, 1.0, 1.0]
    assert np.allclose(c, want, rtol=0, atol=2e-15)


def test_tsit5_fifth_order_on_nonlinear_motif():
    # Tsit5's fifth-order error constant is small, so at these steps the
    # sixth-order term still shows and the ratios approach 2^5 = 32 from
    # above; a wrong coefficient drops the order and the ratio to <= 16.
    t = inputs.toggle_switch_self_activation()
    net = net_of(t)
    prm = oracle.sample(net, seed=3, n_sets=8, n_ic=1)
    opts = oracle.Opts(t_end=8.0, method=oracle.TSIT5)
    ratios = []
    for traj in range(8):
        xs = [oracle.dp5_fixed(net, prm, traj, m, opts)[0] for m in (64, 128, 256)]
        ratios.append(np.max(np.abs(xs[0] - xs[1])) / np.max(np.abs(xs[1] - xs[2])))
    ratios = np.array(ratios)
    assert 28 < np.median(ratios) < 52, ratios
    assert np.sum((ratios > 24) & (ratios < 64)) >= 6, ratios
    # Against the independent RK4 reference the same motif converges at 2^5.
    ref = oracle.rk4(net, prm, 2e-4, [8.0], opts)[:, 0, :]
    e = [np.array([np.max(np.abs(oracle.dp5_fixed(net, prm, i, m, opts)[0] - ref[i]))
                   for i in range(8)]) for m in (32, 64)]
    assert 26 < np.median(e[0] / e[1]) < 56


def test_tsit5_fifth_order_on_linear_decay():
    net = net_of(inputs.unregulated(1))
    prm = hand_params(net, G=[0.0], k=[1.0], ic=[[1.0]])
    opts = oracle.Opts(t_end=4.0, ic_absolute=1, method=oracle.TSIT5)
    e = [abs(oracle.dp5_fixed(net, prm, 0, m, opts)[0][0] - math.exp(-4.0)) for m in (64, 128, 256)]
    assert 28 < e[0] / e[1] < 40 and 28 < e[1] / e[2] < 40


def test_tsit5_embedded_error_estimate_scales_as_h5():
    net = net_of(inputs.toggle_switch())
    prm = oracle.sample(net, seed=5, n_sets=1, n_ic=1)
    opts = oracle.Opts(t_end=0.5, method=oracle.TSIT5)
    e1, e2, e4 = (oracle.dp5_fixed(net, prm, 0, m, opts)[1] for m in (1, 2, 4))
    assert 16 < e2 / e4 < 64 and 8 < e1 / e2 < 128


def test_tsit5_unregulated_time_series_matches_closed_form():
    net = net_of(inputs.unregulated(3))
    prm = oracle.sample(net, seed=7, n_sets=20, n_ic=3)
    tk = np.linspace(0, 100, 101)
    res = oracle.time_series(net, prm, tk, oracle.Opts(method=oracle.TSIT5))
    for traj in range(60):
        p, c = divmod(traj, 3)
        G, k = prm.G[:, p].astype(np.float64), prm.k[:, p].astype(np.float64)
        want = _closed_free(G, k, prm.ic[c].astype(np.float64) * G / k, tk)
        assert np.all(np.abs(res.x[traj] - want) <= 10 * (1e-6 * np.abs(want) + 1e-9))


def test_tsit5_steady_states_are_fixed_points():
    net = net_of(inputs.toggle_switch())
    prm = oracle.sample(net, seed=2001, n_sets=30, n_ic=2)
    opts = oracle.Opts(rtol=1e-12, atol=1e-14, ss_atol=1e-8, t_end=2000.0, max_steps=10**6,
                       method=oracle.TSIT5)
    res = oracle.steady_states(net, prm, opts)
    conv = np.flatnonzero(res.status == oracle.CONVERGED)
    assert conv.size >= 50
    for traj in conv:
        assert np.max(np.abs(oracle.rhs(net, prm, traj // 2, res.x[traj]))) <= 1e-8


@pytest.mark.parametrize("builder", [inputs.toggle_switch, lambda: inputs.erdos_renyi(3, 5, 9)])
def test_tsit5_rk4_cross_check(builder):
    net = net_of(builder())
    prm = oracle.sample(net, seed=44, n_sets=6, n_ic=2)
    tk = np.array([0.0, 1.0, 10.0, 50.0, 200.0])
    opts = oracle.Opts(rtol=1e-10, atol=1e-12, method=oracle.TSIT5)
    ts = oracle.time_series(net, prm, tk, opts)
    ref = oracle.rk4(net, prm, 1e-3, tk, opts)
    for traj in range(12):
        gk = prm.G[:, traj // 2].astype(np.float64) / prm.k[:, traj // 2]
        assert np.max(np.abs(ts.x[traj] - ref[traj]) / gk) < 1e-7


def test_unknown_method_is_rejected():
    net = net_of(inputs.toggle_switch())
    prm = oracle.sample(net, seed=1, n_sets=1, n_ic=1)
    with pytest.raises(ValueError):
        oracle.steady_states(net, prm, oracle.Opts(method=7))
    with pytest.raises(ValueError):
        oracle.tableau(2)
