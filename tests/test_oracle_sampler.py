"""Pins of the oracle's full sampler (Sec. 2.1.2): Sobol' and Latin-hypercube
unit-cube generators and the in-degree-aware half-functional threshold rule.

Checked against what the constructions guarantee: the count of primitive
polynomials of each degree (phi(2^s - 1) / s), one point per elementary
interval in every dimension (and in the first two dimensions jointly), the
t-value bound of two-dimensional projections, the Gray-code generation of
the same point set, bijective permutations and one point per stratum for the
Latin hypercube, the closed-form median for unregulated sources, and an
independent numpy Monte Carlo estimate of the regulated medians.
"""
import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from tests.test_oracle_pins import net_of


def _phi(n):
    out, m, f = n, n, 2
    while f * f <= m:
        if m % f == 0:
            while m % f == 0:
                m //= f
            out -= out // f
        f += 1
    if m > 1:
        out -= out // m
    return out


@pytest.mark.parametrize("s", range(1, 15))
def test_primitive_polynomial_counts(s):
    assert oracle.primitive_count(s) == _phi(2**s - 1) // s


def _points(q, m):
    return np.array([oracle.sobol_u32(i, q) for i in range(2**m)], np.uint64)


@pytest.mark.parametrize("q", [0, 1, 2, 5, 17, 100, 1000, 4000])
def test_sobol_each_dimension_is_a_0m1_net(q):
    m = 10
    top = _points(q, m) >> np.uint64(32 - m)
    assert sorted(top.tolist()) == list(range(2**m))


def test_sobol_first_two_dimensions_form_a_0m2_net():
    m = 8
    x, y = _points(0, m), _points(1, m)
    for j in range(m + 1):
        cells = (x >> np.uint64(32 - j)) * np.uint64(2 ** (m - j)) + (y >> np.uint64(32 - (m - j)))
        assert len(set(cells.tolist())) == 2**m, j


def _degree_of_dim(q):
    # Dimension q >= 1 uses the (q-1)-th primitive polynomial by degree.
    s, seen = 1, 0
    while seen + oracle.primitive_count(s) < q:
        seen += oracle.primitive_count(s)
        s += 1
    return s


@pytest.mark.parametrize("q1,q2", [(1, 2), (3, 7), (10, 40), (50, 300)])
def test_sobol_pairs_meet_the_t_value_bound(q1, q2):
    m = 10
    t = _degree_of_dim(q1) - 1 + _degree_of_dim(q2) - 1
    x, y = _points(q1, m), _points(q2, m)
    # A (t, m, 2)-net: every elementary interval of volume 2^(t - m) holds 2^t points.
    for j in range(m - t + 1):
        cells = (x >> np.uint64(32 - j)) * np.uint64(2 ** (m - t - j)) + (y >> np.uint64(32 - (m - t - j)))
        assert np.all(np.bincount(cells.astype(np.int64), minlength=2 ** (m - t)) == 2**t), (j, t)


def test_sobol_gray_code_gives_the_same_points():
    # Antonov-Saleev: x_{i+1} = x_i ^ V[lowest zero bit of i] walks the same
    # 2^m points in Gray-code order; V[b] is the direct point at 2^b.
    m = 9
    for q in (0, 3, 33):
        V = [oracle.sobol_u32(2**b, q) for b in range(m)]
        x, seq = 0, [0]
        for i in range(2**m - 1):
            c = (~i & (i + 1)).bit_length() - 1
            x ^= V[c]
            seq.append(x)
        assert sorted(seq) == sorted(_points(q, m).tolist())


@pytest.mark.parametrize("n", [1, 2, 7, 100, 1000, 65539])
def test_lhs_permutation_is_a_bijection(n):
    perm = [oracle.lhs_perm(11, 0, 5, n, i) for i in range(n)]
    assert sorted(perm) == list(range(n))


def test_lhs_sampler_one_point_per_stratum():
    net = net_of(inputs.toggle_switch())
    n = 64
    r = oracle.Ranges(g_min=0.0, g_max=float(n), k_min=0.0, k_max=float(n), method=oracle.LHS)
    prm = oracle.sample(net, 3, n, 16, ranges=r)
    for row in (prm.G, prm.k):
        for dim in row:
            assert sorted(np.floor(dim).astype(int).tolist()) == list(range(n))
            frac = dim - np.floor(dim)          # uniform offset inside the stratum
            assert 0.35 < frac.mean() < 0.65 and frac.std() > 0.2
    # Initial conditions: a hypercube over the 16 conditions.
    for i in range(2):
        assert sorted(np.floor(prm.ic[:, i] * 16).astype(int).tolist()) == list(range(16))


def test_sobol_sampler_is_stratified_and_shifted_by_seed():
    net = net_of(inputs.toggle_switch())
    m = 8
    r = oracle.Ranges(g_min=0.0, g_max=1.0, method=oracle.SOBOL)
    a = oracle.sample(net, 1, 2**m, 1, ranges=r)
    b = oracle.sample(net, 2, 2**m, 1, ranges=r)
    for G in (a.G, b.G):
        for dim in G:
            assert sorted(np.floor(dim.astype(np.float64) * 2**m).astype(int).tolist()) == list(range(2**m))
    assert not np.array_equal(a.G, b.G)


@pytest.mark.parametrize("method", [oracle.SOBOL, oracle.LHS, oracle.UNIFORM])
def test_full_sampler_index_addressable(method):
    net = net_of(inputs.erdos_renyi(6, 10, 4))
    r = oracle.Ranges(method=method, threshold_rule=oracle.HALF_FUNCTIONAL, lhs_total=100,
                      hf_samples=4096)
    whole = oracle.sample(net, 7, 100, 3, ranges=r)
    part = oracle.sample(net, 7, 40, 3, set_begin=60, ranges=r)
    for f in ("G", "k", "T", "lam", "n"):
        assert np.array_equal(getattr(whole, f)[:, 60:], getattr(part, f))


def test_half_functional_unregulated_median_is_the_prior_median():
    assert oracle.hf_median(0, 0) == pytest.approx(1010.0 / 11.0, rel=1e-15)


def _numpy_one_step_median(n_act, n_inh, S=400_000, seed=99):
    # Independent estimate with numpy's own generator and the literal Eq. 2.
    rng = np.random.default_rng(seed)
    M0 = 1010.0 / 11.0
    x = rng.uniform(1, 100, S) / rng.uniform(0.1, 1, S)
    for e in range(n_act + n_inh):
        B = rng.uniform(1, 100, S) / rng.uniform(0.1, 1, S)
        T = M0 * rng.uniform(0.02, 1.98, S)
        n = rng.integers(1, 7, S).astype(float)
        if e < n_act:
            lam = rng.uniform(1, 100, S)
        else:
            lam = 1.0 / rng.uniform(1, 100, S)
        hs = (T**n + lam * B**n) / (T**n + B**n)
        x *= hs / lam if e < n_act else hs
    return float(np.median(x))


@pytest.mark.parametrize("na,nh", [(1, 0), (0, 1), (1, 1), (2, 0)])
def test_half_functional_median_matches_independent_monte_carlo(na, nh):
    got = oracle.hf_median(na, nh)
    want = _numpy_one_step_median(na, nh)
    assert abs(got - want) / want < 0.03, (got, want)


def test_half_functional_medians_order_and_thresholds():
    M = {c: oracle.hf_median(*c) for c in ((0, 0), (1, 0), (0, 1), (2, 0))}
    assert M[(1, 0)] < M[(0, 0)] and M[(0, 1)] < M[(0, 0)] and M[(2, 0)] < M[(1, 0)]
    # Edges leaving a gene use that gene's in-degree class.
    net = net_of(inputs.toggle_switch_self_activation())
    r = oracle.Ranges(threshold_rule=oracle.HALF_FUNCTIONAL)
    prm = oracle.sample(net, 5, 2000, 1, ranges=r)
    for e in range(net.n_edges):
        src = net.src[e]
        na = int(np.sum((net.dst == src) & (net.sign > 0)))
        nh = int(np.sum((net.dst == src) & (net.sign < 0)))
        Ms = oracle.hf_median(na, nh)
        Te = prm.T[e].astype(np.float64)
        assert Te.min() >= 0.02 * Ms * (1 - 1e-6) and Te.max() <= 1.98 * Ms * (1 + 1e-6)
        assert abs(np.median(Te) / Ms - 1.0) < 0.05
