"""Pins of the post-processing oracle (CPU).

Each function is checked against something other than itself: the FP64
value of x k / G, the classic two-class Otsu criterion written with class
weights and means (a different formula with the same maximiser), exhaustive
search on tiny histograms, symmetric and separated-mode histograms whose
thresholds are known, string concatenation of levels, and Python sets and
counters.
"""
import itertools

import numpy as np
import pytest

from oracle import postproc as pp


def test_normalize_is_x_over_g_by_k():
    rng = np.random.default_rng(1)
    N, P, n_ic = 5, 7, 3
    G = rng.uniform(1, 100, (N, P)).astype(np.float32)
    k = rng.uniform(0.1, 1, (N, P)).astype(np.float32)
    u = rng.uniform(0, 1, (P * n_ic, N))
    p = np.arange(P * n_ic) // n_ic
    x = (u * (G / k).T[p]).astype(np.float32)
    y = pp.normalize(x, G, k, n_ic)
    exact = x.astype(np.float64) * k.T[p].astype(np.float64) / G.T[p].astype(np.float64)
    assert y.dtype == np.float32
    assert np.all(np.abs(y - exact) <= 2 * np.spacing(np.float32(1)) * np.abs(exact) + 1e-30)
    # x = G/k maps to 1 (up to rounding), x = 0 to 0.
    y1 = pp.normalize((G / k).T[p].astype(np.float32), G, k, n_ic)
    assert np.allclose(y1, 1.0, atol=1e-6)
    assert np.all(pp.normalize(np.zeros_like(x), G, k, n_ic) == 0)


def test_normalize_time_series_rows():
    G = np.array([[2.0, 4.0]], np.float32)   # one gene, two sets
    k = np.array([[1.0, 1.0]], np.float32)
    x = np.array([[1.0], [1.0], [2.0], [2.0]], np.float32)  # n_ic=1, n_t=2
    y = pp.normalize(x, G, k, n_ic=1, n_t=2)
    assert y.ravel().tolist() == [0.5, 0.5, 0.5, 0.5]


def test_bins_and_histogram():
    y = np.array([[0.0, 0.5, 0.99, 1.0, 1.5, -0.2]], np.float32)
    assert pp.bins_of(y, 4).ravel().tolist() == [0, 2, 3, 3, 3, 0]
    h = pp.histogram(np.vstack([y, y]), 4, status=np.array([0, 1]))
    assert h.tolist() == [2, 0, 1, 3] and h.sum() == 6


def _otsu_two_class_classic(hist):
    # Between-class variance w0 w1 (mu0 - mu1)^2 with class weights and means.
    b = np.arange(len(hist))
    best, arg = -1, None
    for t in range(1, len(hist)):
        w0, w1 = hist[:t].sum(), hist[t:].sum()
        if w0 == 0 or w1 == 0:
            v = 0.0
        else:
            m0 = (b[:t] * hist[:t]).sum() / w0
            m1 = (b[t:] * hist[t:]).sum() / w1
            v = w0 * w1 * (m0 - m1) ** 2
        if v > best + 1e-9 * abs(best):
            best, arg = v, t
    return arg


@pytest.mark.parametrize("seed", range(8))
def test_two_level_threshold_matches_classic_otsu(seed):
    rng = np.random.default_rng(seed)
    hist = rng.integers(0, 1000, 32)
    hist[rng.integers(0, 32, 4)] += rng.integers(1000, 5000, 4)
    assert pp.thresholds(hist, 2) == [_otsu_two_class_classic(hist)]


def test_symmetric_bimodal_threshold_is_the_middle():
    B = 20
    b = np.arange(B)
    hist = (1000 * (np.exp(-0.5 * ((b - 3) / 1.5) ** 2) + np.exp(-0.5 * ((b - 16) / 1.5) ** 2))).astype(np.int64)
    t = pp.thresholds(hist, 2)[0]
    assert 9 <= t <= 10          # the classes split at the valley


def test_three_levels_fall_in_the_gaps():
    hist = np.zeros(30, np.int64)
    hist[2:5] = 100
    hist[14:17] = 100
    hist[25:28] = 100
    t1, t2 = pp.thresholds(hist, 3)
    assert 5 <= t1 <= 14 and 17 <= t2 <= 25


def test_thresholds_exhaustive_on_tiny_histograms():
    rng = np.random.default_rng(5)
    for _ in range(20):
        hist = rng.integers(0, 9, 6)
        for L in (2, 3, 4):
            got = pp.thresholds(hist, L)
            vals = {t: pp.otsu_objective(hist, t) for t in itertools.combinations(range(1, 6), L - 1)}
            m = max(vals.values())
            assert tuple(got) == min(t for t, v in vals.items() if v == m)


def test_levels_and_codes():
    y = np.array([[0.1, 0.9], [0.9, 0.1], [0.6, 0.6], [0.0, 1.0]], np.float32)
    lv = pp.levels(y, 10, [5])
    assert lv.tolist() == [[0, 1], [1, 0], [1, 1], [0, 1]]
    c = pp.codes(lv, 2)
    assert [int(v) for v in c] == [int("".join(map(str, r)), 2) for r in lv.tolist()]
    st = np.array([0, 1, 0, 0])
    lv2 = pp.levels(y, 10, [5], status=st)
    assert lv2[1].tolist() == [255, 255]
    assert pp.codes(lv2, 2, status=st)[1] == pp.NO_STATE
    # Three levels: base-3 digits, gene 0 first.
    lv3 = pp.levels(y, 10, [3, 7])
    assert [int(v) for v in pp.codes(lv3, 3)] == [int("".join(map(str, r)), 3) for r in lv3.tolist()]


def test_multistability_and_state_counts():
    rng = np.random.default_rng(3)
    P, n_ic = 50, 7
    code = rng.integers(0, 4, P * n_ic).astype(np.uint64)
    code[rng.integers(0, P * n_ic, 20)] = pp.NO_STATE
    n, states = pp.multistability(code, P, n_ic)
    for p in range(P):
        s = {int(v) for v in code[p * n_ic:(p + 1) * n_ic] if v != pp.NO_STATE}
        assert n[p] == len(s)
        assert [int(v) for v in states[p, :n[p]]] == sorted(s)
        assert np.all(states[p, n[p]:] == pp.NO_STATE)
    keys, counts = pp.state_counts(code)
    assert counts.sum() == np.sum(code != pp.NO_STATE)
    for kk, cc in zip(keys, counts):
        assert cc == np.sum(code == kk)
