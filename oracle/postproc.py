"""Oracle for the post-processing of steady states (test infrastructure only).

Plain numpy and Python loops, written from the paper's description of its
analysis functions (Sec. 2.1.4 and Sec. 3.1): states are normalised by the
maximal expression G/k of each gene under its parameter set, discretised into
levels from the global distribution of normalised values, concatenated into a
state per (parameter set, initial condition), and summarised per parameter
set (number of distinct states: its multistability) and globally (state
frequencies).  The paper does not give the levels algorithm; this module
implements the reading used throughout this repository:

- y = (x * k) / G, each operation rounded to FP32;
- bin b = min(floor(y * B), B - 1) after clamping y to [0, 1] (NaN to 0), FP32;
- a histogram over all genes and all included rows (rows whose status is
  CONVERGED when statuses are given);
- L levels from the thresholds 0 < t_1 < ... < t_{L-1} < B (bin indices) that
  maximise sum_k S_k^2 / W_k over the classes [t_k, t_{k+1}) (W_k = count,
  S_k = sum of bin indices; empty classes add 0), which is Otsu's
  between-class variance up to constants; evaluated in FP64 in class order,
  the first maximum in lexicographic order wins;
- level = number of thresholds <= b; state code = sum_i level_i L^(N-1-i)
  (gene 0 most significant), NO_STATE for excluded rows.

Only tests/, the smoke test and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import collections
import itertools

import numpy as np

NO_STATE = np.uint64(0xFFFFFFFFFFFFFFFF)
NO_LEVEL = 255
CONVERGED = 0


def normalize(x, G, k, n_ic: int, n_t: int = 1):
    """x[rows][N] with row = (p * n_ic + c) * n_t + j; G, k [N][P] float32."""
    x = np.asarray(x, np.float32)
    rows = x.shape[0]
    p = np.arange(rows) // n_t // n_ic
    kk = np.asarray(k, np.float32).T[p]
    GG = np.asarray(G, np.float32).T[p]
    return (x * kk) / GG  # float32 * float32 / float32, each rounded


def bins_of(y, n_bins: int):
    y = np.asarray(y, np.float32)
    # fmax/fmin ignore NaN, so NaN counts as 0.
    yc = np.fmin(np.fmax(y, np.float32(0)), np.float32(1))
    b = np.floor(yc * np.float32(n_bins)).astype(np.int64)
    return np.minimum(b, n_bins - 1)


def histogram(y, n_bins: int, status=None):
    b = bins_of(y, n_bins)
    if status is not None:
        b = b[np.asarray(status) == CONVERGED]
    return np.bincount(b.ravel(), minlength=n_bins).astype(np.int64)


def otsu_objective(hist, thresholds):
    """sum_k S_k^2 / W_k over the classes cut at the given bin indices."""
    B = len(hist)
    cuts = [0, *thresholds, B]
    total = 0.0
    for k in range(len(cuts) - 1):
        lo, hi = cuts[k], cuts[k + 1]
        W = int(sum(int(hist[b]) for b in range(lo, hi)))
        S = int(sum(b * int(hist[b]) for b in range(lo, hi)))
        term = (float(S) * float(S)) / float(W) if W > 0 else 0.0
        total = total + term
    return total


def thresholds(hist, n_levels: int):
    """Multi-level Otsu thresholds (bin indices), first maximum wins."""
    B = len(hist)
    best, arg = -1.0, None
    for t in itertools.combinations(range(1, B), n_levels - 1):
        v = otsu_objective(hist, t)
        if v > best:
            best, arg = v, t
    return list(arg)


def levels(y, n_bins: int, thr, status=None):
    b = bins_of(y, n_bins)
    lv = np.zeros(b.shape, np.int64)
    for t in thr:
        lv += (b >= t)
    lv = lv.astype(np.uint8)
    if status is not None:
        lv[np.asarray(status) != CONVERGED] = NO_LEVEL
    return lv


def codes(lv, n_levels: int, status=None):
    lv = np.asarray(lv)
    out = np.full(lv.shape[0], NO_STATE, np.uint64)
    for r in range(lv.shape[0]):
        if status is not None and status[r] != CONVERGED:
            continue
        c = 0
        for i in range(lv.shape[1]):
            c = c * n_levels + int(lv[r, i])
        out[r] = np.uint64(c)
    return out


def multistability(code, n_sets: int, n_ic: int):
    """(number of distinct states per set, sorted distinct states padded with
    NO_STATE to n_ic) ignoring NO_STATE rows."""
    code = np.asarray(code, np.uint64).reshape(n_sets, n_ic)
    n = np.zeros(n_sets, np.int32)
    states = np.full((n_sets, n_ic), NO_STATE, np.uint64)
    for p in range(n_sets):
        u = sorted({int(v) for v in code[p] if v != NO_STATE})
        n[p] = len(u)
        states[p, :len(u)] = u
    return n, states


def state_counts(code):
    """Sorted (state, count) pairs over rows with a state."""
    c = collections.Counter(int(v) for v in np.asarray(code, np.uint64) if v != NO_STATE)
    keys = np.array(sorted(c), np.uint64)
    return keys, np.array([c[int(k)] for k in keys], np.int64)
