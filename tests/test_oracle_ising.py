"""Pins of the Boolean Ising oracle (CPU): closed-form motifs, brute-force
fixed points of small networks, and the invariants of the update modes."""
import itertools

import numpy as np
import pytest

from oracle import ising
from paper_2503_18356_amd import inputs


def _ts():
    t = inputs.toggle_switch()   # A -| B, B -| A
    return t.n_genes, t.src, t.dst, t.sign


def test_toggle_switch_sync_closed_forms():
    N, s, d, g = _ts()
    J = ising.coupling(N, s, d, g)
    assert J.tolist() == [[0, -1], [-1, 0]]
    # 0/1 states: (1,0) and (0,1) are fixed; (1,1) switches both off and
    # (0,0) has no active input, so it stays.
    for init, want in [((1, 0), (1, 0)), ((0, 1), (0, 1)), ((1, 1), (0, 0)), ((0, 0), (0, 0))]:
        f, steps, st, _ = ising.run(J, np.array(init, bool), "sync", low=0)
        assert tuple(f.astype(int)) == want and st == ising.FIXED_POINT
    # +-1 states: (-1,-1) and (1,1) alternate (period 2) and never settle.
    f, steps, st, rec = ising.run(J, np.array([0, 0], bool), "sync", low=-1, max_steps=7, record=True)
    assert st == ising.MAX_STEPS and steps == 7
    assert [tuple(r.astype(int)) for r in rec[:4]] == [(0, 0), (1, 1), (0, 0), (1, 1)]


def test_activation_chain_copies_the_source():
    # A -> B -> C with A self-activating: every state ends at (a, a, a).
    src, dst, sign = [0, 0, 1], [0, 1, 2], [1, 1, 1]
    J = ising.coupling(3, src, dst, sign)
    for init in itertools.product([0, 1], repeat=3):
        f, _, st, _ = ising.run(J, np.array(init, bool), "sync", low=-1)
        assert st == ising.FIXED_POINT and f.tolist() == [bool(init[0])] * 3


def _brute_fixed_points(J, low):
    N = J.shape[0]
    fps = set()
    for bits in itertools.product([False, True], repeat=N):
        on = np.array(bits)
        s = np.where(on, 1, low)
        h = J @ s
        if np.all((h <= 0) | on) and np.all((h >= 0) | ~on):
            fps.add(bits)
    return fps


@pytest.mark.parametrize("low", [0, -1])
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_endpoints_are_brute_force_fixed_points(mode, low):
    t = inputs.erdos_renyi(8, 16, 3)
    J = ising.coupling(t.n_genes, t.src, t.dst, t.sign)
    fps = _brute_fixed_points(J, low)
    fin, steps, status = ising.simulate(t.n_genes, t.src, t.dst, t.sign, 60, mode, low, 200, seed=5)
    assert np.any(status == ising.FIXED_POINT)
    for f, st in zip(fin, status):
        if st == ising.FIXED_POINT:
            assert tuple(f.tolist()) in fps


def test_async_changes_one_gene_per_update_and_is_seeded():
    t = inputs.dense_core(1004)
    J = ising.coupling(t.n_genes, t.src, t.dst, t.sign)
    s0 = ising.random_state(3, 0, t.n_genes)
    f, steps, st, rec = ising.run(J, s0, "async", low=-1, max_steps=300, seed=3, record=True)
    diffs = [int(np.sum(a != b)) for a, b in zip(rec, rec[1:])]
    assert max(diffs) <= 1
    f2, steps2, _, _ = ising.run(J, s0, "async", low=-1, max_steps=300, seed=3)
    assert np.array_equal(f, f2) and steps == steps2
    f3, steps3, _, _ = ising.run(J, s0, "async", low=-1, max_steps=300, seed=4)
    assert steps3 != steps or not np.array_equal(f3, f)


def test_random_gene_is_uniform_and_state_draws_are_fair():
    N = 22
    picks = np.array([ising.random_gene(9, 0, u, N) for u in range(22000)])
    counts = np.bincount(picks, minlength=N)
    assert counts.min() > 800 and counts.max() < 1200
    on = np.array([ising.random_state(9, t, N) for t in range(500)])
    assert 0.45 < on.mean() < 0.55


def test_custom_order_and_pack_roundtrip():
    N, s, d, g = _ts()
    J = ising.coupling(N, s, d, g)
    f, steps, st, rec = ising.run(J, np.array([1, 1], bool), "async", low=0, order=[1, 0],
                                  check_every=1, record=True)
    # Gene B updates first (B off), then A stays on: fixed at (1, 0).
    assert st == ising.FIXED_POINT and f.tolist() == [True, False] and steps == 1
    on = np.random.default_rng(1).integers(0, 2, (5, 130)).astype(bool)
    assert np.array_equal(ising.unpack(ising.pack(on), 130), on)
