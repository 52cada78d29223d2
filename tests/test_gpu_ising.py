"""GPU Boolean Ising (rac_ising) against the oracle, bit-exact: final
states, update counts and statuses, synchronous and asynchronous, both off
values, random and given update orders, one to four state words."""
import numpy as np
import pytest

from oracle import ising as oi
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


def _check(topo, n_traj, mode, low, max_steps, seed, sample, order=None, check_every=0, init=None,
           extra_ids=()):
    T = rp.Topology.from_inputs(topo)
    dev_init = None
    if init is not None:
        dev_init = torch.from_numpy(oi.pack(init).view(np.int64)).cuda()
    fin, steps, status = rp.ising(T, n_traj, rp.ISING_SYNC if mode == "sync" else rp.ISING_ASYNC, low,
                                  max_steps, seed, init=dev_init, order=order, check_every=check_every)
    torch.cuda.synchronize()
    got = oi.unpack(fin.cpu().numpy().view(np.uint64), topo.n_genes)
    st, sp = status.cpu().numpy(), steps.cpu().numpy()
    J = oi.coupling(topo.n_genes, topo.src, topo.dst, topo.sign)
    ids = np.arange(n_traj) if sample >= n_traj else np.sort(
        np.random.default_rng(seed).choice(n_traj, sample, replace=False))
    ids = np.unique(np.concatenate([ids, np.asarray(extra_ids, np.int64)]))
    for t in ids:
        s0 = init[t] if init is not None else oi.random_state(seed, int(t), topo.n_genes)
        f, k, ss, _ = oi.run(J, s0, mode, low, max_steps, seed, order, check_every, traj=int(t))
        assert np.array_equal(got[t], f) and sp[t] == k and st[t] == ss, (t, k, sp[t], ss, st[t])
    say(f"[gpu] ising {topo.name} {mode} low={low}: {np.mean(st == 0):.3f} fixed, "
        f"{len({tuple(r) for r in got[st == 0].tolist()})} distinct fixed states")
    return got, st


@pytest.mark.parametrize("low", [0, -1])
def test_toggle_switch_all_initial_states(low):
    init = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], bool)
    for mode in ("sync", "async"):
        _check(inputs.toggle_switch(), 4, mode, low, 50, 3, 4, init=init)


@pytest.mark.parametrize("mode", ["sync", "async"])
@pytest.mark.parametrize("low", [0, -1])
def test_dense_core_random_states(mode, low):
    _check(inputs.dense_core(1004), 20000, mode, low, 2000, 11, 150)


def test_async_given_order():
    topo = inputs.dense_core(1004)
    order = np.random.default_rng(2).permutation(topo.n_genes).astype(np.int32)
    _check(topo, 3000, "async", -1, 1000, 5, 100, order=order, check_every=7)


@pytest.mark.parametrize("n,e", [(100, 250), (150, 300), (250, 500)], ids=["W2", "W3", "W4"])
def test_wide_states(n, e):
    topo = inputs.erdos_renyi(n, e, 17)
    for mode in ("sync", "async"):
        _check(topo, 500, mode, -1, 3000, 21, 20)


def test_bad_orders_are_rejected():
    T = rp.Topology.from_inputs(inputs.toggle_switch())
    with pytest.raises(rp.RacError):
        rp.ising(T, 4, rp.ISING_ASYNC, order=[0, 2])
    with pytest.raises(rp.RacError):
        rp.ising(T, 4, rp.ISING_SYNC, low=1)


def test_sync_large_ragged_ensemble():
    # 600,001 random states: checked at wave and block boundaries and at the
    # last trajectory, besides a random sample.
    n = 600_001
    edges = [0, 1, 63, 64, 127, 128, 2047, 2048, 4095, n - 129, n - 65, n - 64, n - 2, n - 1]
    for low in (0, -1):
        _check(inputs.dense_core(1004), n, "sync", low, 300, 5, 40, extra_ids=edges)


def _wide_fan_in(n_genes, seed):
    # Random sparse edges plus genes regulated by 64, 40, 17, 9 and 5 others,
    # self-loops, and genes without regulators.
    rng = np.random.default_rng(seed)
    edges = {}
    for s_, d_ in zip(rng.integers(0, n_genes, 2 * n_genes), rng.integers(0, n_genes, 2 * n_genes)):
        edges[(int(s_), int(d_))] = 1 if rng.random() < 0.5 else -1
    for target, fan in ((0, min(64, n_genes)), (1, 40), (2, 17), (3, 9), (4, 5)):
        for s_ in rng.choice(n_genes, fan, replace=False):
            edges[(int(s_), target)] = 1 if rng.random() < 0.5 else -1
    for g in (5, 6, 7):
        edges[(g, g)] = 1 if g % 2 else -1
    for g in (n_genes - 1, n_genes - 2):  # no regulators
        edges = {k: v for k, v in edges.items() if k[1] != g}
    src = np.array([k[0] for k in edges], np.int32)
    dst = np.array([k[1] for k in edges], np.int32)
    sign = np.array(list(edges.values()), np.int8)
    return inputs.Topology(n_genes, src, dst, sign, f"fanin{n_genes}")


@pytest.mark.parametrize("n_genes", [64, 65])
def test_sync_wide_fan_in(n_genes):
    # Regulator counts up to 64 (the popcounts of a full state word), self-
    # loops, genes without regulators; 64 genes fill one state word, 65 need
    # two.  Given initial states, both off values.
    topo = _wide_fan_in(n_genes, 23)
    rng = np.random.default_rng(n_genes)
    init = rng.random((3000, n_genes)) < 0.5
    for low in (0, -1):
        _check(topo, 3000, "sync", low, 500, 9, 60, init=init, extra_ids=[0, 2999])


@pytest.mark.parametrize("low", [0, -1])
def test_sync_cycles_at_many_step_limits(low):
    # Periodic synchronous trajectories stop stepping once their cycle is
    # found and step only the remainder modulo the period: the final state,
    # count and status must equal the oracle's plain stepping for any limit,
    # including limits shorter than the detection and every residue.
    topo = inputs.dense_core(1004)
    for max_steps in (0, 1, 2, 3, 7, 64, 65, 127, 1000, 1001):
        _check(topo, 4000, "sync", low, max_steps, 31 + max_steps, 60)
    topo = inputs.erdos_renyi(40, 100, 23)
    for max_steps in (5, 333, 2048):
        _check(topo, 2000, "sync", low, max_steps, 41 + max_steps, 40)


def test_sync_evaluation_counter():
    # Toggle switch with off = -1: (0,0) and (1,1) alternate with period 2,
    # found after four updates (checkpoints after 1 and 2 updates); (0,1) and
    # (1,0) are fixed at once.  Performed gene evaluations: 4 x 2 + 1 x 2 +
    # 1 x 2 + 4 x 2 = 20, though the results stand for 50 updates of the
    # periodic pair.
    T = rp.Topology.from_inputs(inputs.toggle_switch())
    init = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], bool)
    dev_init = torch.from_numpy(oi.pack(init).view(np.int64)).cuda()
    ev = torch.zeros(1, dtype=torch.int64, device="cuda")
    fin, steps, status = rp.ising(T, 4, rp.ISING_SYNC, -1, 50, 0, init=dev_init, evals=ev)
    torch.cuda.synchronize()
    assert int(ev.item()) == 20
    got = oi.unpack(fin.cpu().numpy().view(np.uint64), 2)
    assert np.array_equal(got, init)  # even step count: back where they started
    assert steps.cpu().tolist() == [50, 0, 0, 50] and status.cpu().tolist() == [1, 0, 0, 1]


def test_async_test_interval_beyond_the_step_limit():
    # A fixed-point test interval far above max_steps: one test at the start,
    # then plain updates to the limit (the round loop ends with the updates
    # left, not after `check_every` empty passes).
    _check(inputs.dense_core(1004), 3000, "async", -1, 60, 13, 80, check_every=1_000_000)
    _check(inputs.dense_core(1004), 3000, "async", 0, 61, 14, 80, check_every=7)


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_lanes_that_take_several_trajectories(mode):
    # Past a grid's worth of lanes (synchronous: 256 blocks of 256 per CU,
    # 16.8 M on 256 CUs; asynchronous: 16 per CU, 1.05 M) a lane starts its
    # next trajectory when one ends.  Trajectories of the second pass, and
    # the first-pass ones of the same lanes, against the oracle.
    topo = inputs.dense_core(1004)
    lanes = (256 if mode == "sync" else 16) * 256 * 256
    n = lanes + 3000
    tail = np.arange(lanes, n, 97)
    extra = np.concatenate([tail, tail - lanes, [0, n - 1]])
    max_steps = 1000 if mode == "sync" else 3000
    _check(topo, n, mode, -1, max_steps, 17, 20, extra_ids=extra)
