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


def _check(topo, n_traj, mode, low, max_steps, seed, sample, order=None, check_every=0, init=None):
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
