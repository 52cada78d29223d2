"""GPU post-processing against the oracle (bit-exact).

The device chain (rac_normalize, rac_level_thresholds, rac_discretize,
rac_multistability, rac_state_counts) and oracle/postproc.py take the same
inputs: states from the GPU integrator (or synthetic ones) and the same
parameters.  Normalised values are compared bit for bit (both sides round the
same two FP32 operations); bins, levels, codes, thresholds and counts are
integers and must be equal.  At full size (10^6 trajectories) the oracle
checks sampled rows and sets.
"""
import numpy as np
import pytest

from oracle import postproc as pp
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def _run_chain(T, dp, res, n_bins, n_levels, capacity=1 << 12):
    out = rp.analyse_steady_states(T, dp, res, n_bins, n_levels, capacity)
    torch.cuda.synchronize()
    return out


def _oracle_chain(hp, x, status, n_ic, n_bins, n_levels):
    y = pp.normalize(x, hp.G, hp.k, n_ic)
    hist = pp.histogram(y, n_bins, status)
    thr = pp.thresholds(hist, n_levels)
    lv = pp.levels(y, n_bins, thr, status)
    cd = pp.codes(lv, n_levels, status)
    n, st = pp.multistability(cd, hp.G.shape[1], n_ic)
    keys, counts = pp.state_counts(cd)
    return dict(y=y, hist=hist, thresholds=thr, levels=lv, codes=cd, n_states=n, states=st,
                keys=keys, counts=counts)


def _compare(g, o):
    assert np.array_equal(g["y"].cpu().numpy().view(np.uint32), o["y"].view(np.uint32))
    assert np.array_equal(g["hist"].cpu().numpy(), o["hist"])
    assert g["thresholds"].cpu().numpy().tolist() == o["thresholds"]
    assert np.array_equal(g["levels"].cpu().numpy(), o["levels"])
    assert np.array_equal(u64(g["codes"]), o["codes"])
    assert np.array_equal(g["n_states"].cpu().numpy(), o["n_states"])
    assert np.array_equal(u64(g["states"]), o["states"])
    nu = int(g["n_unique"].item())
    assert nu == len(o["keys"])
    assert np.array_equal(u64(g["keys"])[:nu], o["keys"])
    assert np.array_equal(g["counts"].cpu().numpy()[:nu], o["counts"])
    assert np.all(u64(g["keys"])[nu:] == pp.NO_STATE)


@pytest.mark.parametrize("topo,levels,bins", [(inputs.toggle_switch(), 2, 64),
                                              (inputs.toggle_switch_self_activation(), 3, 32),
                                              (inputs.dense_core(1004), 2, 128)],
                         ids=["TS", "TSSA", "core22"])
def test_chain_on_integrated_states(topo, levels, bins):
    T = rp.Topology.from_inputs(topo)
    P, n_ic = (1000, 10) if topo.n_genes <= 2 else (200, 8)
    hp = rp.sample_params(T, 2001, P, n_ic)
    dp = hp.to_device()
    res = rp.steady_states(T, dp, rp.Opts(precision=rp.FP32))
    torch.cuda.synchronize()
    say(f"[gpu] postproc {topo.name} P={P} n_ic={n_ic} L={levels} B={bins}")
    g = _run_chain(T, dp, res, bins, levels)
    o = _oracle_chain(hp, res.x.cpu().numpy(), res.status.cpu().numpy(), n_ic, bins, levels)
    _compare(g, o)
    say("    thresholds", o["thresholds"], "states", len(o["keys"]),
        "multistability histogram", np.bincount(o["n_states"]).tolist())


@pytest.mark.parametrize("n_ic", [1, 3, 64, 128, 129, 1000, 4096])
def test_chain_on_synthetic_states(n_ic):
    # Random levels with excluded rows, four levels, ragged set sizes.
    rng = np.random.default_rng(n_ic)
    topo = inputs.erdos_renyi(5, 8, 7)
    T = rp.Topology.from_inputs(topo)
    P = max(2, 4000 // n_ic)
    hp = rp.sample_params(T, 9, P, n_ic)
    dp = hp.to_device()
    rows = P * n_ic
    p = np.arange(rows) // n_ic
    gk = (hp.G / hp.k).T[p]
    modes = rng.choice([0.03, 0.35, 0.7, 0.97], size=(rows, 5))
    x = (np.clip(modes + rng.normal(0, 0.02, (rows, 5)), 0, 1.05) * gk).astype(np.float32)
    status = rng.choice([0, 0, 0, 0, 1, 2], size=rows).astype(np.int8)
    res = rp.Result(torch.from_numpy(x).cuda(), torch.zeros(rows, dtype=torch.float64).cuda(),
                    torch.from_numpy(status).cuda(), torch.zeros(rows, dtype=torch.int32).cuda(),
                    torch.zeros(rows, dtype=torch.int32).cuda())
    g = _run_chain(T, dp, res, 32, 4, capacity=1 << 11)
    _compare(g, _oracle_chain(hp, x, status, n_ic, 32, 4))


def test_time_series_normalisation():
    T = rp.Topology.from_inputs(inputs.toggle_switch())
    hp = rp.sample_params(T, 4, 50, 3)
    dp = hp.to_device()
    tk = np.linspace(0, 20, 11)
    res = rp.integrate(T, dp, tk, rp.Opts(precision=rp.FP32))
    y = rp.normalize(T, dp, res.x, n_t=11)
    torch.cuda.synchronize()
    want = pp.normalize(res.x.cpu().numpy().reshape(-1, 2), hp.G, hp.k, 3, n_t=11)
    assert np.array_equal(y.cpu().numpy().reshape(-1, 2).view(np.uint32), want.view(np.uint32))


def test_empty_and_overflow():
    T = rp.Topology.from_inputs(inputs.toggle_switch())
    y = torch.zeros((0, 2), dtype=torch.float32, device="cuda")
    hist, thr = rp.level_thresholds(y, 2, None, 16, 2)
    torch.cuda.synchronize()
    assert hist.sum().item() == 0 and thr.cpu().tolist() == [1]   # first tuple on ties
    codes = torch.tensor([0, 1, 2, 2, -1], dtype=torch.int64, device="cuda")
    keys, counts, nu = rp.state_counts(codes, capacity=2)
    torch.cuda.synchronize()
    assert nu.item() == -1                                         # 3 states, 2 slots
    keys, counts, nu = rp.state_counts(codes, capacity=4)
    torch.cuda.synchronize()
    assert nu.item() == 3 and u64(keys)[:3].tolist() == [0, 1, 2]
    assert counts.cpu().tolist()[:3] == [1, 1, 2]


def test_full_size_er10_sampled():
    # 10^6 steady states of the 10-gene network; the oracle checks samples.
    T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    P, n_ic = 10000, 100
    hp = rp.sample_params(T, 2002, P, n_ic)
    dp = hp.to_device()
    res = rp.steady_states(T, dp, rp.Opts(precision=rp.FP32))
    g = _run_chain(T, dp, res, 64, 2, capacity=1 << 16)
    x = res.x.cpu().numpy()
    st = res.status.cpu().numpy()
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(P * n_ic, 20000, replace=False))
    yo = pp.normalize(x, hp.G, hp.k, n_ic)
    assert np.array_equal(g["y"].cpu().numpy()[rows].view(np.uint32), yo[rows].view(np.uint32))
    hist = g["hist"].cpu().numpy()
    assert np.array_equal(hist, pp.histogram(yo, 64, st))
    thr = pp.thresholds(hist, 2)
    assert g["thresholds"].cpu().numpy().tolist() == thr
    lv = pp.levels(yo[rows], 64, thr, st[rows])
    assert np.array_equal(g["levels"].cpu().numpy()[rows], lv)
    assert np.array_equal(u64(g["codes"])[rows], pp.codes(lv, 2, st[rows]))
    sets = rng.choice(P, 300, replace=False)
    cd = u64(g["codes"]).reshape(P, n_ic)
    n, s = pp.multistability(cd[sets].ravel(), len(sets), n_ic)
    assert np.array_equal(g["n_states"].cpu().numpy()[sets], n)
    assert np.array_equal(u64(g["states"])[sets], s)
    nu = int(g["n_unique"].item())
    keys, counts = pp.state_counts(u64(g["codes"]))
    assert nu == len(keys) and np.array_equal(g["counts"].cpu().numpy()[:nu], counts)
    say(f"    ER10 1e6: thresholds {thr}, {nu} states, multistability "
        f"{np.bincount(g['n_states'].cpu().numpy()).tolist()[:6]}")
