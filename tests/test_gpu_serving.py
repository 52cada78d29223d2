"""GPU: device sampling, serving step batches and continuous batching.

A trajectory's result must not depend on how it was scheduled: alone or in
a mix, in one launch or parked and resumed across many step batches, it is
bit-identical to rac_steady_states with the same lane count.
"""
import sys

import numpy as np
import pytest

import oracle
from tests import parity
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp
from paper_2503_18356_amd.serve import GpuExecutor, Request, Scheduler, poisson_requests

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("topo,seed", [(inputs.toggle_switch(), 1), (inputs.dense_core(1004), 7),
                                       (inputs.erdos_renyi(100, 250, 3), 11)])
def test_device_sampler_is_bit_identical(topo, seed):
    T = rp.Topology.from_inputs(topo)
    for begin, P, n_ic in [(0, 1000, 7), (123456, 77, 3)]:
        h = rp.sample_params(T, seed, P, n_ic, set_begin=begin)
        d = rp.sample_params_device(T, seed, P, n_ic, set_begin=begin)
        torch.cuda.synchronize()
        for f in ("G", "k", "T", "lam", "n", "ic"):
            assert np.array_equal(getattr(h, f), getattr(d, f).cpu().numpy()), f


def test_device_sampler_custom_ranges():
    T = rp.Topology.from_inputs(inputs.erdos_renyi(8, 14, 2))
    r = rp.Ranges(g_min=1, g_max=10, k_min=0.01, k_max=1, n_min=2, n_max=4, lam_inh_min=0.1)
    h = rp.sample_params(T, 5, 300, 2, ranges=r)
    d = rp.sample_params_device(T, 5, 300, 2, ranges=r)
    torch.cuda.synchronize()
    for f in ("G", "k", "T", "lam", "n", "ic"):
        assert np.array_equal(getattr(h, f), getattr(d, f).cpu().numpy()), f


@pytest.mark.parametrize("method", [rp.SAMPLE_UNIFORM, rp.SAMPLE_SOBOL])
def test_device_sampler_continuous_hill(method):
    T = rp.Topology.from_inputs(inputs.dense_core(1004))
    r = rp.Ranges(method=method, n_continuous=1)
    h = rp.sample_params(T, 19, 2000, 3, ranges=r)
    d = rp.sample_params_device(T, 19, 2000, 3, ranges=r)
    torch.cuda.synchronize()
    for f in ("G", "k", "T", "lam", "nf", "ic"):
        assert np.array_equal(getattr(h, f), getattr(d, f).cpu().numpy()), f


@pytest.mark.parametrize("rule", [rp.PRIOR_MEDIAN, rp.HALF_FUNCTIONAL])
@pytest.mark.parametrize("method", [rp.SAMPLE_UNIFORM, rp.SAMPLE_SOBOL, rp.SAMPLE_LHS])
def test_device_sampler_all_generators(method, rule):
    T = rp.Topology.from_inputs(inputs.dense_core(1004))
    r = rp.Ranges(method=method, threshold_rule=rule, hf_samples=4096, lhs_total=5000)
    for begin, P, n_ic in [(0, 3000, 9), (4000, 1000, 2)]:
        h = rp.sample_params(T, 77, P, n_ic, set_begin=begin, ranges=r)
        d = rp.sample_params_device(T, 77, P, n_ic, set_begin=begin, ranges=r)
        torch.cuda.synchronize()
        for f in ("G", "k", "T", "lam", "n", "ic"):
            assert np.array_equal(getattr(h, f), getattr(d, f).cpu().numpy()), (f, method, rule)


def _direct(T, params, lanes):
    out = rp.steady_states(T, params, rp.Opts(precision=rp.FP32, lanes_per_traj=lanes))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("batch_steps,wide", [(7, False), (64, False), (100000, False), (7, True)])
def test_step_batches_equal_one_shot(batch_steps, wide):
    # wide: lambdas ten times beyond Table 1's on each side, all 16 edges in
    # one lane, so most lanes start their running product below 1 (the start
    # must survive suspension between step batches).
    if wide:
        T = rp.Topology.from_inputs(inputs.erdos_renyi(8, 16, 1010))
        lanes = 1
        params = rp.sample_params(T, 93, 300, 10, ranges=rp.Ranges(lam_act_max=1e3, lam_inh_min=1e-3)).to_device()
    else:
        T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
        lanes = T.auto_lanes()
        params = rp.sample_params(T, 2002, 300, 10).to_device()
    epl, gpl = T.shape(lanes)
    ref = _direct(T, params, lanes)
    srv = rp.StepServer(rp.Opts(precision=rp.FP32), lanes, epl, gpl, max_requests=16,
                        batch_steps=batch_steps)
    out = rp.alloc_result(3000, T.n_genes, rp.FP32)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    srv.submit(T, params, out, stream=stream)
    counts = np.zeros(1, np.int32)
    batches = 0
    while True:
        srv.step(stream=stream)
        batches += 1
        srv.done_counts(0, 1, counts, stream=stream)
        torch.cuda.synchronize()
        if counts[0] >= 3000:
            break
        assert batches < 100000
    say(f"batch_steps={batch_steps}: {batches} step batches")
    assert counts[0] == 3000
    assert torch.equal(out.x, ref.x)
    assert torch.equal(out.n_acc, ref.n_acc) and torch.equal(out.n_rej, ref.n_rej)
    assert torch.equal(out.status, ref.status) and torch.equal(out.t_final, ref.t_final)


def test_requests_joining_mid_flight_match_alone():
    # Several networks of one kernel class; later ones arrive while earlier
    # ones are parked mid-trajectory.
    topos = [inputs.erdos_renyi(10, 25, s) for s in (1002, 3, 4, 5)]
    Ts = [rp.Topology.from_inputs(t) for t in topos]
    lanes = 4
    shapes = {T.shape(lanes) for T in Ts}
    epl = max(s[0] for s in shapes)
    gpl = max(s[1] for s in shapes)
    Ts = [T for T in Ts if T.shape(lanes) == (epl, gpl)]
    assert len(Ts) >= 2
    srv = rp.StepServer(rp.Opts(precision=rp.FP32), lanes, epl, gpl, max_requests=16, batch_steps=32)
    stream = torch.cuda.Stream()
    jobs = []
    counts = np.zeros(len(Ts), np.int32)
    for i, T in enumerate(Ts):
        prm = rp.sample_params(T, 40 + i, 200 + 50 * i, 5).to_device()
        out = rp.alloc_result(prm.n_sets * 5, T.n_genes, rp.FP32)
        torch.cuda.synchronize()
        srv.submit(T, prm, out, stream=stream)
        jobs.append((T, prm, out))
        for _ in range(3):  # the next request arrives while this one runs
            srv.step(stream=stream)
    for _ in range(20000):
        srv.done_counts(0, len(jobs), counts, stream=stream)
        torch.cuda.synchronize()
        if all(counts[i] >= jobs[i][1].n_sets * 5 for i in range(len(jobs))):
            break
        srv.step(stream=stream)
    else:
        pytest.fail(f"requests did not finish: done {counts.tolist()}")
    for T, prm, out in jobs:
        if T.shape(lanes) == (epl, gpl):
            ref = _direct(T, prm, lanes)
            assert torch.equal(out.x, ref.x)
            assert torch.equal(out.n_acc, ref.n_acc)


def test_request_after_drained_queue_is_served():
    # The first request is fully claimed in its first batch, so the queue
    # head runs past the tail; a request appended afterwards must still run.
    T = rp.Topology.from_inputs(inputs.toggle_switch())
    lanes = T.auto_lanes()
    epl, gpl = T.shape(lanes)
    srv = rp.StepServer(rp.Opts(precision=rp.FP32), lanes, epl, gpl, max_requests=8, batch_steps=16)
    stream = torch.cuda.Stream()
    jobs = []
    counts = np.zeros(3, np.int32)
    for i, P in enumerate((30, 5, 64)):
        prm = rp.sample_params(T, 70 + i, P, 2).to_device()
        out = rp.alloc_result(P * 2, T.n_genes, rp.FP32)
        torch.cuda.synchronize()
        srv.submit(T, prm, out, stream=stream)
        jobs.append((prm, out))
        for _ in range(50):
            srv.step(stream=stream)
    for _ in range(5000):
        srv.done_counts(0, 3, counts, stream=stream)
        torch.cuda.synchronize()
        if all(counts[i] >= jobs[i][0].n_sets * 2 for i in range(3)):
            break
        srv.step(stream=stream)
    else:
        pytest.fail(f"requests did not finish: done {counts.tolist()}")
    for prm, out in jobs:
        ref = _direct(T, prm, lanes)
        assert torch.equal(out.x, ref.x) and torch.equal(out.n_acc, ref.n_acc)


def test_network_in_a_larger_shape_matches_its_own():
    # A server of a larger kernel shape pads the network's slots with factors
    # of exactly one: results are bit-identical to the network's own shape.
    T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    lanes = T.auto_lanes()
    epl, gpl = T.shape(lanes)
    big = (min(e for e in (4, 8, 12, 16, 24, 32) if e > epl), min(g for g in (1, 2, 3, 4, 6, 8) if g > gpl))
    assert rp.factor_form(rp.FP32, big[0]) == rp.factor_form(rp.FP32, epl)
    params = rp.sample_params(T, 91, 400, 3).to_device()
    ref = _direct(T, params, lanes)
    try:
        srv = rp.StepServer(rp.Opts(precision=rp.FP32), lanes, big[0], big[1], max_requests=4,
                            batch_steps=40)
    except rp.RacError:
        pytest.skip(f"no compiled serving shape {big}")
    say(f"own shape {(epl, gpl)}, server shape {big}, lanes {lanes}")
    out = rp.alloc_result(1200, T.n_genes, rp.FP32)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    srv.submit(T, params, out, stream=stream)
    counts = np.zeros(1, np.int32)
    for _ in range(5000):
        srv.step(stream=stream)
        srv.done_counts(0, 1, counts, stream=stream)
        torch.cuda.synchronize()
        if counts[0] >= 1200:
            break
    else:
        pytest.fail("request did not finish")
    assert torch.equal(out.x, ref.x)
    assert torch.equal(out.n_acc, ref.n_acc) and torch.equal(out.status, ref.status)


def _serve_all(srv, T, params, n):
    out = rp.alloc_result(n, T.n_genes, rp.FP32)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    srv.submit(T, params, out, stream=stream)
    counts = np.zeros(1, np.int32)
    for _ in range(5000):
        srv.step(stream=stream)
        srv.done_counts(0, 1, counts, stream=stream)
        torch.cuda.synchronize()
        if counts[0] >= n:
            return out
    pytest.fail("request did not finish")


def test_both_factor_forms_agree_with_the_oracle():
    # One network solved by kernels of both Hill-factor forms: its own shape
    # (1 + D / (1 + 2^z)) and a serving shape past the switch point (the
    # symmetric sqrt(lam) form).  Each meets the parity bar against the oracle.
    T = rp.Topology.from_inputs(inputs.erdos_renyi(10, 25, 1002))
    lanes = T.auto_lanes()
    epl, gpl = T.shape(lanes)
    wide = 24
    assert rp.factor_form(rp.FP32, epl) == 1 and rp.factor_form(rp.FP32, wide) == 0
    n_sets, n_ic, seed = 200, 5, 93
    params = rp.sample_params(T, seed, n_sets, n_ic).to_device()
    own = _direct(T, params, lanes)
    srv = rp.StepServer(rp.Opts(precision=rp.FP32), lanes, wide, gpl, max_requests=4, batch_steps=64)
    other = _serve_all(srv, T, params, n_sets * n_ic)
    say(f"own shape {(epl, gpl)} vs {(wide, gpl)} at {lanes} lanes")
    net = oracle.canonicalize(T.n_genes, *[np.asarray(v) for v in (T.src, T.dst, T.sign)])
    op = oracle.sample(net, seed, n_sets, n_ic)
    oo = oracle.Opts(ss_rtol=1e-5)
    ids = np.arange(0, n_sets * n_ic, 7)
    ref = oracle.steady_states(net, op, oo, traj_ids=ids, n_threads=8)
    for name, res in (("unit", own), ("symmetric", other)):
        rep = parity.compare_steady(net, op, oo, ids, res.x.cpu().numpy()[ids], ref.x, n_ic,
                                    res.status.cpu().numpy()[ids], ref.status)
        say(name, rep)
        assert rep.ok(), (name, str(rep))


def test_scheduler_on_gpu_poisson_stream():
    rng = np.random.default_rng(7)
    reqs = poisson_requests(rng, 40, rate=400.0, n_lo=2, n_hi=30, p_lo=50, p_hi=3000)
    ex = GpuExecutor(batch_steps=128)
    sched = Scheduler(ex, hbm_budget=8 << 30)
    done = sched.run(reqs, max_seconds=120)
    assert len(done) == 40
    st = sched.stats()
    say("serving:", st)
    # Each request equals its own one-shot solve at the same lane count.
    for req in done[:10]:
        T = req.handle["T"]
        lanes = req.handle["class"][0]
        prm = rp.sample_params(T, req.seed, req.n_sets, req.n_ic).to_device()
        ref = _direct(T, prm, lanes)
        assert torch.equal(req.result.x, ref.x), req.rid
    # ... and agrees with the oracle on a few trajectories.
    req = done[0]
    net = oracle.canonicalize(req.topo.n_genes, req.topo.src, req.topo.dst, req.topo.sign)
    op = oracle.sample(net, req.seed, req.n_sets, req.n_ic)
    ids = np.arange(min(20, req.n_traj))
    ref = oracle.steady_states(net, op, oracle.Opts(ss_rtol=1e-5), traj_ids=ids, n_threads=8)
    gk = (op.G / op.k).T.astype(np.float64)[ids // req.n_ic]
    err = np.abs(req.result.x.cpu().numpy()[ids] - ref.x) / gk
    assert np.sum(err.max(axis=1) > 1e-4) <= 1


def test_full_request_tables_open_new_generations():
    # Request tables of three entries: a stream of twelve requests of one
    # network class runs through several step servers; drained ones are
    # destroyed, and every result still equals its one-shot solve.
    rng = np.random.default_rng(11)
    topo = inputs.erdos_renyi(10, 25, 1002)
    reqs = [Request(i, topo, 900 + i, int(rng.integers(20, 200)), 5, arrival=0.002 * i) for i in range(12)]
    ex = GpuExecutor(batch_steps=32, max_requests=3)
    sched = Scheduler(ex, hbm_budget=1 << 30)
    peak = 0
    orig = ex.start

    def start(req):
        nonlocal peak
        orig(req)
        peak = max(peak, ex.generations())

    ex.start = start
    done = sched.run(reqs, max_seconds=120)
    assert len(done) == 12
    say("generations alive at most:", peak, "at the end:", ex.generations())
    assert peak >= 2                       # twelve requests cannot fit one table of three
    assert ex.generations() <= 2           # drained generations were destroyed
    for req in done:
        T = req.handle["T"]
        prm = rp.sample_params(T, req.seed, req.n_sets, req.n_ic).to_device()
        ref = _direct(T, prm, req.handle["class"][0])
        assert torch.equal(req.result.x, ref.x), req.rid


def test_interactive_server_futures():
    # The submit -> future front end: requests submitted from two threads
    # while earlier ones are on the GPU; each future's request equals its own
    # one-shot solve at the lane count its class used, bit for bit.
    import concurrent.futures as cf
    import time as _time
    from paper_2503_18356_amd import inputs as _inputs
    from paper_2503_18356_amd.serve import Server
    rng = np.random.default_rng(23)
    specs = [_inputs.serving_request(rng, 2, 30, 50, 2000, 1, 5) for _ in range(12)]
    say("[gpu] interactive server,", len(specs), "requests")
    with Server(hbm_budget=8 << 30, batch_steps=128) as srv:
        def feed(part):
            out = []
            for i, (topo, P, n_ic) in part:
                out.append(srv.submit(topo, 900 + i, P, n_ic))
                _time.sleep(0.003)
            return out
        items = list(enumerate(specs))
        with cf.ThreadPoolExecutor(2) as pool:
            parts = list(pool.map(feed, (items[0::2], items[1::2])))
        futs = [f for part in parts for f in part]
        done = [f.result(timeout=240) for f in futs]
    assert len({d.rid for d in done}) == len(specs)
    for req in done:
        T = req.handle["T"]
        prm = rp.sample_params(T, req.seed, req.n_sets, req.n_ic).to_device()
        ref = _direct(T, prm, req.handle["class"][0])
        assert torch.equal(req.result.x, ref.x), req.rid
        assert req.latency > 0
