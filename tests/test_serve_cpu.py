"""Serving scheduler on the CPU: admission by footprint, first-come order,
continuous batching and latency accounting, driven by a stand-in executor
that solves tiny networks with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd.serve import Request, Scheduler, footprint_bytes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class OracleExecutor:
    """Finishes each request after a number of step batches proportional to
    its size; its results come from the oracle."""

    def __init__(self, sched_ref, clock, batch_cost=1000):
        self.sched = sched_ref
        self.clock = clock
        self.batch_cost = batch_cost
        self.inflight = {}
        self.max_used = 0
        self.concurrent = []

    def start(self, req):
        net = oracle.canonicalize(req.topo.n_genes, req.topo.src, req.topo.dst, req.topo.sign)
        prm = oracle.sample(net, req.seed, req.n_sets, req.n_ic)
        req.result = oracle.steady_states(net, prm, oracle.Opts(ss_rtol=1e-5), n_threads=2)
        self.inflight[req.rid] = [req, req.n_traj]

    def step(self):
        self.clock.t += 0.001
        self.max_used = max(self.max_used, self.sched[0].used)
        self.concurrent.append(len(self.inflight))
        share = self.batch_cost / max(1, len(self.inflight))
        for v in self.inflight.values():
            v[1] -= share

    def finished(self):
        out = [rid for rid, v in self.inflight.items() if v[1] <= 0]
        for rid in out:
            del self.inflight[rid]
        return out

    def release(self, req):
        pass


def _reqs(n, rate, seed=0, p_hi=400):
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        topo, P, n_ic = inputs.serving_request(rng, 2, 6, 5, p_hi, 1, 4)
        out.append(Request(i, topo, 100 + i, P, n_ic, arrival=t))
    return out


def _run(reqs, budget, clock=None):
    clock = clock or FakeClock()
    holder = [None]
    ex = OracleExecutor(holder, clock)
    s = Scheduler(ex, budget, clock=clock)
    holder[0] = s
    # Drive the loop on the fake clock: advance to the next arrival when idle.
    pending = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    while i < len(pending) or not s.idle():
        while i < len(pending) and pending[i].arrival <= clock.t:
            s.arrive(pending[i])
            i += 1
        s.admit()
        if s.running:
            s.step()
        elif i < len(pending):
            clock.t = pending[i].arrival
    return s, ex


def test_all_requests_complete_with_oracle_results():
    reqs = _reqs(30, rate=200)
    s, ex = _run(reqs, budget=10**9)
    assert len(s.done) == 30 and not s.rejected
    for r in s.done:
        assert r.finished >= r.admitted >= r.arrival
        assert np.all(np.isin(r.result.status, (oracle.CONVERGED, oracle.T_END)))
        assert r.result.x.shape == (r.n_traj, r.topo.n_genes)
    st = s.stats()
    assert st["requests"] == 30 and st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_never_exceeds_budget_and_is_fifo():
    reqs = _reqs(40, rate=5000)
    sizes = [footprint_bytes(r.topo.n_genes, r.topo.n_edges, r.n_sets, r.n_ic) for r in reqs]
    budget = int(np.percentile(sizes, 90) * 2)
    s, ex = _run(reqs, budget=budget)
    assert ex.max_used <= budget
    # First come, first admitted: a later request is never admitted earlier.
    by_rid = sorted(s.done, key=lambda r: r.rid)
    adm = [r.admitted for r in by_rid]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_requests_overlap_while_others_run():
    # Continuous batching: later arrivals join while earlier ones are in flight.
    reqs = _reqs(20, rate=3000)
    s, ex = _run(reqs, budget=10**9)
    assert max(ex.concurrent) >= 3


def test_oversized_request_is_rejected_not_blocking():
    reqs = _reqs(6, rate=1000)
    big = reqs[2]
    budget = footprint_bytes(big.topo.n_genes, big.topo.n_edges, big.n_sets, big.n_ic) - 1
    others = [r for r in reqs if r is not big]
    budget = max(budget, max(footprint_bytes(r.topo.n_genes, r.topo.n_edges, r.n_sets, r.n_ic)
                             for r in others))
    big.n_sets *= 1000  # certainly beyond the budget now
    s, ex = _run(reqs, budget=budget)
    assert [r.rid for r in s.rejected] == [big.rid]
    assert len(s.done) == len(reqs) - 1


def test_footprint_formula():
    # parameters + ICs + states + 17 bytes of info per trajectory
    assert footprint_bytes(2, 2, 10, 3) == 10 * (16 + 16 + 2) + 3 * 8 + 30 * (8 + 17)


def test_server_futures_from_several_threads():
    # The interactive front end: requests submitted from four threads while
    # others run; every future resolves to its finished request with the
    # stand-in executor's (oracle) result, and a request that can never fit
    # the budget fails with MemoryError.
    import concurrent.futures as cf
    from paper_2503_18356_amd.serve import Server
    reqs = _reqs(16, 200.0, seed=4)
    clock = FakeClock()
    holder = [None]
    ex = OracleExecutor(holder, clock, batch_cost=400)
    budget = 3 * max(footprint_bytes(r.topo.n_genes, r.topo.n_edges, r.n_sets, r.n_ic) for r in reqs)
    with Server(hbm_budget=budget, executor=ex, clock=clock) as srv:
        holder[0] = srv.sched
        with cf.ThreadPoolExecutor(4) as pool:
            futs = list(pool.map(lambda r: srv.submit(r.topo, r.seed, r.n_sets, r.n_ic), reqs))
        too_big = srv.submit(reqs[0].topo, 1, 10**9, 10)
        done = [f.result(timeout=120) for f in futs]
        with pytest.raises(MemoryError):
            too_big.result(timeout=120)
    assert sorted(d.rid for d in done) == sorted(set(d.rid for d in done))
    for r, d in zip(reqs, done):
        assert (d.topo, d.seed, d.n_sets, d.n_ic) == (r.topo, r.seed, r.n_sets, r.n_ic)
        assert d.finished >= d.admitted >= d.arrival >= 0
        net = oracle.canonicalize(r.topo.n_genes, r.topo.src, r.topo.dst, r.topo.sign)
        ref = oracle.steady_states(net, oracle.sample(net, r.seed, r.n_sets, r.n_ic), oracle.Opts(ss_rtol=1e-5),
                                   n_threads=2)
        assert np.array_equal(d.result.x, ref.x)
    assert ex.max_used <= budget and max(ex.concurrent) >= 2
    with pytest.raises(RuntimeError):
        srv.submit(reqs[0].topo, 1, 10, 1)
