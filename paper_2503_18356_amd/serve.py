"""Continuous-batching serving loop for RACIPE simulation requests.

A request is (network, seed, parameter sets P, initial conditions n_ic): the
steady states of all P * n_ic trajectories (GRiNS Sec. 2.1.3).  Requests
arrive over time; the scheduler admits them while their device footprint fits
the HBM budget, samples their parameters on the GPU, and hands them to a
per-kernel-class step server (rac_server_*): every step batch advances all
in-flight trajectories of every admitted request of that class, so requests
that arrive while others run share the same launches.  Finished requests
release their memory, which admits waiting ones.  Latency is measured from
arrival to the host seeing the request's last trajectory finish.

The scheduler talks to an executor (``GpuExecutor`` here); tests drive it
with a CPU stand-in to check admission, ordering and accounting.
``Server`` is the interactive form: ``submit()`` from any thread returns a
future while a background thread runs the scheduler loop.
"""
from __future__ import annotations

import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    topo: object          # inputs.Topology
    seed: int
    n_sets: int
    n_ic: int
    arrival: float = 0.0  # seconds (scheduler clock)
    admitted: float = -1.0
    finished: float = -1.0
    nbytes: int = 0
    result: object = None
    handle: object = None  # executor-private

    @property
    def n_traj(self) -> int:
        return self.n_sets * self.n_ic

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Interactive front end of the serving loop: ``submit()`` may be called
    from any thread, also while other requests are on the GPU, and returns a
    ``concurrent.futures.Future`` that resolves to the finished ``Request``
    (``.result`` holds its steady states and per-trajectory info on the
    device, ``.latency`` its arrival-to-finish time).  A background thread
    admits requests by HBM footprint and runs the continuous-batching steps;
    a request that can never fit the budget fails its future with
    ``MemoryError``.  ``close()`` lets the requests in flight finish and
    stops the thread."""

    def __init__(self, hbm_budget: int = 64 << 30, opts=None, batch_steps: int = 512, executor=None,
                 clock=time.perf_counter):
        self.ex = executor if executor is not None else GpuExecutor(opts=opts, batch_steps=batch_steps)
        self.sched = Scheduler(self.ex, hbm_budget, clock=clock)
        self._cv = threading.Condition()
        self._new: collections.deque[Request] = collections.deque()
        self._futures: dict[int, concurrent.futures.Future] = {}
        self._next = 0
        self._closed = False
        self._n_done = self._n_rejected = 0
        self._thread = threading.Thread(target=self._loop, name="racipe-server", daemon=True)
        self._thread.start()

    def submit(self, topo, seed: int, n_sets: int, n_ic: int) -> concurrent.futures.Future:
        fut: concurrent.futures.Future = concurrent.futures.Future()
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed")
            req = Request(self._next, topo, seed, n_sets, n_ic)
            self._next += 1
            self._futures[req.rid] = fut
            self._new.append(req)
            self._cv.notify()
        return fut

    def _settle(self):
        done, rej = self.sched.done, self.sched.rejected
        for req in done[self._n_done:]:
            self._futures.pop(req.rid).set_result(req)
        for req in rej[self._n_rejected:]:
            self._futures.pop(req.rid).set_exception(
                MemoryError(f"request {req.rid} needs {req.nbytes} bytes, over the HBM budget"))
        self._n_done, self._n_rejected = len(done), len(rej)

    def _loop(self):
        try:
            while True:
                with self._cv:
                    while not self._new and self.sched.idle() and not self._closed:
                        self._cv.wait()
                    if self._closed and not self._new and self.sched.idle():
                        return
                    new = list(self._new)
                    self._new.clear()
                for req in new:
                    self.sched.arrive(req)
                self.sched.admit()
                if self.sched.running:
                    self.sched.step()
                self._settle()
        except BaseException as e:  # fail every outstanding future, then stop
            with self._cv:
                self._closed = True
                for fut in self._futures.values():
                    if not fut.done():
                        fut.set_exception(e)
                self._futures.clear()

    def close(self, timeout: float | None = None):
        with self._cv:
            self._closed = True
            self._cv.notify()
        self._thread.join(timeout)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def footprint_bytes(n_genes: int, n_edges: int, n_sets: int, n_ic: int, x_bytes: int = 4) -> int:
    """Device bytes a request holds while admitted: parameters, initial
    conditions, steady states and per-trajectory info."""
    params = n_sets * (2 * n_genes * 4 + 2 * n_edges * 4 + n_edges)
    ics = n_ic * n_genes * 4
    outs = n_sets * n_ic * (n_genes * x_bytes + 8 + 1 + 4 + 4)
    return int(params + ics + outs)


class Scheduler:
    """Admission by HBM footprint, continuous batching, latency accounting."""

    def __init__(self, executor, hbm_budget: int, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.used = 0
        self.clock = clock
        self.waiting: collections.deque[Request] = collections.deque()
        self.running: dict[int, Request] = {}
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.t0 = clock()

    def now(self) -> float:
        return self.clock() - self.t0

    def arrive(self, req: Request):
        req.arrival = self.now() if req.arrival <= 0 else req.arrival
        req.nbytes = footprint_bytes(req.topo.n_genes, req.topo.n_edges, req.n_sets, req.n_ic)
        if req.nbytes > self.budget:
            self.rejected.append(req)  # can never fit
            return
        self.waiting.append(req)

    def admit(self):
        # First come, first served: a large request at the head waits for
        # memory rather than being overtaken indefinitely.
        while self.waiting and self.used + self.waiting[0].nbytes <= self.budget:
            req = self.waiting.popleft()
            self.used += req.nbytes
            req.admitted = self.now()
            self.ex.start(req)
            self.running[req.rid] = req

    def step(self):
        if self.running:
            self.ex.step()
            for rid in self.ex.finished():
                req = self.running.pop(rid)
                req.finished = self.now()
                self.ex.release(req)
                self.used -= req.nbytes
                self.done.append(req)

    def idle(self) -> bool:
        return not self.waiting and not self.running

    def run(self, arrivals: list[Request], until_idle: bool = True, max_seconds: float = 600.0,
            progress=None, progress_every: float = 10.0):
        """Feed requests at their arrival times (seconds from now) and serve.
        ``progress(msg)`` is called every ``progress_every`` seconds."""
        pending = sorted(arrivals, key=lambda r: r.arrival)
        i = 0
        self.t0 = self.clock()
        next_report = progress_every
        while True:
            now = self.now()
            if progress is not None and now >= next_report:
                next_report = now + progress_every
                progress(f"serve t={now:.1f}s arrived={i}/{len(pending)} waiting={len(self.waiting)} "
                         f"running={len(self.running)} done={len(self.done)}")
            while i < len(pending) and pending[i].arrival <= now:
                self.arrive(pending[i])
                i += 1
            self.admit()
            if self.running:
                self.step()
            elif i < len(pending):
                time.sleep(min(0.001, max(0.0, pending[i].arrival - self.now())))
            if i >= len(pending) and self.idle():
                break
            if self.now() > max_seconds:
                raise TimeoutError("serving did not drain in time")
        return self.done

    def stats(self, skip: int = 0) -> dict:
        reqs = sorted(self.done, key=lambda r: r.rid)[skip:]
        if not reqs:
            return {}
        lat = np.array([r.latency for r in reqs])
        t_first = min(r.arrival for r in reqs)
        t_last = max(r.finished for r in reqs)
        solves = sum(r.n_traj for r in reqs)
        return {"requests": len(reqs), "solves": int(solves),
                "solves_per_s": solves / max(t_last - t_first, 1e-9),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "rejected": len(self.rejected)}


class GpuExecutor:
    """Runs admitted requests on the GPU through rac_server step batches, one
    server per kernel class (lanes per trajectory, slot shape).

    A network joins an existing class (any lane count it fits, with a shape
    at least its own at that lane count) when the class costs at most
    ``merge_slack`` times the per-trajectory work of the network's own choice
    (padding slots compute factors of exactly one), so a mix of networks runs
    in few classes.  Classes share a small pool of
    streams.  The loop is pipelined: each iteration enqueues one batch per
    active class and a copy of every class's finished counts into pinned
    memory, then reads the counts the previous iteration copied (waiting on
    its event), so the GPU already holds the next batch while the host
    admits and retires requests.  A request is seen finished one batch after
    its last trajectory ends.

    A step server's request table has ``max_requests`` entries and is never
    reused, so a class whose newest server is full opens another one (a
    generation); an older generation is destroyed once all its requests are
    seen finished and the copies and batches enqueued before that have
    completed.  A class under continuous load therefore runs indefinitely
    with at most a few generations alive."""

    def __init__(self, opts=None, batch_steps: int = 512, max_requests: int = 65536,
                 device="cuda", keep_results: bool = True, merge_slack: float = 2.0,
                 n_streams: int = 4):
        import torch
        from . import racipe as rp
        self.rp = rp
        self.torch = torch
        self.opts = opts or rp.Opts(precision=rp.FP32)
        self.batch_steps = batch_steps
        self.max_requests = max_requests
        self.device = device
        self.keep_results = keep_results
        self.keep_rids: set[int] = set()  # results kept even without keep_results
        self.merge_slack = merge_slack
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, n_streams))]
        self.classes: dict[tuple, dict] = {}
        self.pending = None  # (events, [(generation, lo, hi, buffer)]) of the last poll
        self.polls = 0
        self.retired: list[tuple[int, dict]] = []  # (poll number, drained generation)

    @staticmethod
    def slot_cost(lanes: int, epl: int, gpl: int) -> float:
        # Per-trajectory issue cost model of a kernel class: lanes per
        # trajectory times the per-lane work of its edge and gene slots.
        return lanes * (14.0 * epl + 25.0 * gpl + 40.0)

    def _class(self, T):
        fp32 = self.rp.FP32
        lanes = T.auto_lanes(fp32)
        epl, gpl = T.shape(lanes, fp32)
        own = self.slot_cost(lanes, epl, gpl)
        best = None
        for key in self.classes:
            kl, ke, kg = key
            if not T.lanes_supported(kl, fp32):
                continue
            ne, ng = T.shape(kl, fp32)
            # Only classes whose kernels use the same Hill-factor form as the
            # network's own shape, so that a merged request gives the same
            # bits as a direct solve at that lane count.
            same_form = self.rp.factor_form(fp32, ke) == self.rp.factor_form(fp32, ne)
            if ke >= ne and kg >= ng and same_form:
                c = self.slot_cost(kl, ke, kg)
                if c <= self.merge_slack * own and (best is None or c < best[0]):
                    best = (c, key)
        if best is not None:
            return best[1], self.classes[best[1]]
        key = (lanes, epl, gpl)
        self.classes[key] = {"stream": self.streams[len(self.classes) % len(self.streams)],
                             "generations": []}
        return key, self.classes[key]

    def _generation(self, key, cl) -> dict:
        """The class's newest step server with a free request-table entry."""
        gens = cl["generations"]
        if gens and gens[-1]["server"].n_requests < self.max_requests:
            return gens[-1]
        lanes, epl, gpl = key
        srv = self.rp.StepServer(self.opts, lanes, epl, gpl, self.max_requests, self.batch_steps)
        bufs = [self.torch.zeros(self.max_requests, dtype=self.torch.int32, pin_memory=True)
                for _ in range(2)]
        gen = {"server": srv, "stream": cl["stream"], "active": {}, "bufs": bufs,
               "counts": [b.numpy() for b in bufs]}
        gens.append(gen)
        return gen

    def start(self, req: Request):
        rp = self.rp
        T = rp.Topology.from_inputs(req.topo)
        key, cl = self._class(T)
        gen = self._generation(key, cl)
        stream = cl["stream"]
        with self.torch.cuda.stream(stream):
            params = rp.alloc_params(T, req.n_sets, req.n_ic, device=self.device)
            rp.sample_params_device(T, req.seed, req.n_sets, req.n_ic, out=params, stream=stream)
            res = rp.alloc_result(req.n_traj, T.n_genes, rp.FP32, device=self.device)
        srv_rid = gen["server"].submit(T, params, res, stream=stream)
        req.handle = {"class": key, "srv_rid": srv_rid, "T": T, "params": params}
        req.result = res
        gen["active"][srv_rid] = req

    def generations(self) -> int:
        """Step servers currently alive over all classes."""
        return sum(len(cl["generations"]) for cl in self.classes.values())

    def step(self):
        for cl in self.classes.values():
            for gen in cl["generations"]:
                if gen["active"]:
                    gen["server"].step(stream=gen["stream"])

    def finished(self) -> list[int]:
        torch = self.torch
        # Enqueue this iteration's counts copies (after the batches just
        # launched) and record one event behind them on every stream used.
        which = self.polls % 2
        poll = self.polls
        self.polls += 1
        polled = []
        for cl in self.classes.values():
            for gen in cl["generations"]:
                act = gen["active"]
                if act:
                    lo, hi = min(act), max(act) + 1
                    gen["server"].done_counts(lo, hi - lo, gen["counts"][which], stream=gen["stream"])
                    polled.append((gen, lo, hi, which))
        events = []
        for st in {id(gen["stream"]): gen["stream"] for gen, *_ in polled}.values():
            ev = torch.cuda.Event()
            ev.record(st)
            events.append(ev)
        prev, self.pending = self.pending, (events, polled)
        if prev is None:
            return []
        # Read what the previous iteration copied.
        for ev in prev[0]:
            ev.synchronize()
        # Generations drained before the previous poll: everything enqueued
        # on them (their last batch and counts copy) preceded its events.
        while self.retired and self.retired[0][0] < poll:
            self.retired.pop(0)
        out = []
        for gen, lo, hi, w in prev[1]:
            act = gen["active"]
            cnt = gen["counts"][w]
            for srv_rid in range(lo, hi):
                req = act.get(srv_rid)
                if req is not None and cnt[srv_rid - lo] >= req.n_traj:
                    out.append(req.rid)
                    del act[srv_rid]
        # A full generation with nothing left in flight leaves its class; it
        # is destroyed after the events of this poll have completed.
        for cl in self.classes.values():
            gens = cl["generations"]
            keep = [g for g in gens[:-1] if g["active"]] + gens[-1:]
            for g in gens[:-1]:
                if not g["active"]:
                    self.retired.append((poll, g))
            cl["generations"] = keep
        return out

    def release(self, req: Request):
        # Parameters go; the result tensors stay with the request unless the
        # caller only wants throughput and latency.
        req.handle["params"] = None
        if not self.keep_results and req.rid not in self.keep_rids:
            req.result = None


def poisson_requests(rng, n: int, rate: float, n_lo=2, n_hi=100, p_lo=100, p_hi=100000,
                     ic_lo=1, ic_hi=10, seed0: int = 5000) -> list[Request]:
    """Poisson arrivals of random networks with log-uniform sizes."""
    from . import inputs
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        topo, P, n_ic = inputs.serving_request(rng, n_lo, n_hi, p_lo, p_hi, ic_lo, ic_hi)
        out.append(Request(i, topo, seed0 + i, P, n_ic, arrival=t))
    return out
