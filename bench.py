"""RACIPE ensemble benchmark on one MI355X.

Default workload (one "step"): steady states of every trajectory of an uneven
batch of 64 seeded random signed networks (N ~ U{5..50} genes, E = 2.5N edges,
half inhibitory, Erdos-Renyi without isolated genes), each with a
log-uniform 2,000-50,000 parameter sets x 10 initial conditions (about 10^7
trajectories in all), Table 1 parameter ranges (GRiNS Sec. 2.1.2), DP5(4)
with rtol 1e-6, atol 1e-9, t_end 200, steady when |dx_i/dt| <= 1e-6 +
1e-5 k_i |x_i|.  Parameters and initial conditions are resident in HBM before
timing starts.  The chosen form is FP32 state with FP64 time / error norm /
steady test in persistent work-queue launches, with the library's lane
model and the autotuner's choices switched in class by class where whole
untimed batch calls get faster; the plain form is FP64, one launch per
network.

The JSON line reports solves/s of the chosen form, the plain form, the
credited FP32 FLOP/s of the batch call against the MI355X vector peak, the
CPU oracle timed on a bounded sample on this host, parity against the oracle
on 1 % of every network, and, under "extras", the other configurations: the
10-gene network (10^6 trajectories), the 22-gene series (10^6 trajectories x
101 outputs), the toggle switch and the Poisson serving stream (2,000
requests after 200 warm-up at 200 req/s, p50/p99 latency).

Single workloads (--workload): er10, ts, uneven64 (without extras: --no-extras),
core22ts, serve, ising.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RACIPE ODE solves/s to steady state, batched FP32 vs plain FP64; p50/p99 latency"
PEAK_FP32 = 157.3e12   # MI355X FP32 vector (published; needs packed FP32)
# FP32 FMA issue without packed instructions, which these kernels are built
# without: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
PEAK_FP32_UNPACKED = 78.6e12
PEAK_FP64 = 78.6e12     # MI355X FP64 vector (published)
PEAK_HBM = 8.0e12


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("dp5_kernel.h", "kernel_common.h"):
        with open(os.path.join(ROOT, "paper_2503_18356_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    import glob
    import re
    want = kernel_source_hash()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        txt = open(f).read()
        m = re.search(r"`traffic_bytes_per_launch: (\d+)` `kernel_source_hash: ([0-9a-f]+)` "
                      r"`workload: ([\w.]+)`", txt)
        if m and m.group(2) == want and m.group(3) == workload:
            return float(m.group(1))
    return None


def profile_counter(workload: str, counter: str):
    """The chosen-form (first) value of a counter in the committed rocprofv3
    summary of a workload, or None when the kernel sources changed since the
    counters were taken."""
    import glob
    import re
    want = kernel_source_hash()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        txt = open(f).read()
        m = re.search(r"`kernel_source_hash: ([0-9a-f]+)` `workload: ([\w.]+)`", txt)
        if m and m.group(1) == want and m.group(2) == workload:
            v = re.search(r"\| " + re.escape(counter) + r" \| ([0-9.eE+-]+) \|", txt)
            return float(v.group(1)) if v else None
    return None


_CEILINGS = {}


def ceilings(rp, args):
    """VALU ceilings measured once per run on this device (None with --no-ceilings)."""
    if args.no_ceilings:
        return None
    if "c" not in _CEILINGS:
        _CEILINGS["c"] = rp.valu_ceilings()
    return _CEILINGS["c"]


def transcendental_rate(rp, args, workload: str, kernel_ms: float):
    """Transcendental throughput of the FP32 kernels: the transcendental
    instructions of the committed counter run (SQ_INSTS_VALU_TRANS_F32, per
    launch or batch call) x 64 lanes over this run's kernel time, against the
    sustained v_exp_f32 rate measured on this device (v_exp, v_log and v_rcp
    issue alike)."""
    n = profile_counter(workload, "SQ_INSTS_VALU_TRANS_F32")
    c = ceilings(rp, args)
    if n is None or c is None:
        return None
    ach = n * 64 / (kernel_ms * 1e-3)
    return {"achieved_tops": ach / 1e12, "ceiling_tops": c["v_exp_f32"] / 1e12, "frac": ach / c["v_exp_f32"],
            "what": "transcendental lane operations per second (counter run's instruction count x 64 "
                    "lanes, this run's kernel time) against the measured v_exp_f32 rate"}


def timed(fn, steps, stream, torch, before_last=None):
    """Run fn() `steps` times between synchronisations; HIP events on the
    launch stream bracket each call.  before_last() runs ahead of the last
    call, outside its event pair (it marks the outputs with sentinels, so
    that the statuses counted afterwards are the last call's own)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i, (e0, e1) in enumerate(evs):
        if before_last is not None and i == steps - 1:
            before_last()
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return wall, np.array([e0.elapsed_time(e1) for e0, e1 in evs])


def solved(rp, out) -> int:
    """Trajectories of `out` that ended CONVERGED or T_END; fails if any
    output still holds the sentinel of fill_sentinels (a dropped trajectory)."""
    left = rp.unfinished(out)
    if left:
        raise RuntimeError(f"{left} trajectories were never written")
    st = out.status.cpu().numpy()
    return int(np.isin(st, (rp.CONVERGED, rp.T_END)).sum())


def grow(run, n, n_max, target_s):
    """Run samples of growing size until one takes at least half of target_s
    (or covers the whole workload); return (size, seconds) of that one."""
    while True:
        k, w = run(n)
        if w >= 0.5 * target_s or k >= n_max:
            return k, w
        n = int(n * min(8.0, 1.1 * target_s / max(w, 1e-3)))


def cpu_oracle(topo, seed, n_sets, n_ic, n_pilot, opts_kw=None, t_out=None, target_s=12.0,
               gpu_steps=None):
    """The FP64 oracle on the host's cores over a seeded random sample of the
    workload's trajectories, grown from n_pilot until one sample takes about
    target_s seconds (capped at the whole workload), then one thread on a
    slice of that sample.  With gpu_steps (the GPU's accepted + rejected step
    counts per trajectory) it also reports their ratio to the oracle's on the
    sample."""
    import oracle
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    op = oracle.sample(net, seed, n_sets, n_ic)
    threads = min(os.cpu_count() or 1, 16)
    n_traj = n_sets * n_ic
    o = oracle.Opts(**(opts_kw or {"ss_rtol": 1e-5}))
    rng = np.random.default_rng(0)

    last = {}

    def run(n, n_threads=threads):
        ids = np.sort(rng.choice(n_traj, min(n, n_traj), replace=False))
        c0 = time.perf_counter()
        if t_out is None:
            r = oracle.steady_states(net, op, o, traj_ids=ids, n_threads=n_threads)
        else:
            r = oracle.time_series(net, op, t_out, o, traj_ids=ids, n_threads=n_threads)
        last.update(ids=ids, res=r)
        return ids.size, time.perf_counter() - c0

    n1, cw = grow(run, n_pilot, n_traj, target_s)
    rec = {"value": n1 / cw, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{n1} seeded random trajectories of the same workload, FP64 DP5(4), "
                     f"{threads} threads, {cw:.1f} s wall",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if gpu_steps is not None:
        r, ids = last["res"], last["ids"]
        rec["steps_gpu_over_oracle"] = float(np.asarray(gpu_steps)[ids].sum()
                                             / max(1, int((r.n_acc.astype(np.int64) + r.n_rej).sum())))
    k1, w1 = run(max(1, n1 // (4 * threads)), 1)
    rec["single_thread"] = {"value": k1 / w1, "unit": "solves/s",
                            "sample": f"{k1} seeded random trajectories, {w1:.1f} s wall"}
    return rec


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parity_report(topo, seed, n_sets, n_ic, ids, x_rows, opts_kw, t_out=None):
    """The FP64 oracle on trajectories `ids` of the workload against the GPU's
    results for them (x_rows, host, same order): the per-component error
    normalised by G/k (the parity metric, tolerance 1e-4) and the plain
    relative error.  A report for the bench line; the parity tests are the
    pass/fail checks (they also adjudicate basin flips near separatrices and
    stops on slow manifolds)."""
    import oracle
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    op = oracle.sample(net, seed, n_sets, n_ic)
    o = oracle.Opts(**opts_kw)
    threads = min(os.cpu_count() or 1, 16)
    if t_out is None:
        ref = oracle.steady_states(net, op, o, traj_ids=ids, n_threads=threads)
    else:
        ref = oracle.time_series(net, op, t_out, o, traj_ids=ids, n_threads=threads)
    gk = (op.G.astype(np.float64) / op.k.astype(np.float64)).T[ids // n_ic]
    if t_out is not None:
        gk = gk[:, None, :]
    x = np.asarray(x_rows, dtype=np.float64)
    d = np.abs(x - ref.x)
    err = d / gk
    rel = d / np.maximum(np.abs(ref.x), 1e-12)
    # The step control is relative only where |x| >= atol / rtol (1e-9 / 1e-6
    # by default); below that it bounds the absolute error, and the plain
    # relative error of a level near zero says little.
    floor = opts_kw.get("atol", 1e-9) / opts_kw.get("rtol", 1e-6)
    rel_c = np.where(np.abs(ref.x) >= floor, rel, 0.0)
    per_traj = err.reshape(len(ids), -1).max(axis=1)
    rec = {"n": int(len(ids)), "max_norm_err": float(err.max()),
           "p99_norm_err": float(np.percentile(err, 99)),
           "rel_p50": float(np.percentile(rel, 50)), "rel_p99": float(np.percentile(rel, 99)),
           "rel_max": float(rel.max()), "rel_max_where_x_ge_atol_over_rtol": float(rel_c.max()),
           "trajectories_over_1e-4": int((per_traj > 1e-4).sum()),
           "what": "GPU FP32 vs the FP64 oracle on a seeded sample; error = |x_gpu - x_ref| / (G/k) "
                   "per component"}
    if t_out is not None:
        # Per output time over the sample and the genes (3 significant digits).
        r3 = lambda a: [float(f"{v:.3g}") for v in a]
        rec["per_time"] = {"t": r3(t_out), "max_norm_err": r3(err.max(axis=(0, 2))),
                           "max_rel_err": r3(rel.max(axis=(0, 2))),
                           "rel_p99": r3(np.percentile(rel, 99, axis=(0, 2))),
                           "max_rel_err_where_x_ge_atol_over_rtol": r3(rel_c.max(axis=(0, 2))),
                           "what": "at every output time: the largest normalised error, the "
                                   "largest plain relative error |x_gpu - x_ref| / max(|x_ref|, 1e-12), "
                                   "its 99th percentile over the sample's components, and the largest "
                                   "over components with |x_ref| >= atol / rtol, where the step control "
                                   "is relative (below it the control bounds the absolute error)"}
    return rec


def cpu_oracle_multi(nets, n_pilot, target_s=12.0):
    """cpu_oracle over several networks: nets = [(topo, seed, n_sets, n_ic)];
    the sample draws trajectories across networks in proportion to their
    counts."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    prepared = []
    for topo, seed, P, n_ic in nets:
        net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
        prepared.append((net, oracle.sample(net, seed, P, n_ic), P * n_ic))
    sizes = np.array([n for _, _, n in prepared], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    o = oracle.Opts(ss_rtol=1e-5)
    rng = np.random.default_rng(0)

    def run(n, n_threads=threads):
        ids = np.sort(rng.choice(int(starts[-1]), min(n, int(starts[-1])), replace=False))
        c0 = time.perf_counter()
        for i, (net, op, _) in enumerate(prepared):
            sel = ids[(ids >= starts[i]) & (ids < starts[i + 1])] - starts[i]
            if sel.size:
                oracle.steady_states(net, op, o, traj_ids=sel, n_threads=n_threads)
        return ids.size, time.perf_counter() - c0

    n1, cw = grow(run, n_pilot, int(starts[-1]), target_s)
    rec = {"value": n1 / cw, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{n1} seeded random trajectories across the workload's networks, FP64 "
                     f"DP5(4), {threads} threads, {cw:.1f} s wall",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    k1, w1 = run(max(1, n1 // (4 * threads)), 1)
    rec["single_thread"] = {"value": k1 / w1, "unit": "solves/s",
                            "sample": f"{k1} seeded random trajectories, {w1:.1f} s wall"}
    return rec


def serving_parity(reqs, rng, per_request=20):
    """GPU results of sampled serving requests against the FP64 oracle:
    parity_report on seeded trajectories of each request."""
    reps = []
    for req in reqs:
        ids = np.sort(rng.choice(req.n_traj, min(per_request, req.n_traj), replace=False))
        x = req.result.x.cpu().numpy()[ids]
        reps.append(parity_report(req.topo, req.seed, req.n_sets, req.n_ic, ids, x, {"ss_rtol": 1e-5}))
    if not reps:
        return {}
    return {"requests": len(reps), "n": sum(r["n"] for r in reps),
            "max_norm_err": max(r["max_norm_err"] for r in reps),
            "trajectories_over_1e-4": sum(r["trajectories_over_1e-4"] for r in reps),
            "what": "a seeded 1 % of the measured requests, 20 seeded trajectories each (all of smaller "
                    "ones), GPU FP32 vs the FP64 oracle; error = |x_gpu - x_ref| / (G/k) per component"}


def serving_run(n_req, warm, rate, seed=5, budget=64 << 30, batch_steps=512, check_parity=True):
    from paper_2503_18356_amd.serve import GpuExecutor, Scheduler, poisson_requests
    rng = np.random.default_rng(seed)
    reqs = poisson_requests(rng, n_req + warm, rate=rate)
    ex = GpuExecutor(batch_steps=batch_steps, keep_results=False)
    # A seeded 1 % of the measured requests keep their results for parity.
    prng = np.random.default_rng(seed + 1)
    ex.keep_rids = set(int(r) for r in prng.choice(np.arange(warm, n_req + warm), max(1, n_req // 100),
                                                  replace=False))
    sched = Scheduler(ex, hbm_budget=budget)
    t0 = time.perf_counter()
    sched.run(reqs, max_seconds=900, progress=lambda m: print(m, file=sys.stderr, flush=True))
    st = sched.stats(skip=warm)
    if check_parity:
        st["parity"] = serving_parity([r for r in sched.done if r.rid in ex.keep_rids], prng)
    st.update({"offered_req_per_s": rate, "warmup_requests": warm, "wall_s": time.perf_counter() - t0,
               "kernel_classes": len(ex.classes), "batch_steps": batch_steps,
               "what": "Poisson arrivals of random networks (N log-uniform 2-100, E = 2.5N, "
                       "P log-uniform 1e2-1e5, n_ic U{1..10}); latency = arrival to last "
                       "trajectory done; continuous batching in hipGraph step batches"})
    return st


def base_record(args):
    return {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic"}


def bench_er10(args, torch, rp, flops, inputs):
    dev = torch.device("cuda:0")
    topo = inputs.erdos_renyi(10, 25, seed=1002, inhib_frac=0.5)
    T = rp.Topology.from_inputs(topo)
    t0 = time.time()
    hp = rp.sample_params(T, 2002, args.n_sets, args.n_ic)
    t_sample = time.time() - t0
    dp = hp.to_device(dev)
    n_traj = args.n_sets * args.n_ic
    opts = rp.Opts(precision=rp.FP32, lanes_per_traj=args.lanes, refill_min=args.refill_min)
    out = rp.alloc_result(n_traj, T.n_genes, rp.FP32, device=dev)
    stream = torch.cuda.current_stream()
    step = lambda: rp.steady_states(T, dp, opts, out=out, stream=stream)
    for _ in range(args.warmup):
        step()
    wall, lat = timed(step, args.steps, stream, torch, before_last=lambda: rp.fill_sentinels(out))
    value = solved(rp, out) * args.steps / wall
    nacc = out.n_acc.cpu().numpy().astype(np.int64)
    nrej = out.n_rej.cpu().numpy().astype(np.int64)
    x_er10 = out.x.cpu().numpy()
    achieved = flops.credited(T.n_genes, hp.n, args.n_ic, nacc + nrej) / (lat.mean() * 1e-3)
    nbytes = flops.algorithmic_bytes(T.n_genes, T.n_edges, args.n_sets, args.n_ic, 4)
    default_cfg = (args.n_sets, args.n_ic, args.lanes, args.refill_min) == (10000, 100, 0, 0)
    st = out.status.cpu().numpy()
    rec = base_record(args)
    rec.update({
        "value": value, "unit": "solves/s", "ms_per_step": wall / args.steps * 1e3,
        "config": {
            "workload": "steady states, random 10-gene/25-edge signed network (ER, 50% inhibitory), "
                        "10000 parameter sets x 100 initial conditions = 1e6 trajectories, Table 1 "
                        "ranges, DP5(4) rtol 1e-6 atol 1e-9 t_end 200",
            "n_genes": T.n_genes, "n_edges": T.n_edges, "n_sets": args.n_sets, "n_ic": args.n_ic,
            "lanes_per_traj": args.lanes or T.auto_lanes(rp.FP32),
            "precision": "FP32 state/RHS, FP64 t, error norm, steady test"},
        "roofline": {
            "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "frac_of_unpacked_fma_peak": achieved / PEAK_FP32_UNPACKED,
            "traffic": measured_traffic("er10_1e6_fp32") if default_cfg else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": nbytes,
            "hbm_frac": nbytes / (lat.mean() * 1e-3) / PEAK_HBM},
        "kernel_ms": {"mean": float(lat.mean()), "p50": float(np.percentile(lat, 50)),
                      "p99": float(np.percentile(lat, 99))},
        "status_counts": {rp.STATUS_NAMES[i]: int(c) for i, c in enumerate(np.bincount(st, minlength=5))},
        "steps_per_solve": float((nacc + nrej).mean()),
        "host_sampling_s": t_sample,
    })
    if not args.no_ceilings:
        # Secondary ceilings measured on this device (unpacked FP32 FMA, the
        # transcendentals, FP64 FMA), beside the published peaks.
        c = ceilings(rp, args)
        rec["measured_ceilings"] = {
            "fp32_fma_tflops": 2 * c["fp32_fma"] / 1e12,
            "v_exp_f32_tops": c["v_exp_f32"] / 1e12, "v_log_f32_tops": c["v_log_f32"] / 1e12,
            "v_rcp_f32_tops": c["v_rcp_f32"] / 1e12, "fp64_fma_tflops": 2 * c["fp64_fma"] / 1e12,
            "what": "sustained rates of one-operation kernels built like the solver kernels (no packed "
                    "FP32), all lanes of the device; fp32_fma takes its operands from registers "
                    "(v_fma_f32, as the solver does)"}
        rec["roofline"]["frac_of_measured_fp32_fma"] = achieved / (2 * c["fp32_fma"])
        if default_cfg:
            rec["roofline"]["transcendental"] = transcendental_rate(rp, args, "er10_1e6_fp32",
                                                                    float(lat.mean()))
    if not args.no_plain:
        o64 = rp.Opts(precision=rp.FP64, ss_rtol=1e-5, lanes_per_traj=args.lanes)
        out64 = rp.alloc_result(n_traj, T.n_genes, rp.FP64, device=dev)
        s64 = lambda: rp.steady_states(T, dp, o64, out=out64, stream=stream)
        s64()
        w64, _ = timed(s64, 1, stream, torch, before_last=lambda: rp.fill_sentinels(out64))
        v64 = solved(rp, out64) / w64
        steps64 = out64.n_acc.cpu().numpy().astype(np.int64) + out64.n_rej.cpu().numpy()
        fl64 = flops.credited(T.n_genes, hp.n, args.n_ic, steps64) / w64
        rec["plain_fp64"] = {"value": v64, "unit": "solves/s", "ms_per_step": w64 * 1e3,
                             "what": "FP64 state and RHS, same kernel family, same steady criterion",
                             "steps_per_solve": float(steps64.mean()),
                             "credited_fp64_tflops": fl64 / 1e12,
                             "frac_of_fp64_peak": fl64 / PEAK_FP64}
        if "measured_ceilings" in rec:
            rec["plain_fp64"]["frac_of_measured_fp64_fma"] = fl64 / (rec["measured_ceilings"]["fp64_fma_tflops"] * 1e12)
        rec["speedup_fp32_vs_fp64"] = value / v64
        del out64
    if not args.no_plain:
        # Post-processing of the 10^6 steady states on the device (normalise,
        # levels, codes, multistability, state counts): HBM-bound.
        post = lambda: rp.analyse_steady_states(T, dp, out, 64, 2, 1 << 16, stream=stream)
        post()
        w_pp, lat_pp = timed(post, 5, stream, torch)
        nb = flops.postproc_bytes(T.n_genes, args.n_sets, args.n_ic, n_bins=64,
                                  capacity=rp.state_table_size(n_traj, T.n_genes, 2, 1 << 16))
        rec["postproc"] = {
            "ms": float(lat_pp.mean()), "algorithmic_bytes": nb,
            "achieved_GBps": nb / (lat_pp.mean() * 1e-3) / 1e9, "peak_GBps": PEAK_HBM / 1e9,
            "frac": nb / (lat_pp.mean() * 1e-3) / PEAK_HBM,
            "what": "normalise + histogram/thresholds + levels/codes + multistability + state counts "
                    "of the 1e6 x 10 steady states, 64 bins, 2 levels"}
    if not args.no_plain:
        # The same workload with the paper's own solver (Tsitouras 5(4)).
        o_ts = rp.Opts(precision=rp.FP32, method=rp.TSIT5, lanes_per_traj=args.lanes,
                       refill_min=args.refill_min)
        step_ts = lambda: rp.steady_states(T, dp, o_ts, out=out, stream=stream)
        step_ts()
        w_ts, lat_ts = timed(step_ts, max(1, args.steps), stream, torch, before_last=lambda: rp.fill_sentinels(out))
        rec["tsit5_fp32"] = {
            "value": solved(rp, out) * max(1, args.steps) / w_ts, "unit": "solves/s",
            "kernel_ms": float(lat_ts.mean()),
            "steps_per_solve": float((out.n_acc.cpu().numpy().astype(np.int64)
                                      + out.n_rej.cpu().numpy()).mean()),
            "what": "FP32 chosen form with the Tsitouras 5(4) pair instead of Dormand-Prince"}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_oracle(topo, 2002, args.n_sets, args.n_ic, args.cpu_sample or 20000,
                                          gpu_steps=nacc + nrej, target_s=args.cpu_seconds)
        ids = np.sort(np.random.default_rng(1).choice(n_traj, min(n_traj, 10000), replace=False))
        rec["parity"] = parity_report(topo, 2002, args.n_sets, args.n_ic, ids, x_er10[ids],
                                      {"ss_rtol": 1e-5})
    return rec


def bench_ts(args, torch, rp, flops, inputs):
    topo = inputs.toggle_switch()
    T = rp.Topology.from_inputs(topo)
    hp = rp.sample_params(T, 2001, 1000, 10)
    dp = hp.to_device()
    stream = torch.cuda.current_stream()
    res = {}
    for name, o in (("fp64_plain", rp.Opts(precision=rp.FP64)), ("fp32", rp.Opts(precision=rp.FP32))):
        out = rp.alloc_result(10000, 2, o.precision)
        fn = lambda: rp.steady_states(T, dp, o, out=out, stream=stream)
        fn()
        wall, lat = timed(fn, args.steps, stream, torch, before_last=lambda: rp.fill_sentinels(out))
        res[name] = {"solves_per_s": solved(rp, out) * args.steps / wall,
                     "kernel_ms": float(lat.mean())}
        x_last = out.x.cpu().numpy()
    rec = base_record(args)
    rec.update({"value": res["fp32"]["solves_per_s"], "unit": "solves/s",
                "ms_per_step": res["fp32"]["kernel_ms"],
                "config": {"workload": "toggle switch (A -| B, B -| A), 1000 sets x 10 ICs, "
                                       "FP64 plain (steady |f| < 1e-6) and FP32"},
                "forms": res})
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_oracle(topo, 2001, 1000, 10, 2000, {"ss_rtol": 0.0}, target_s=args.cpu_seconds)
        # The whole ensemble, FP32 form (the last one run) against the oracle
        # with the FP32 steady criterion.
        rec["parity"] = parity_report(topo, 2001, 1000, 10, np.arange(10000), x_last, {"ss_rtol": 1e-5})
    return rec


def uneven64_inputs(rp, inputs):
    """The 64-network uneven batch: topologies, parameter-set counts, seeds."""
    rng = np.random.default_rng(1003)
    topos = inputs.uneven_batch(1003, n_networks=64, n_min=5, n_max=50)
    Ps = [inputs.log_uniform_int(rng, 2000, 50000) for _ in topos]
    return topos, Ps


def bench_uneven64(args, torch, rp, flops, inputs):
    topos, Ps = uneven64_inputs(rp, inputs)
    Ts = [rp.Topology.from_inputs(t) for t in topos]
    t0 = time.time()
    items = []
    for i, (T, P) in enumerate(zip(Ts, Ps)):
        items.append((T, rp.sample_params_device(T, 3000 + i, P, 10)))
    torch.cuda.synchronize()
    t_sample = time.time() - t0
    n_traj = sum(P * 10 for P in Ps)
    stream = torch.cuda.current_stream()
    o32 = rp.Opts(precision=rp.FP32, lanes_per_traj=args.lanes, refill_min=args.refill_min)
    outs = [rp.alloc_result(p.n_sets * 10, T.n_genes, rp.FP32) for T, p in items]
    fill = lambda: [rp.fill_sentinels(o) for o in outs]
    # Lane counts and refill batches: the library's cost model (default),
    # with the autotuner's per-network choices switched in class by class
    # where whole batch calls get faster (decided on untimed calls before
    # the timed ones).
    knobs = [(0, 0)] * len(items)
    tune_rec = None
    if not args.no_tune and args.lanes == 0 and args.refill_min == 0:
        import tempfile
        from paper_2503_18356_amd.autotune import Autotuner
        tu = Autotuner(os.path.join(tempfile.gettempdir(), f"racipe_autotune_{os.getpid()}.json"))
        t_tune = time.time()
        choices = tu.tune_batch(Ts, rp.FP32, n_ic=10)
        t_tune = time.time() - t_tune
        tuned = [(c.lanes, c.refill_min) for c in choices]

        def run_knobs(kn):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rp.steady_states_batch([(T, p, o, k) for (T, p), o, k in zip(items, outs, kn)], o32, stream=stream)
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) * 1e-3
        default_knobs = knobs
        # Networks grouped by the launch class the lane model gives them,
        # largest class first; each group switches to its tuned knobs only
        # if a whole batch call gets faster.
        n_total = sum(p.n_sets * 10 for _, p in items)
        cls = {}
        for i, (T, p) in enumerate(items):
            lanes = T.auto_lanes(rp.FP32, n_total)
            cls.setdefault((lanes, T.shape(lanes, rp.FP32)), []).append(i)
        groups = sorted(cls.values(), key=lambda g: -sum(items[i][1].n_sets for i in g))
        knobs, refine_log = Autotuner.refine_batch(run_knobs, default_knobs, tuned, groups)
        run_d = lambda: rp.steady_states_batch([(T, p, o) for (T, p), o in zip(items, outs)], o32, stream=stream)
        wall_d, lat_d = timed(run_d, args.steps, stream, torch, before_last=fill)
        tune_rec = {"seconds": t_tune,
                    "sample": "per network bucket, marginal solves/s between 2x and 4x the GPU's resident "
                              "trajectories, HIP-event timed; then per launch class of the lane model, "
                              "largest first, the tuned knobs kept only where a whole untimed batch call "
                              "runs more than 1 % faster",
                    "groups_switched": sum(1 for r in refine_log[1:] if r["kept"]),
                    "refine": refine_log,
                    "default_value": sum(solved(rp, o) for o in outs) * args.steps / wall_d,
                    "default_ms": float(lat_d.mean()),
                    "choices": [{"N": T.n_genes, "E": T.n_edges, "lanes_default": T.auto_lanes(rp.FP32),
                                 "lanes": c.lanes, "refill_min": c.refill_min, "shape": list(T.shape(c.lanes))}
                                for T, c in zip(Ts, choices)]}
    fn = lambda: rp.steady_states_batch([(T, p, o, k) for (T, p), o, k in zip(items, outs, knobs)], o32,
                                        stream=stream)
    for _ in range(max(1, args.warmup)):
        fn()
    wall, lat = timed(fn, args.steps, stream, torch, before_last=fill)
    v32 = sum(solved(rp, o) for o in outs) * args.steps / wall
    steps_all = [o.n_acc.cpu().numpy().astype(np.int64) + o.n_rej.cpu().numpy() for o in outs]
    ns = [p.n.cpu().numpy() for _, p in items]
    fl = sum(flops.credited(T.n_genes, n, 10, st) for (T, _), n, st in zip(items, ns, steps_all))
    launch_ms = float(lat.mean())
    achieved = fl / (launch_ms * 1e-3)
    nbytes = sum(flops.algorithmic_bytes(T.n_genes, T.n_edges, p.n_sets, 10, 4) for T, p in items)
    st_all = np.concatenate([o.status.cpu().numpy() for o in outs])
    default_cfg = args.lanes == 0 and args.refill_min == 0
    rec = base_record(args)
    rec.update({
        "value": v32, "unit": "solves/s", "ms_per_step": wall / args.steps * 1e3,
        "config": {"workload": "steady states of an uneven batch of 64 seeded random signed networks "
                               "(N ~ U{5..50}, E = 2.5N, half inhibitory, ER without isolated genes), "
                               "P log-uniform in [2000, 50000] parameter sets x 10 initial conditions "
                               "each, Table 1 ranges, DP5(4) rtol 1e-6 atol 1e-9 t_end 200, FP32 state "
                               "with FP64 t / error norm / steady test",
                   "trajectories": n_traj, "networks": len(items),
                   "genes": [T.n_genes for T in Ts]},
        "roofline": {
            "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "frac_of_unpacked_fma_peak": achieved / PEAK_FP32_UNPACKED,
            "traffic": measured_traffic("uneven64_fp32") if default_cfg else None,
            "traffic_unit": "bytes per batch call (rocprofv3 FETCH_SIZE + WRITE_SIZE over its launches, "
                            "copy-calibrated)",
            "algorithmic_bytes_per_launch": nbytes,
            "hbm_frac": nbytes / (launch_ms * 1e-3) / PEAK_HBM,
            "what": "credited FLOP of the whole batch call (all its persistent launches, overlapped on "
                    "four streams) over the call's duration between HIP events on the caller's stream, "
                    "which the call forks from and joins"},
        "kernel_ms": {"mean": launch_ms, "p50": float(np.percentile(lat, 50)),
                      "p99": float(np.percentile(lat, 99))},
        "status_counts": {rp.STATUS_NAMES[i]: int(c) for i, c in enumerate(np.bincount(st_all, minlength=5))},
        "steps_per_solve": float(np.concatenate(steps_all).mean()),
        "device_sampling_s": t_sample,
    })
    if default_cfg:
        rec["roofline"]["transcendental"] = transcendental_rate(rp, args, "uneven64_fp32", launch_ms)
    if tune_rec is not None:
        tune_rec["picked_over_default"] = v32 / tune_rec["default_value"]
        rec["autotune"] = tune_rec
    if not args.no_plain:
        o64 = rp.Opts(precision=rp.FP64, ss_rtol=1e-5)
        outs64 = [rp.alloc_result(p.n_sets * 10, T.n_genes, rp.FP64) for T, p in items]

        def plain():
            for (T, p), o in zip(items, outs64):
                rp.steady_states(T, p, o64, out=o, stream=stream)
        plain()
        w64, l64 = timed(plain, 1, stream, torch, before_last=lambda: [rp.fill_sentinels(o) for o in outs64])
        v64 = sum(solved(rp, o) for o in outs64) / w64
        fl64 = sum(flops.credited(T.n_genes, n, 10, o.n_acc.cpu().numpy().astype(np.int64) + o.n_rej.cpu().numpy())
                   for (T, _), n, o in zip(items, ns, outs64))
        rec["plain_fp64"] = {"value": v64, "unit": "solves/s", "ms": float(l64.mean()),
                             "credited_fp64_tflops": fl64 / (l64.mean() * 1e-3) / 1e12,
                             "frac_of_fp64_peak": fl64 / (l64.mean() * 1e-3) / PEAK_FP64,
                             "what": "FP64 state and RHS, one launch per network in sequence on one stream, "
                                     "same steady criterion"}
        rec["speedup_fp32_vs_fp64"] = v32 / v64
        del outs64
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_oracle_multi(
            [(t, 3000 + i, P, 10) for i, (t, P) in enumerate(zip(topos, Ps))], 4000, target_s=args.cpu_seconds)
        # 1 % of every network (at least 200 trajectories), seeded.
        reps = []
        prng = np.random.default_rng(2)
        worst = 0.0
        for i, (t, P, o) in enumerate(zip(topos, Ps, outs)):
            ids = np.sort(prng.choice(P * 10, max(200, P * 10 // 100), replace=False))
            idt = torch.from_numpy(ids).to(o.x.device)
            rep = parity_report(t, 3000 + i, P, 10, ids, o.x[idt].cpu().numpy(), {"ss_rtol": 1e-5})
            reps.append(rep)
        rec["parity"] = {"n": sum(r["n"] for r in reps),
                         "max_norm_err": max(r["max_norm_err"] for r in reps),
                         "p99_norm_err": max(r["p99_norm_err"] for r in reps),
                         "rel_max_where_x_ge_atol_over_rtol": max(r["rel_max_where_x_ge_atol_over_rtol"]
                                                                  for r in reps),
                         "trajectories_over_1e-4": sum(r["trajectories_over_1e-4"] for r in reps),
                         "networks": len(reps),
                         "what": "GPU FP32 vs the FP64 oracle on 1 % of every network (at least 200), "
                                 "seeded; error = |x_gpu - x_ref| / (G/k) per component; p99 is the "
                                 "worst network's"}
    if not args.no_plain:
        # The same batch with the paper's own solver (Tsitouras 5(4)), in its
        # own output buffers.
        o_ts = rp.Opts(precision=rp.FP32, method=rp.TSIT5)
        outs_ts = [rp.alloc_result(p.n_sets * 10, T.n_genes, rp.FP32) for T, p in items]
        fn_ts = lambda: rp.steady_states_batch([(T, p, o) for (T, p), o in zip(items, outs_ts)], o_ts,
                                               stream=stream)
        fn_ts()
        w_ts, l_ts = timed(fn_ts, max(1, args.steps), stream, torch,
                           before_last=lambda: [rp.fill_sentinels(o) for o in outs_ts])
        rec["tsit5_fp32"] = {
            "value": sum(solved(rp, o) for o in outs_ts) * max(1, args.steps) / w_ts, "unit": "solves/s",
            "kernel_ms": float(l_ts.mean()),
            "steps_per_solve": float(np.concatenate([o.n_acc.cpu().numpy().astype(np.int64)
                                                     + o.n_rej.cpu().numpy() for o in outs_ts]).mean()),
            "what": "FP32 chosen form with the Tsitouras 5(4) pair instead of Dormand-Prince, library lane "
                    "model"}
        del outs_ts
    return rec


def bench_core22ts(args, torch, rp, flops, inputs):
    topo = inputs.dense_core(1004)
    T = rp.Topology.from_inputs(topo)
    P, n_ic = 100000, 10
    hp = rp.sample_params(T, 2004, P, n_ic)
    dp = hp.to_device()
    tk = np.linspace(0.0, 100.0, 101)
    stream = torch.cuda.current_stream()
    o32 = rp.Opts(precision=rp.FP32)
    out = rp.alloc_result(P * n_ic, T.n_genes, rp.FP32, n_t=101)
    fn = lambda: rp.integrate(T, dp, tk, o32, out=out, stream=stream)
    fn()
    wall, lat = timed(fn, args.steps, stream, torch, before_last=lambda: rp.fill_sentinels(out))
    v32 = solved(rp, out) * args.steps / wall
    steps = out.n_acc.cpu().numpy().astype(np.int64) + out.n_rej.cpu().numpy()
    fl = flops.credited(T.n_genes, hp.n, n_ic, steps)
    # 1 % seeded sample of the series kept on the host for the parity report.
    par_ids = np.sort(np.random.default_rng(3).choice(P * n_ic, (P * n_ic) // 100, replace=False))
    x_par = out.x[torch.from_numpy(par_ids).to(out.x.device)].cpu().numpy()
    del out
    o64 = rp.Opts(precision=rp.FP64)
    out64 = rp.alloc_result(P * n_ic, T.n_genes, rp.FP64, n_t=101)
    f64 = lambda: rp.integrate(T, dp, tk, o64, out=out64, stream=stream)
    f64()
    w64, l64 = timed(f64, 1, stream, torch, before_last=lambda: rp.fill_sentinels(out64))
    v64 = solved(rp, out64) / w64
    steps64 = out64.n_acc.cpu().numpy().astype(np.int64) + out64.n_rej.cpu().numpy()
    fl64 = flops.credited(T.n_genes, hp.n, n_ic, steps64)
    del out64
    nbytes = flops.algorithmic_bytes(T.n_genes, T.n_edges, P, n_ic, 4, n_t=101)
    rec = base_record(args)
    rec.update({"value": v32, "unit": "solves/s", "ms_per_step": wall / args.steps * 1e3,
                "config": {"workload": "22-gene / 82-edge dense-core network (49 inhibitory), "
                                       "1e5 sets x 10 ICs, 101 outputs on [0, 100]",
                           "lanes_per_traj": T.auto_lanes()},
                "roofline": {"bound": "alu", "achieved": fl / (lat.mean() * 1e-3) / 1e12,
                             "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                             "frac": fl / (lat.mean() * 1e-3) / PEAK_FP32,
                             "frac_of_unpacked_fma_peak": fl / (lat.mean() * 1e-3) / PEAK_FP32_UNPACKED,
                             "traffic": measured_traffic("core22ts_fp32"),
                             "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                             "algorithmic_bytes_per_launch": nbytes,
                             "hbm_frac": nbytes / (lat.mean() * 1e-3) / PEAK_HBM},
                "plain_fp64": {"value": v64, "unit": "solves/s", "ms": float(l64.mean()),
                               "credited_fp64_tflops": fl64 / (l64.mean() * 1e-3) / 1e12,
                               "frac_of_fp64_peak": fl64 / (l64.mean() * 1e-3) / PEAK_FP64},
                "speedup_fp32_vs_fp64": v32 / v64})
    rec["roofline"]["transcendental"] = transcendental_rate(rp, args, "core22ts_fp32", float(lat.mean()))
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_oracle(topo, 2004, P, n_ic, 1000, {"ss_rtol": 1e-5}, t_out=tk,
                                         target_s=args.cpu_seconds)
        rec["parity"] = parity_report(topo, 2004, P, n_ic, par_ids, x_par, {"ss_rtol": 1e-5}, t_out=tk)
    return rec


PEAK_INT32 = 256 * 4 * 16 * 2.4e9   # 32-bit VALU lane-ops/s (unpacked)


def bench_ising(args, torch, rp, flops, inputs):
    """Boolean Ising (Eq. 3) on the 22-gene network: 10^6 random initial
    states, synchronous and asynchronous updates with +-1 states."""
    topo = inputs.dense_core(1004)
    T = rp.Topology.from_inputs(topo)
    n_traj, W = 1_000_000, 1
    rec = base_record(args)
    forms = {}
    stream = torch.cuda.current_stream()
    for mode, name, max_steps in ((rp.ISING_SYNC, "sync", 1000), (rp.ISING_ASYNC, "async", 20000)):
        out = {}
        fn = lambda: out.update(r=rp.ising(T, n_traj, mode, -1, max_steps, seed=7, stream=stream))
        fn()
        wall, lat = timed(fn, max(1, args.steps), stream, torch)
        fin, steps, status = out["r"]
        sp = steps.cpu().numpy().astype(np.int64)
        st = status.cpu().numpy()
        # Gene evaluations the kernel performs (counted on the device: a
        # periodic synchronous trajectory stops stepping once its cycle is
        # found), and those its results stand for (sync: N per update plus
        # the final check; async: one per update plus N per fixed-point test).
        ev = torch.zeros(1, dtype=torch.int64, device="cuda")
        rp.ising(T, n_traj, mode, -1, max_steps, seed=7, stream=stream, evals=ev)
        evals = int(ev.item())
        N = T.n_genes
        if mode == rp.ISING_SYNC:
            represented = int(((sp + 1) * N).sum())
        else:
            represented = int((sp + (sp // N + 1) * N).sum())
        ops = evals * (8 * W + 6)
        forms[name] = {"trajectories_per_s": n_traj / (lat.mean() * 1e-3), "kernel_ms": float(lat.mean()),
                       "fixed_point_fraction": float(np.mean(st == 0)),
                       "mean_updates": float(sp.mean()), "gene_evaluations": evals,
                       "gene_evaluations_represented": represented,
                       "gene_evaluations_per_s": evals / (lat.mean() * 1e-3),
                       "int_ops_per_s": ops / (lat.mean() * 1e-3), "int_frac": ops / (lat.mean() * 1e-3) / PEAK_INT32}
    rec.update({"value": forms["sync"]["trajectories_per_s"], "unit": "trajectories/s",
                "metric": "Boolean Ising trajectories to a fixed point per second",
                "ms_per_step": forms["sync"]["kernel_ms"],
                "config": {"workload": "Boolean Ising, 22-gene / 82-edge dense-core network, 1e6 random "
                                       "initial states, +-1 states, sync (<= 1000 updates) and async "
                                       "(<= 20000 single-gene updates)"},
                "forms": forms,
                "roofline": {"bound": "alu", "achieved": forms["sync"]["int_ops_per_s"] / 1e12,
                             "peak": PEAK_INT32 / 1e12, "unit": "Tops/s (int32 VALU)",
                             "frac": forms["sync"]["int_frac"], "traffic": None}})
    return rec


def bench_serve(args, torch, rp, flops, inputs):
    st = serving_run(args.serve_requests, args.serve_warmup, args.serve_rate)
    rec = base_record(args)
    rec.update({"value": st["solves_per_s"], "unit": "solves/s", "ms_per_step": None,
                "latency_ms": {"p50": st["p50_ms"], "p99": st["p99_ms"]},
                "config": {"workload": f"serving: Poisson request stream at {args.serve_rate:g} req/s"},
                "serving": st})
    if args.serve_stable_rate > 0:
        # The offered stream above can exceed capacity (the queue then grows
        # and p99 measures the backlog); also serve at a lower stated rate.
        rec["serving_lower_rate"] = serving_run(args.serve_requests, args.serve_warmup,
                                                args.serve_stable_rate)
    return rec


EXTRA_DROP = ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
              "dtype", "data")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven64",
                    choices=["er10", "ts", "uneven64", "core22ts", "serve", "ising"])
    ap.add_argument("--no-extras", action="store_true",
                    help="uneven64 only: skip the other configurations and serving")
    ap.add_argument("--n-sets", type=int, default=10000)
    ap.add_argument("--n-ic", type=int, default=100)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--refill-min", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="uneven64: the library's lane model instead of the autotuner's choices")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-stable-rate", type=float, default=100.0)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle trajectories (0 = auto)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of one CPU-oracle sample")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the VALU ceiling microbenchmarks (FP32 FMA, transcendentals, FP64 FMA)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy, whose FETCH_SIZE/WRITE_SIZE "
                         "counters scale the kernel's HBM traffic figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (trajectories are "
              "independent, so several GPUs would each take a share of the ensemble)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_18356_amd import flops, inputs
    from paper_2503_18356_amd import racipe as rp

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fn = {"er10": bench_er10, "ts": bench_ts, "uneven64": bench_uneven64,
          "core22ts": bench_core22ts, "serve": bench_serve, "ising": bench_ising}[args.workload]
    rec = fn(args, torch, rp, flops, inputs)
    if args.workload == "uneven64" and not args.no_extras:
        extras = {}
        for name, f in (("c2_er10_1e6", bench_er10), ("c4_core22_series_1e6", bench_core22ts),
                        ("c1_toggle_switch_1e4", bench_ts)):
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            r = f(args, torch, rp, flops, inputs)
            extras[name] = {k: v for k, v in r.items() if k not in EXTRA_DROP}
            torch.cuda.empty_cache()
        rec["extras"] = extras
        if not args.no_serve:
            print("[bench] serving", file=sys.stderr, flush=True)
            rec["serving"] = serving_run(args.serve_requests, args.serve_warmup, args.serve_rate)
            rec["latency_ms"] = {"p50": rec["serving"]["p50_ms"], "p99": rec["serving"]["p99_ms"],
                                 "what": "serving request latency (arrival to last trajectory done) at "
                                         f"{args.serve_rate:g} requests/s offered, {args.serve_requests} "
                                         f"requests after {args.serve_warmup} warm-up"}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
