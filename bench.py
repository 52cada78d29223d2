"""RACIPE ensemble benchmark on one MI355X.

Workload (one "step"): steady states of every trajectory of a seeded random
10-gene / 25-edge signed network (Erdos-Renyi, half inhibitory, no isolated
node), 10,000 parameter sets x 100 initial conditions = 10^6 trajectories,
parameters from the Table 1 ranges (GRiNS Sec. 2.1.2), rtol 1e-6, atol 1e-9,
t_end 200, steady when |dx_i/dt| <= 1e-6 + 1e-5 k_i |x_i|.  Parameters and
initial conditions are resident in HBM before timing starts.

Reported: solves/s of the chosen form (FP32 state, FP64 time / error norm /
steady test, persistent work-queue kernel), the plain FP64 form on the same
workload, the kernel's credited FP32 FLOP/s against the MI355X vector peak,
and the CPU oracle timed on a bounded sample on this host.
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
PEAK_FP32 = 157.3e12   # MI355X FP32 vector, TFLOP/s (packed)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-sets", type=int, default=10000)
    ap.add_argument("--n-ic", type=int, default=100)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--refill-min", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle trajectories (0 = auto)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy, whose FETCH_SIZE/WRITE_SIZE "
                         "counters scale the kernel's HBM traffic figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(trajectories are independent; see the sharding note in the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_18356_amd import inputs, flops
    from paper_2503_18356_amd import racipe as rp

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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

    def step(o, res):
        rp.steady_states(T, dp, o, out=res, stream=stream)

    for _ in range(args.warmup):
        step(opts, out)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step(opts, out)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    lat = np.array([e0.elapsed_time(e1) for e0, e1 in evs])  # ms per launch
    st = out.status.cpu().numpy()
    nacc = out.n_acc.cpu().numpy().astype(np.int64)
    nrej = out.n_rej.cpu().numpy().astype(np.int64)
    solved = int(np.isin(st, (rp.CONVERGED, rp.T_END)).sum())
    value = solved * args.steps / wall
    fl = flops.credited(T.n_genes, hp.n, args.n_ic, nacc + nrej)
    achieved = fl / (lat.mean() * 1e-3)
    bytes_per_launch = flops.algorithmic_bytes(T.n_genes, T.n_edges, args.n_sets, args.n_ic, 4)

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "steady states, random 10-gene/25-edge signed network (ER, 50% inhibitory), "
                        "10000 parameter sets x 100 initial conditions = 1e6 trajectories, Table 1 "
                        "ranges, DP5(4) rtol 1e-6 atol 1e-9 t_end 200",
            "n_genes": T.n_genes, "n_edges": T.n_edges, "n_sets": args.n_sets, "n_ic": args.n_ic,
            "lanes_per_traj": args.lanes or T.auto_lanes(rp.FP32),
            "precision": "FP32 state/RHS, FP64 t, error norm, steady test",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": measured_traffic("er10_1e6_fp32") if (args.n_sets, args.n_ic, args.lanes) == (10000, 100, 0) else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "hbm_frac": bytes_per_launch / (lat.mean() * 1e-3) / PEAK_HBM,
        },
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one full-ensemble call, enqueue to completion"},
        "status_counts": {rp.STATUS_NAMES[i]: int(c) for i, c in enumerate(np.bincount(st, minlength=5))},
        "steps_per_solve": float((nacc + nrej).mean()),
        "host_sampling_s": t_sample,
    }

    if not args.no_plain:
        o64 = rp.Opts(precision=rp.FP64, ss_rtol=1e-5)
        out64 = rp.alloc_result(n_traj, T.n_genes, rp.FP64, device=dev)
        step(o64, out64)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        step(o64, out64)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - w0
        st64 = out64.status.cpu().numpy()
        s64 = int(np.isin(st64, (rp.CONVERGED, rp.T_END)).sum())
        rec["plain_fp64"] = {"value": s64 / w64, "unit": "solves/s", "ms_per_step": w64 * 1e3,
                             "what": "FP64 state and RHS, same kernel family, same steady criterion",
                             "steps_per_solve": float((out64.n_acc.cpu().numpy().astype(np.int64)
                                                       + out64.n_rej.cpu().numpy()).mean())}
        rec["speedup_fp32_vs_fp64"] = value / (s64 / w64)

    if not args.no_cpu:
        import oracle
        net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
        op = oracle.sample(net, 2002, args.n_sets, args.n_ic)
        threads = min(os.cpu_count() or 1, 16)
        n_cpu = args.cpu_sample or 40000
        ids = np.sort(np.random.default_rng(0).choice(n_traj, min(n_cpu, n_traj), replace=False))
        c0 = time.perf_counter()
        ref = oracle.steady_states(net, op, oracle.Opts(ss_rtol=1e-5), traj_ids=ids, n_threads=threads)
        cw = time.perf_counter() - c0
        rec["cpu_baseline"] = {"value": ids.size / cw, "unit": "solves/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{ids.size} seeded random trajectories of the same "
                                         f"workload, FP64 DP5(4), {cw:.1f} s wall"}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
