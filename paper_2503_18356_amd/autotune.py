"""Autotuner for the launch knobs of the DP5 kernel.

Knobs: lanes per trajectory, which fixes the lane plan and with it the
compiled kernel shape (edge slots and gene slots per lane: the register
budget and the per-wave LDS tile), and the refill batch (how many trajectory
groups of a wave must be free before it pulls new work).  For a network it
measures every combination within a factor of two of the library's lane
model and keeps the fastest.  What is measured is the marginal throughput
with the GPU full: solves of n and 2n trajectories, n twice what the GPU
holds resident at that lane count, timed with HIP events on the launch
stream, give 1 / (per-trajectory cost) = n / (t(2n) - t(n)).  The difference
cancels the launch cost and the drain at the end of a launch, which a
network inside a large batch does not pay on its own; a plain timing of a
small sample counts them and so favours more lanes per trajectory than a
full GPU wants.  Choices are cached as JSON per (GPU architecture,
precision, network bucket), where the bucket is (N, E, largest in-degree)
rounded up to powers of two, so similar networks reuse a measurement;
tune_batch() gives the per-network choices that rac_steady_states_batch
takes per item, and pick_faster() checks them against the lane model on
the real batch.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass

import numpy as np

from . import racipe as rp

DEFAULT_CACHE = os.environ.get("RACIPE_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "racipe", "autotune.json"))
LANES = (1, 2, 4, 8, 16, 32, 64)
# Waves the GPU holds resident at the usual occupancy (256 CUs x 4 SIMDs x 4
# waves per SIMD): the measured samples are sized against it.
RESIDENT_WAVES = 4096


def _pow2(v: int) -> int:
    return 1 << max(0, int(v - 1).bit_length())


def bucket(topo) -> str:
    indeg = np.bincount(topo.dst, minlength=topo.n_genes).max() if topo.n_edges else 0
    return f"N{_pow2(topo.n_genes)}_E{_pow2(max(topo.n_edges, 1))}_D{_pow2(max(int(indeg), 1))}"


def arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


@dataclass
class Choice:
    lanes: int
    refill_min: int
    solves_per_s: float


class Autotuner:
    def __init__(self, cache_path: str = DEFAULT_CACHE):
        self.path = cache_path
        self.cache = {}
        if os.path.exists(cache_path):
            # A cache that cannot be read (cut short, edited by hand) is
            # dropped and measured again rather than failing the caller.
            try:
                with open(cache_path) as f:
                    c = json.load(f)
                if isinstance(c, dict):
                    self.cache = c
            except (OSError, ValueError):
                self.cache = {}

    def _key(self, topo, precision: int) -> str:
        return f"{arch()}|{'fp32' if precision == rp.FP32 else 'fp64'}|{bucket(topo)}"

    def save(self):
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def candidates(self, T, precision: int, span: int = 2):
        """(lanes, refill) pairs: lane counts within a factor `span` of the
        lane model's choice, each with four refill batches."""
        d = T.auto_lanes(precision)
        out = []
        for lanes in LANES:
            if d // span <= lanes <= d * span and T.lanes_supported(lanes, precision):
                groups = 64 // lanes
                for rm in sorted({max(1, groups // 8), max(1, groups // 4), max(1, groups // 2), groups}):
                    out.append((lanes, rm))
        return out

    def measure(self, T, precision: int, n_ic: int = 10, seed: int = 1, reps: int = 2,
                opts: rp.Opts | None = None, n_sets: int | None = None, span: int = 2) -> list[Choice]:
        """Marginal solves/s of every candidate: best of `reps` HIP-event
        timings of n and of 2n trajectories after one untimed run, with n =
        2 x RESIDENT_WAVES x 64 / lanes (or n_sets x n_ic when given)."""
        import torch
        base = opts or rp.Opts(precision=precision)
        stream = torch.cuda.current_stream()
        dev = torch.device("cuda", torch.cuda.current_device())

        def timed(params, o, out):
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rp.steady_states(T, params, o, out=out, stream=stream)
                e1.record(stream)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e-3)
            return best

        res = []
        per_lanes = {}
        for lanes, rm in self.candidates(T, precision, span):
            if lanes not in per_lanes:
                s1 = n_sets or -(-2 * RESIDENT_WAVES * (64 // lanes) // n_ic)
                p1 = rp.sample_params_device(T, seed, s1, n_ic)
                p2 = rp.sample_params_device(T, seed, 2 * s1, n_ic)
                out = rp.alloc_result(2 * s1 * n_ic, T.n_genes, precision, device=dev)
                per_lanes[lanes] = (p1, p2, out)
            p1, p2, out = per_lanes[lanes]
            o = rp.Opts(**{**base.__dict__, "precision": precision, "lanes_per_traj": lanes,
                           "refill_min": rm})
            rp.steady_states(T, p2, o, out=out, stream=stream)
            t1, t2 = timed(p1, o, out), timed(p2, o, out)
            n1 = p1.n_sets * n_ic
            # A difference lost in timing noise falls back to the plain rate.
            rate = n1 / (t2 - t1) if t2 > 1.2 * t1 else 2 * n1 / t2
            res.append(Choice(lanes, rm, rate))
        return res

    def tune(self, topo, precision: int = rp.FP32, force: bool = False, **kw) -> Choice:
        """Best (lanes, refill_min) for this network's bucket, measuring if needed."""
        T = topo if isinstance(topo, rp.Topology) else rp.Topology.from_inputs(topo)
        key = self._key(T, precision)
        if key in self.cache and not force:
            c = self.cache[key]
            if T.lanes_supported(c["lanes"], precision):
                return Choice(c["lanes"], c["refill_min"], c["solves_per_s"])
        results = self.measure(T, precision, **kw)
        best = max(results, key=lambda c: c.solves_per_s)
        self.cache[key] = {"lanes": best.lanes, "refill_min": best.refill_min,
                           "solves_per_s": best.solves_per_s,
                           "all": [[c.lanes, c.refill_min, c.solves_per_s] for c in results]}
        self.save()
        return best

    def tune_batch(self, topos, precision: int = rp.FP32, **kw) -> list[Choice]:
        """Choices for every network of a batch (one measurement per bucket)."""
        return [self.tune(t, precision, **kw) for t in topos]

    def opts(self, topo, precision: int = rp.FP32, base: rp.Opts | None = None, **kw) -> rp.Opts:
        c = self.tune(topo, precision, **kw)
        b = base or rp.Opts(precision=precision)
        return rp.Opts(**{**b.__dict__, "precision": precision, "lanes_per_traj": c.lanes,
                          "refill_min": c.refill_min})

    @staticmethod
    def pick_faster(run, tuned, default, reps: int = 2):
        """Whichever of two per-item knob lists runs a whole batch faster:
        run(knobs) solves the batch once and returns its seconds.  The batch
        is the final judge because per-network measurements miss how the
        networks share launches; each list is run once untimed first."""
        t = {}
        for name, knobs in (("default", default), ("tuned", tuned)):
            run(knobs)
            t[name] = min(run(knobs) for _ in range(reps))
        return (tuned if t["tuned"] < t["default"] else default), t

    @staticmethod
    def refine_batch(run, default, tuned, groups, reps: int = 2, margin: float = 0.01):
        """Greedy refinement on the whole batch: starting from the default
        knob list, switch one group of items (e.g. the networks of one
        launch class of the default plan, largest first) to its tuned
        knobs, and keep the switch when a whole batch call runs more than
        `margin` faster than the best so far.  run(knobs) solves the batch
        once and returns its seconds; each timing is the best of `reps`
        after one untimed call.  Returns (knobs, log)."""
        def best_of(knobs):
            run(knobs)
            return min(run(knobs) for _ in range(reps))
        current = list(default)
        t_best = best_of(current)
        log = [{"group": None, "ms": t_best * 1e3, "kept": True}]
        for g in groups:
            if all(tuned[i] == current[i] for i in g):
                continue
            trial = list(current)
            for i in g:
                trial[i] = tuned[i]
            t = best_of(trial)
            kept = t < t_best * (1.0 - margin)
            log.append({"group": list(g), "ms": t * 1e3, "kept": kept})
            if kept:
                current, t_best = trial, t
        return current, log
