"""Autotuner for the launch knobs of the DP5 kernel.

Knobs: lanes per trajectory, which fixes the lane plan and with it the
compiled kernel shape (edge slots and gene slots per lane: the register
budget and the per-wave LDS tile), and the refill batch (how many trajectory
groups of a wave must be free before it pulls new work).  For a network it
times solves of a parameter-set sample at every feasible combination, with
HIP events on the launch stream, and keeps the fastest.  Choices are cached
as JSON per (GPU architecture, precision, network bucket), where the bucket
is (N, E, largest in-degree) rounded up to powers of two, so similar
networks reuse a measurement; tune_batch() gives the per-network choices
that rac_steady_states_batch takes per item.
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
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _key(self, topo, precision: int) -> str:
        return f"{arch()}|{'fp32' if precision == rp.FP32 else 'fp64'}|{bucket(topo)}"

    def save(self):
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def candidates(self, T, precision: int):
        out = []
        for lanes in LANES:
            if T.lanes_supported(lanes, precision):
                groups = 64 // lanes
                for rm in sorted({max(1, groups // 8), max(1, groups // 4), max(1, groups // 2), groups}):
                    out.append((lanes, rm))
        return out

    def measure(self, T, precision: int, n_sets: int = 4000, n_ic: int = 10, seed: int = 1,
                reps: int = 2, opts: rp.Opts | None = None) -> list[Choice]:
        """Time every candidate on a sample of n_sets x n_ic trajectories:
        HIP events on the launch stream around each solve, best of `reps`
        after one untimed run."""
        import torch
        params = rp.sample_params(T, seed, n_sets, n_ic).to_device()
        base = opts or rp.Opts(precision=precision)
        stream = torch.cuda.current_stream()
        res = []
        out = None
        for lanes, rm in self.candidates(T, precision):
            o = rp.Opts(**{**base.__dict__, "precision": precision, "lanes_per_traj": lanes,
                           "refill_min": rm})
            out = rp.steady_states(T, params, o, out=out, stream=stream)
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rp.steady_states(T, params, o, out=out, stream=stream)
                e1.record(stream)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e-3)
            res.append(Choice(lanes, rm, n_sets * n_ic / best))
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
