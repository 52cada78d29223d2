"""Oracle for the Boolean Ising formalism (test infrastructure only).

Plain numpy and Python loops, written from Sec. 2.2 (Eq. 3): gene i's next
state is on if the signed sum of its regulators' states is positive, off if
negative, unchanged if zero, with J[i][j] = +1 for an activating edge j -> i,
-1 for an inhibiting one and 0 otherwise.  An off gene counts as `low` in the
sums (0 or -1, the paper's flip values).

Synchronous mode updates every gene at once; a trajectory stops at the first
state that maps to itself, or after max_steps updates.  Asynchronous mode
updates one gene per step, chosen uniformly at random or cycled from a given
order; every `check_every` updates (and at the start) the state is tested
for being a fixed point of the synchronous map, and the trajectory stops at
the first such test that passes.

Random choices use Philox4x64-10 (the oracle's own implementation), so the
device and this module make the same choices:
- update u of trajectory t picks gene (h * N) >> 32, where h is the low (u
  even) or high (u odd) 32-bit half of word (u % 8) // 2 of the block at
  counter (t, u // 8, 8, 0), key (seed, 0);
- a random initial state has gene i on when the uniform draw at counter
  (t, i // 4, 9, 0), word i % 4 (top 53 bits over 2^53) is >= 1/2.

States are bit-packed: bit i of word i // 64 is gene i.  Only tests/, the
smoke test and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np

import oracle

FIXED_POINT, MAX_STEPS = 0, 1
_M64 = (1 << 64) - 1


def coupling(n_genes: int, src, dst, sign) -> np.ndarray:
    J = np.zeros((n_genes, n_genes), np.int64)
    for s, d, g in zip(src, dst, sign):
        J[d, s] = 1 if g > 0 else -1
    return J


def _block(seed: int, ctr):
    return oracle.philox4x64_10(ctr, (seed & _M64, 0))


def random_state(seed: int, t: int, n_genes: int) -> np.ndarray:
    on = np.zeros(n_genes, bool)
    for i in range(n_genes):
        w = int(_block(seed, (t, i // 4, 9, 0))[i % 4])
        on[i] = (w >> 11) * 2.0**-53 >= 0.5
    return on


def random_gene(seed: int, t: int, u: int, n_genes: int) -> int:
    w = int(_block(seed, (t, u // 8, 8, 0))[(u % 8) // 2])
    h = (w & 0xFFFFFFFF) if u % 2 == 0 else (w >> 32)
    return (h * n_genes) >> 32


def sync_map(J, on, low):
    s = np.where(on, 1, low)
    h = J @ s
    return np.where(h > 0, True, np.where(h < 0, False, on))


def run(J, init_on, mode: str, low: int = 0, max_steps: int = 1000, seed: int = 0,
        order=None, check_every: int = 0, record: bool = False, traj: int = 0):
    """One trajectory from init_on (bool[N]).  Returns (final bool[N], steps,
    status, record list of states after each update when asked)."""
    N = J.shape[0]
    on = np.array(init_on, bool)
    rec = [on.copy()] if record else None
    if mode == "sync":
        for step in range(max_steps + 1):
            nxt = sync_map(J, on, low)
            if np.array_equal(nxt, on):
                return on, step, FIXED_POINT, rec
            if step == max_steps:
                break
            on = nxt
            if record:
                rec.append(on.copy())
        return on, max_steps, MAX_STEPS, rec
    every = check_every if check_every > 0 else N
    for u in range(max_steps + 1):
        if u % every == 0 and np.array_equal(sync_map(J, on, low), on):
            return on, u, FIXED_POINT, rec
        if u == max_steps:
            break
        i = order[u % len(order)] if order is not None else random_gene(seed, traj, u, N)
        s = np.where(on, 1, low)
        h = int(J[i] @ s)
        if h > 0:
            on[i] = True
        elif h < 0:
            on[i] = False
        if record:
            rec.append(on.copy())
    return on, max_steps, MAX_STEPS, rec


def pack(on) -> np.ndarray:
    on = np.asarray(on, bool)
    W = (on.shape[-1] + 63) // 64
    out = np.zeros(on.shape[:-1] + (W,), np.uint64)
    for i in range(on.shape[-1]):
        out[..., i // 64] |= (on[..., i].astype(np.uint64) << np.uint64(i % 64))
    return out


def unpack(words, n_genes: int) -> np.ndarray:
    words = np.asarray(words, np.uint64)
    on = np.zeros(words.shape[:-1] + (n_genes,), bool)
    for i in range(n_genes):
        on[..., i] = (words[..., i // 64] >> np.uint64(i % 64)) & np.uint64(1)
    return on


def simulate(n_genes, src, dst, sign, n_traj, mode, low=0, max_steps=1000, seed=0, init=None,
             order=None, check_every=0):
    """All trajectories; init bool[n_traj][N] or None for random states.
    Returns (final bool[n_traj][N], steps int32, status int8)."""
    J = coupling(n_genes, src, dst, sign)
    fin = np.zeros((n_traj, n_genes), bool)
    steps = np.zeros(n_traj, np.int32)
    status = np.zeros(n_traj, np.int8)
    for t in range(n_traj):
        s0 = init[t] if init is not None else random_state(seed, t, n_genes)
        f, st, ss, _ = run(J, s0, mode, low, max_steps, seed, order, check_every, traj=t)
        fin[t], steps[t], status[t] = f, st, ss
    return fin, steps, status
