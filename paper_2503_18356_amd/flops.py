"""Algorithmic work and traffic per solve, used by every report.

FLOPs (FP32, credited from the GPU's own step counts):
  per right-hand side   F_rhs = sum_e (6 + c(n_e)) + 3N
      6 per edge: x/T scaling 1, 1 + r 1, reciprocal 1, two for the affine
      Hill factor, 1 for the product; c(n) = length of the shortest
      multiplication chain for q^n ({0,1,2,2,3,3} for n = 1..6); 3N for
      G*P - k*x.
  per attempted step    F_step = 6 F_rhs + 56N  (20 stage and 6 error
      multiply-adds = 52, plus 4 for the error scale and ratio, per gene).
  per solve             (accepted + rejected steps) * F_step.
Bytes (HBM, per launch): parameters (2N + 2E) * 4 + E per set, initial
conditions N * 4 per IC, outputs N * prec + 17 per trajectory.
"""
from __future__ import annotations

import numpy as np

CHAIN = np.array([0, 0, 1, 2, 2, 3, 3, 4, 3, 4, 4, 5, 4], dtype=np.int64)  # index n


def rhs_flops_per_set(n_genes: int, n: np.ndarray) -> np.ndarray:
    """F_rhs for every parameter set; n is [E][P] (u8)."""
    n = np.asarray(n)
    if n.size == 0:
        P = n.shape[1] if n.ndim == 2 else 0
        return np.full(P, 3 * n_genes, dtype=np.int64)
    return (6 + CHAIN[n.astype(np.int64)]).sum(axis=0) + 3 * n_genes


def step_flops_per_set(n_genes: int, n: np.ndarray) -> np.ndarray:
    return 6 * rhs_flops_per_set(n_genes, n) + 56 * n_genes


def credited(n_genes: int, n: np.ndarray, n_ic: int, steps_per_traj: np.ndarray) -> float:
    """Total credited FLOPs; steps_per_traj = accepted + rejected, per trajectory
    in id order p * n_ic + c."""
    fs = step_flops_per_set(n_genes, n)
    steps = np.asarray(steps_per_traj, dtype=np.int64).reshape(-1, n_ic).sum(axis=1)
    return float((fs * steps).sum())


def algorithmic_bytes(n_genes: int, n_edges: int, n_sets: int, n_ic: int, x_bytes: int,
                      n_t: int = 0) -> float:
    per_set = (2 * n_genes + 2 * n_edges) * 4 + n_edges
    per_traj = n_genes * x_bytes * (n_t if n_t else 1) + 8 + 1 + 4 + 4
    return float(per_set * n_sets + n_genes * 4 * n_ic + per_traj * n_sets * n_ic)


def postproc_bytes(n_genes: int, n_sets: int, n_ic: int, n_bins: int = 64,
                   capacity: int = 1 << 16) -> int:
    """Algorithmic HBM bytes of the device post-processing chain on a
    steady-state result of n_sets * n_ic rows: normalise (read x, G and k per
    set, write y), histogram (read y and status), levels and codes (read y
    and status, write one byte per level and eight per code), multistability
    (read codes, write the per-set state lists and counts), state counts
    (read codes; write and read the hash table and the sorted output)."""
    rows = n_sets * n_ic
    el = rows * n_genes
    normalise = el * 4 * 2 + n_sets * n_genes * 8
    hist = el * 4 + rows + n_bins * 8
    disc = el * 4 + rows + el + rows * 8
    multi = rows * 8 * 2 + n_sets * 4
    counts = rows * 8 + capacity * 16 * 3
    return int(normalise + hist + disc + multi + counts)
