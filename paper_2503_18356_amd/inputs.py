"""Seeded synthetic network topologies shaped like the GRiNS workloads.

These are inputs to RACIPE, not part of the method: a signed directed edge
list (src, dst, sign) with sign +1 = activation and -1 = inhibition (Sec. 2.1.1).
The module holds none of the method's arithmetic and imports neither the GPU
library nor the oracle, so both sides may take their topologies from here.

Shapes:
  - toggle switch (TS) and TS with self-activation (TSSA), Sec. 3.1;
  - seeded directed Erdos-Renyi G(n, M) networks with a fixed inhibitory share;
  - a 22-gene / 82-edge "dense core" network with the size and sign mix of the
    EMT case study (Sec. 3.2); the EMT topology itself is not reproduced;
  - request streams of random networks with log-uniform sizes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Topology:
    n_genes: int
    src: np.ndarray   # int32
    dst: np.ndarray   # int32
    sign: np.ndarray  # int8, +1 activation / -1 inhibition
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.src.size)

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.dst, minlength=self.n_genes)

    def out_degree(self) -> np.ndarray:
        return np.bincount(self.src, minlength=self.n_genes)


def _topo(n, edges, name):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return Topology(n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32),
                    e[:, 2].astype(np.int8), name)


def toggle_switch() -> Topology:
    """A -| B, B -| A, no self-loops."""
    return _topo(2, [(0, 1, -1), (1, 0, -1)], "TS")


def toggle_switch_self_activation() -> Topology:
    """TS plus A -> A and B -> B."""
    return _topo(2, [(0, 1, -1), (1, 0, -1), (0, 0, 1), (1, 1, 1)], "TSSA")


def cascade(n_genes: int = 2, sign: int = 1) -> Topology:
    """0 -> 1 -> ... -> n-1 with one sign."""
    return _topo(n_genes, [(i, i + 1, sign) for i in range(n_genes - 1)], f"cascade{n_genes}")


def unregulated(n_genes: int = 1) -> Topology:
    return Topology(n_genes, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8),
                    f"free{n_genes}")


def _signs(rng, m, inhib_frac):
    n_inh = int(round(inhib_frac * m))
    s = np.ones(m, np.int8)
    s[rng.permutation(m)[:n_inh]] = -1
    return s


def erdos_renyi(n_genes: int, n_edges: int, seed: int, inhib_frac: float = 0.5,
                self_loops: bool = False, max_tries: int = 10000) -> Topology:
    """Directed G(n, M): M distinct ordered pairs drawn uniformly, redrawn until
    no gene is isolated (when M allows it)."""
    rng = np.random.default_rng(seed)
    cap = n_genes * n_genes if self_loops else n_genes * (n_genes - 1)
    m = min(n_edges, cap)
    pairs = [(s, d) for s in range(n_genes) for d in range(n_genes) if self_loops or s != d]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    need_cover = 2 * m >= n_genes and n_genes > 1
    for _ in range(max_tries):
        pick = pairs[rng.choice(len(pairs), size=m, replace=False)] if m > 0 else pairs[:0]
        touched = np.zeros(n_genes, bool)
        touched[pick[:, 0]] = True
        touched[pick[:, 1]] = True
        if not need_cover or touched.all():
            break
    signs = _signs(rng, m, inhib_frac)
    return Topology(n_genes, pick[:, 0].astype(np.int32), pick[:, 1].astype(np.int32), signs,
                    f"er{n_genes}_{m}")


def dense_core(seed: int, n_genes: int = 22, n_edges: int = 82, n_core: int = 10,
               core_edges: int = 60, n_inhib: int = 49, n_self_inhib: int = 2) -> Topology:
    """A core of densely connected genes (carrying most edges, including a few
    self-inhibitions) and a periphery of input-only, output-only and lightly
    connected genes."""
    rng = np.random.default_rng(seed)
    core = np.arange(n_core)
    periph = np.arange(n_core, n_genes)
    edges = set()
    self_nodes = rng.choice(core, size=n_self_inhib, replace=False)
    for g in self_nodes:
        edges.add((int(g), int(g)))
    core_pairs = [(s, d) for s in core for d in core if s != d]
    order = rng.permutation(len(core_pairs))
    for idx in order:
        if len(edges) >= core_edges:
            break
        edges.add(tuple(int(v) for v in core_pairs[idx]))
    n_per = len(periph)
    n_in = n_per // 3          # input-only genes: edges into the core
    n_out = n_per // 3         # output-only genes: edges from the core
    inputs, outputs, mids = periph[:n_in], periph[n_in:n_in + n_out], periph[n_in + n_out:]
    rest = n_edges - len(edges)
    cand = []
    for g in inputs:
        cand += [(int(g), int(c)) for c in core]
    for g in outputs:
        cand += [(int(c), int(g)) for c in core]
    for g in mids:
        cand += [(int(c), int(g)) for c in core] + [(int(g), int(c)) for c in core]
    cand = [c for c in cand if c not in edges]
    # Every peripheral gene gets at least one edge, then fill at random.
    for g in periph:
        mine = [c for c in cand if g in c and c not in edges]
        if mine and rest > 0:
            edges.add(mine[rng.integers(len(mine))])
            rest -= 1
    cand = [c for c in cand if c not in edges]
    for idx in rng.permutation(len(cand))[:max(rest, 0)]:
        edges.add(cand[idx])
    e = sorted(edges)
    src = np.asarray([a for a, _ in e], np.int32)
    dst = np.asarray([b for _, b in e], np.int32)
    sign = np.ones(len(e), np.int8)
    is_self = src == dst
    sign[is_self] = -1
    others = np.flatnonzero(~is_self)
    sign[rng.permutation(others)[:max(n_inhib - int(is_self.sum()), 0)]] = -1
    return Topology(n_genes, src, dst, sign, f"densecore{n_genes}_{len(e)}")


def uneven_batch(seed: int, n_networks: int = 64, n_min: int = 5, n_max: int = 50,
                 mean_out_degree: float = 2.5) -> list[Topology]:
    """Networks of uneven size: N ~ U{n_min..n_max}, E = round(2.5 N) capped."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_networks):
        n = int(rng.integers(n_min, n_max + 1))
        m = min(int(round(mean_out_degree * n)), n * (n - 1))
        out.append(erdos_renyi(n, m, seed=int(rng.integers(1 << 31)), inhib_frac=0.5))
    return out


def log_uniform_int(rng, lo: float, hi: float) -> int:
    return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))


def serving_request(rng, n_lo: int = 2, n_hi: int = 100, p_lo: int = 100, p_hi: int = 100000,
                    ic_lo: int = 1, ic_hi: int = 10) -> tuple[Topology, int, int]:
    """One request: a random network of log-uniform size, a log-uniform number of
    parameter sets and a uniform number of initial conditions."""
    n = max(n_lo, min(n_hi, log_uniform_int(rng, n_lo, n_hi)))
    m = min(int(round(2.5 * n)), n * (n - 1))
    topo = erdos_renyi(n, m, seed=int(rng.integers(1 << 31)), inhib_frac=0.5)
    p = max(p_lo, min(p_hi, log_uniform_int(rng, p_lo, p_hi)))
    n_ic = int(rng.integers(ic_lo, ic_hi + 1))
    return topo, p, n_ic


# Edge-type codes of the topology text layout: 1 activation, 2 inhibition.
_TOPO_SIGN = {1: 1, 2: -1}


def parse_topo(text: str, name: str = "") -> tuple[Topology, list[str]]:
    """A network from a topology text: one edge per line as whitespace-separated
    "source target type", type 1 = activation and 2 = inhibition (the paper
    takes networks as a topology file, Sec. 2.1.1, without stating its layout;
    this is the layout RACIPE tools commonly use).  A first line whose type
    field is not an integer is a header and is skipped, as are blank lines and
    lines starting with '#'.  Genes are numbered in order of first appearance
    (source before target, line by line); the names come back in that order.
    Raises ValueError on a line without three fields or with another type code.
    Duplicate edges pass through: the library's topology call rejects them."""
    names: dict[str, int] = {}
    edges = []
    first = True
    for ln, raw in enumerate(text.splitlines(), 1):
        line = raw.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if len(parts) != 3:
            raise ValueError(f"line {ln}: expected 'source target type', got {raw!r}")
        try:
            code = int(parts[2])
        except ValueError:
            if first:
                first = False
                continue
            raise ValueError(f"line {ln}: edge type {parts[2]!r} is not an integer") from None
        first = False
        if code not in _TOPO_SIGN:
            raise ValueError(f"line {ln}: edge type {code} (1 = activation, 2 = inhibition)")
        s = names.setdefault(parts[0], len(names))
        d = names.setdefault(parts[1], len(names))
        edges.append((s, d, _TOPO_SIGN[code]))
    if not names:
        raise ValueError("topology text holds no edges")
    return _topo(len(names), edges, name), list(names)


def read_topo(path: str) -> tuple[Topology, list[str]]:
    """parse_topo() on a file; the network is named after the file."""
    import os
    with open(path) as f:
        return parse_topo(f.read(), os.path.splitext(os.path.basename(path))[0])
