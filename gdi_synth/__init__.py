"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds graph generators and the temperature schedule only. It contains
none of the annealer's arithmetic (no colouring, no random numbers the annealer
draws, no energies): both the CPU oracle and the HIP library receive exactly the
arrays produced here.

Every graph is returned as a symmetric CSR with int32 row pointers, int32 column
indices sorted within each row, and int32 edge weights; there are no self-loops
and no duplicate edges. Each undirected edge appears twice (once per endpoint)
with the same weight, so nnz = 2|E|.

The workload shapes follow the paper's benchmark graphs (Sec. VI, Table I: n from
1,000 to 20,000, mean degree 2 to 20) and the configurations this project
measures: an Erdos-Renyi graph (n=800, p=0.06), a 100x100 torus with +-1 weights,
a random geometric graph with mean degree 8, and mixes of these.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph",
    "er_graph",
    "torus_graph",
    "rgg_graph",
    "rgg_radius",
    "from_edges",
    "geometric_temps",
    "batch_mix",
    "training_graphs",
    "workload",
    "WORKLOADS",
]


@dataclass
class Graph:
    """Symmetric CSR graph (int32 arrays, rows sorted, no self-loops)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def from_edges(n: int, a: np.ndarray, b: np.ndarray, w: np.ndarray, name: str = "") -> Graph:
    """Builds the symmetric CSR from a list of undirected edges (a[k], b[k], w[k]), a != b."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    if a.size and (np.any(a == b) or a.min() < 0 or b.min() < 0 or max(a.max(), b.max()) >= n):
        raise ValueError("edge list has a self-loop or an out-of-range endpoint")
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    if src.size > 1:
        dup = (src[1:] == src[:-1]) & (dst[1:] == dst[:-1])
        if np.any(dup):
            raise ValueError("edge list has duplicate edges")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Graph(
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col=dst.astype(np.int32),
        w=ww.astype(np.int32),
        name=name,
    )


def _weights(rng: np.random.Generator, m: int, kind: str) -> np.ndarray:
    if kind == "unit":
        return np.ones(m, dtype=np.int64)
    if kind == "pm1":
        return rng.integers(0, 2, size=m, dtype=np.int64) * 2 - 1
    raise ValueError(f"unknown weight kind {kind!r}")


def er_graph(n: int, p: float, seed: int, weights: str = "unit") -> Graph:
    """Erdos-Renyi G(n, p): every pair i<j is an edge independently with probability p.

    Pairs are enumerated row-major over the upper triangle; the kept pair indices are
    drawn by geometric skipping (gap-1 ~ Geometric(p)), which has the same law as one
    Bernoulli(p) trial per pair and needs memory proportional to the edge count only.
    """
    rng = np.random.default_rng(seed)
    n_pairs = n * (n - 1) // 2
    kept = []
    pos = -1
    if p > 0:
        while True:
            need = int(max(1024, 1.2 * p * (n_pairs - pos) + 64))
            gaps = rng.geometric(p, size=need)
            idx = pos + np.cumsum(gaps)
            inside = idx < n_pairs
            kept.append(idx[inside])
            if not np.all(inside):
                break
            pos = int(idx[-1])
    lin = np.concatenate(kept) if kept else np.zeros(0, dtype=np.int64)
    # row i of the upper triangle starts at off[i] = i*(2n-i-1)/2
    i_all = np.arange(n, dtype=np.int64)
    off = i_all * (2 * n - i_all - 1) // 2
    a = np.searchsorted(off, lin, side="right") - 1
    b = lin - off[a] + a + 1
    w = _weights(rng, lin.size, weights)
    return from_edges(n, a, b, w, name=f"er_n{n}_p{p:g}_s{seed}")


def torus_graph(L: int, seed: int, weights: str = "pm1") -> Graph:
    """L x L toroidal grid (4-regular): node id = L*r + c, edges to (r, c+1) and (r+1, c) mod L."""
    if L < 3:
        raise ValueError("torus side must be >= 3 (smaller sides create duplicate edges)")
    rng = np.random.default_rng(seed)
    ids = np.arange(L * L, dtype=np.int64).reshape(L, L)
    a = np.concatenate([ids.ravel(), ids.ravel()])
    b = np.concatenate([np.roll(ids, -1, axis=1).ravel(), np.roll(ids, -1, axis=0).ravel()])
    w = _weights(rng, a.size, weights)
    return from_edges(L * L, a, b, w, name=f"torus_{L}x{L}_s{seed}")


def rgg_radius(n: int, mean_degree: float) -> float:
    """Radius r with expected degree (n-1)(pi r^2 - 8 r^3/3 + r^4/2) = mean_degree.

    The left side is (n-1) times the probability that two uniform points of the unit
    square lie within distance r (valid for r <= 1), which accounts for the border.
    Solved by bisection in double precision.
    """
    target = mean_degree / (n - 1)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = math.pi * mid * mid - 8.0 * mid ** 3 / 3.0 + mid ** 4 / 2.0
        if f < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def rgg_graph(n: int, mean_degree: float, seed: int, weights: str = "unit") -> Graph:
    """Random geometric graph: n uniform points in [0,1)^2, edge iff distance <= r.

    Node ids are assigned in cell-major order (cells of side r, rows of cells
    bottom to top, cells left to right, then by x inside a cell), so that nearby
    ids are nearby points.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = rgg_radius(n, mean_degree)
    ncell = max(1, int(1.0 / r))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((pts[:, 0], cx, cy))
    pts = pts[order]
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    w = _weights(rng, pairs.shape[0], weights)
    return from_edges(n, pairs[:, 0], pairs[:, 1], w, name=f"rgg_n{n}_d{mean_degree:g}_s{seed}")


def geometric_temps(t_start: float, t_end: float, n_sweeps: int) -> np.ndarray:
    """Geometric cooling T_t = T0 * (T1/T0)^(t/(S-1)), t = 0..S-1, both ends included (FP64)."""
    if n_sweeps == 1:
        return np.array([t_start], dtype=np.float64)
    t = np.arange(n_sweeps, dtype=np.float64)
    return (t_start * (t_end / t_start) ** (t / (n_sweeps - 1))).astype(np.float64)


def batch_mix(n_graphs: int = 64, seed: int = 300, n_lo: int = 800, n_hi: int = 20000,
              d_lo: float = 4.0, d_hi: float = 48.0) -> list:
    """Uneven graphs for the batched launch: n ~ U_int[n_lo, n_hi], mean degree ~ U[d_lo, d_hi].

    Even indices are Erdos-Renyi (p = d/(n-1)), odd indices are random geometric
    graphs (planar-like). Weights: index mod 4 < 2 -> unit, else +-1.
    """
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n_graphs):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = float(rng.uniform(d_lo, d_hi))
        kind = "unit" if g % 4 < 2 else "pm1"
        gseed = seed * 1000 + g
        if g % 2 == 0:
            out.append(er_graph(n, d / (n - 1), gseed, weights=kind))
        else:
            out.append(rgg_graph(n, d, gseed, weights=kind))
    return out


def training_graphs(n_graphs: int = 8, seed0: int = 200, n_lo: int = 10_000, n_hi: int = 100_000,
                    mean_degree: float = 8.0) -> list:
    """Training graphs for the learned proposal: random geometric graphs of mean degree 8,
    unit weights, n log-uniform in [n_lo, n_hi], graph seeds seed0 .. seed0 + n_graphs - 1."""
    out = []
    for k in range(n_graphs):
        rng = np.random.default_rng(seed0 + k)
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        out.append(rgg_graph(n, mean_degree, seed0 + k, "unit"))
    return out


# Named workloads: graph builder, temperature schedule, sweeps, coefficients.
WORKLOADS = {
    # Erdos-Renyi n=800, p=0.06, unit weights; 1000 sweeps, T 2.0 -> 0.05
    "er800": dict(graph=lambda: er_graph(800, 0.06, 101, "unit"), t0=2.0, t1=0.05, sweeps=1000),
    # 100x100 torus, +-1 weights; 2000 sweeps, T 3.0 -> 0.05
    "torus100": dict(graph=lambda: torus_graph(100, 102, "pm1"), t0=3.0, t1=0.05, sweeps=2000),
    # random geometric graph n=1e6, mean degree 8, unit weights; 2000 sweeps, T 3.0 -> 0.05
    "rgg1m": dict(graph=lambda: rgg_graph(1_000_000, 8.0, 104, "unit"), t0=3.0, t1=0.05, sweeps=2000),
    # random geometric graph n=8e6 (working set above the on-package cache), 50 sweeps
    "rgg8m": dict(graph=lambda: rgg_graph(8_000_000, 8.0, 108, "unit"), t0=3.0, t1=0.05, sweeps=50),
    # evaluation graph for the learned proposal: RGG n=2e5, mean degree 8
    "rgg200k": dict(graph=lambda: rgg_graph(200_000, 8.0, 105, "unit"), t0=3.0, t1=0.05, sweeps=2000),
    # one ER n=2000 graph with ~19,990 edges (replicated 256x in the batched workload)
    "er2000": dict(graph=lambda: er_graph(2000, 0.01, 103, "unit"), t0=2.0, t1=0.05, sweeps=1000),
}


def workload(name: str):
    """Returns (graph, temps) for a named workload."""
    spec = WORKLOADS[name]
    g = spec["graph"]()
    return g, geometric_temps(spec["t0"], spec["t1"], spec["sweeps"])
