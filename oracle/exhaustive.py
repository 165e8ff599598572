"""Brute-force solvers for tiny graphs -- TEST INFRASTRUCTURE ONLY.

* ``all_energies``: E(s) = A M^2 + B cut_w(s) for all 2^n spin states
  (paper Sec. IV, eq. 4 with eq. 5 and eq. 6, weighted cut), n <= 20.
* ``balanced_min_cut``: the minimum weighted cut over all partitions with
  |V1| - |V2| in {0} (n even) or {-1, +1} (n odd) -- the problem statement of
  Sec. IV-A -- by enumerating every such partition.
* ``crossing_edges``: the number of edges whose ends lie in different parts (the
  paper's "cut", Sec. VI), for every row of a state matrix, counted over the
  undirected edge list.
"""
from __future__ import annotations

import numpy as np


def _edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = src < g.col
    return src[keep], g.col[keep].astype(np.int64), g.w[keep].astype(np.int64)


def all_states(n: int) -> np.ndarray:
    """(2^n, n) int8 matrix of spins: bit i of the row index set -> spin +1."""
    idx = np.arange(1 << n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def all_energies(g, A: int, B: int) -> tuple:
    """Returns (states, M, cut_w, E) over all 2^n states."""
    if g.n > 20:
        raise ValueError("exhaustive enumeration is limited to n <= 20")
    S = all_states(g.n).astype(np.int64)
    a, b, w = _edges(g)
    cut = ((S[:, a] != S[:, b]) * w[None, :]).sum(axis=1)
    M = S.sum(axis=1)
    return S, M, cut, A * M * M + B * cut


def balanced_min_cut(g) -> tuple:
    """(min weighted cut, number of optimal balanced partitions counted over spin states)."""
    S, M, cut, _ = all_energies(g, 0, 1)
    target = 1 if g.n % 2 else 0
    ok = np.abs(M) == target
    best = int(cut[ok].min())
    return best, int(np.count_nonzero(ok & (cut == best)))


def crossing_edges(g, states) -> np.ndarray:
    """Crossing-edge count of each state (rows of +-1 spins), over the undirected edge list."""
    S = np.atleast_2d(np.asarray(states, dtype=np.int64))
    a, b, _ = _edges(g)
    return (S[:, a] != S[:, b]).sum(axis=1)
