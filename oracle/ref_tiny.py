"""Second, independent implementation of the annealing schedule in pure Python.

TEST INFRASTRUCTURE ONLY (see the package docstring). Written separately from
``gdi_oracle.c`` and meant for tiny graphs (n up to a few hundred, a few sweeps):
its only purpose is to cross-check the C oracle.

It follows the same reading of the paper (Sec. V Alg. 3, eq. 5-6): colour
classes by first-fit greedy colouring in ascending id, one phase per class in
ascending colour, the magnetisation read once per phase, GATED or SNAPSHOT
balance, Metropolis acceptance against floor(2^32 exp(-dE/T)), Philox4x32-10
words keyed by the seed. Within a phase every decision reads the pre-phase
spins; ``visit_seed`` shuffles the visiting order inside each class, which
must not change the result.
"""
from __future__ import annotations

import math
import random

MASK = 0xFFFFFFFF


def philox4x32_10(key: int, ctr: tuple) -> tuple:
    """Philox4x32-10 (Salmon et al., SC'11) with Python integers."""
    key = int(key)
    k0, k1 = key & MASK, (key >> 32) & MASK
    x = [int(v) for v in ctr]
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & MASK
            k1 = (k1 + 0xBB67AE85) & MASK
        a = 0xD2511F53 * x[0]
        b = 0xCD9E8D57 * x[2]
        x = [((b >> 32) ^ x[1] ^ k0) & MASK, b & MASK, ((a >> 32) ^ x[3] ^ k1) & MASK, a & MASK]
    return tuple(x)


def threshold(d: int, T: float) -> int:
    v = math.floor(math.ldexp(math.exp(-d / T), 32))
    return min(v, MASK)


def colouring(n, adj):
    colour = [0] * n
    for i in range(n):
        used = {colour[j] for j in adj[i] if j < i}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def flip_threshold(pf: float) -> int:
    """min(2^32 - 1, floor(2^32 P_f)) for the paper's random flips."""
    return min(math.floor(math.ldexp(pf, 32)), MASK)


def anneal(n, edges, temps, seed, A=1, B=1, replica=0, gated=True, init=None, start_sweep=0,
           visit_seed=None, skip=(), last_flip=None, paper_rule=False):
    """edges: list of (i, j, w) with i != j, each undirected edge once. Returns (spins, M, cut).

    Nodes in ``skip`` make no decision (their spins stay, they still count in the
    magnetisation); ``last_flip`` (a list of n ints) receives each flip's sweep. With
    ``paper_rule`` temps are flip probabilities: a spin takes its energy-minimising
    value (flips iff dE < 0; when dE = 0 its value is random, +1 iff Philox word x2 is
    odd) and then flips again when x0 < floor(2^32 P_f).
    """
    skip = set(skip)
    adj = [[] for _ in range(n)]
    for i, j, w in edges:
        adj[i].append((j, w))
        adj[j].append((i, w))
    nbrs = [[j for j, _ in adj[i]] for i in range(n)]
    colour = colouring(n, nbrs)
    C = max(colour) + 1
    classes = [[i for i in range(n) if colour[i] == c] for c in range(C)]
    if visit_seed is not None:
        rnd = random.Random(visit_seed)
        for cl in classes:
            rnd.shuffle(cl)
    if init is None:
        s = [1 if philox4x32_10(seed, (i, 0, replica, 1))[0] & 1 else -1 for i in range(n)]
    else:
        s = [1 if v > 0 else -1 for v in init]
    for t in range(start_sweep, len(temps)):
        T = temps[t]
        for c in range(C):
            M0 = sum(s)
            sg = (M0 > 0) - (M0 < 0)
            D = abs(M0) // 2
            over = sum(1 for i in classes[c] if s[i] == sg) if sg != 0 else 0
            flips = []
            for i in classes[c]:
                if i in skip:
                    continue
                x = philox4x32_10(seed, (i, t, replica, 0))
                h = sum(w * s[j] for j, w in adj[i])
                if gated:
                    seen = M0 if (s[i] == sg and x[1] * over < (D << 32)) else 0
                else:
                    seen = M0
                dE = B * s[i] * h + 4 * A * (1 - s[i] * seen)
                if paper_rule:
                    if dE < 0:
                        argmin = -s[i]
                    elif dE > 0:
                        argmin = s[i]
                    else:
                        argmin = 1 if x[2] & 1 else -1
                    if (argmin != s[i]) != (x[0] < flip_threshold(T)):
                        flips.append(i)
                elif dE <= 0 or x[0] < threshold(dE, T):
                    flips.append(i)
            for i in flips:
                s[i] = -s[i]
                if last_flip is not None:
                    last_flip[i] = t
    M = sum(s)
    cut = sum(w for i, j, w in edges if s[i] != s[j])
    return s, M, cut
