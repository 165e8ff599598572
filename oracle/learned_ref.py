"""CPU reference of the learned frozen-node proposal -- TEST INFRASTRUCTURE ONLY.

The proposal is not part of the paper: it is this library's extension of the
annealing schedule (Sec. V, Alg. 3), defined by the learned-proposal section of
``include/gdi.h``. A full sweep runs every ``k_full`` sweeps; after it, a proposal
marks nodes to skip in the next ``k_full - 1`` sweeps, where a skipped node makes
no decision (keeps its spin, draws nothing) but still counts in the magnetisation
and its class's over-side count. Everything else is the plain schedule, so the
sweeps themselves run through the C oracle (``oracle.anneal`` with ``skip``).

Proposals:
  * none       -- no node is skipped (the plain schedule);
  * heuristic  -- skip nodes whose last flip is at least ``k`` sweeps old;
  * network    -- skip nodes whose logit exceeds logit(p) for a 6 -> 64 -> 64 -> 1
                  ReLU network on six per-node features.

Precision. Features and the network's decision (an integer: skip or not) are
taken in the precision the kernels use -- features in FP32 rounded to BF16,
weights W1, W2 in BF16, hidden activations H1 in BF16, FP32 accumulation --
following the kernels' order of FP32 operations (see ``mlp_logits_f32``). The
loss and gradient reference (``mlp_loss_grad``) is FP64 with optional BF16
rounding at the same storage points; with rounding off it is pinned by finite
differences.

Weights travel as one flat array in the order w1[64][6], b1[64], w2[64][64],
b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

from . import anneal as oracle_anneal

MLP_PARAMS = 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1


def unflatten(w) -> dict:
    w = np.asarray(w, dtype=np.float64)
    o, d = 0, {}
    for name, shape in (("w1", (64, 6)), ("b1", (64,)), ("w2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", ())):
        k = int(np.prod(shape)) if shape else 1
        d[name] = w[o:o + k].reshape(shape) if shape else float(w[o])
        o += k
    return d


def flatten(d) -> np.ndarray:
    return np.concatenate([np.ravel(d["w1"]), d["b1"], np.ravel(d["w2"]), d["b2"], d["w3"], [d["b3"]]])


def bf16(x) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value, ties to even (returned as FP32)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(f.shape)


def bf16_bits(x) -> np.ndarray:
    """Upper 16 bits of BF16-valued FP32 numbers (the BF16 encoding)."""
    return (np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32) >> 16).astype(np.uint16)


# ---------------------------------------------------------------- features
def features(g, spins, last_flip, t: int, T: float, A: int, B: int, M: int) -> np.ndarray:
    """Six per-node features after sweep t, original order, FP32 rounded to BF16 (n x 6).

    f0 = degree / 16; f1 = sum |w| / 16; f2 = fraction of neighbours with the
    other spin (0 without neighbours); f3 = clamp(B s h / T, -16, 16) / 4 with
    h = sum_j w_ij s_j (positive = the cut term opposes a flip); f4 = min(|4A(1 - s
    M)| / T, 64) / 16 (the balance term of eq. 6 in units of T); f5 = min(t -
    last_flip, 255) / 64 (sweeps since the node's last flip). T is taken in FP32.
    """
    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    w = np.asarray(g.w, dtype=np.int64)
    s = np.asarray(spins, dtype=np.int64)
    deg = np.diff(rp)
    rows = np.repeat(np.arange(n), deg)
    h = np.bincount(rows, weights=(w * s[col]).astype(np.float64), minlength=n).astype(np.int64)
    wabs = np.bincount(rows, weights=np.abs(w).astype(np.float64), minlength=n).astype(np.int64)
    other = np.bincount(rows, weights=(s[col] != s[rows]).astype(np.float64), minlength=n).astype(np.int64)
    T32 = np.float32(T)
    f = np.zeros((n, 6), dtype=np.float32)
    f[:, 0] = deg.astype(np.float32) / np.float32(16)
    f[:, 1] = wabs.astype(np.float32) / np.float32(16)
    with np.errstate(invalid="ignore", divide="ignore"):
        frac = other.astype(np.float32) / deg.astype(np.float32)
    f[:, 2] = np.where(deg > 0, frac, np.float32(0))
    loc = (B * s * h).astype(np.float32) / T32
    f[:, 3] = np.minimum(np.maximum(loc, np.float32(-16)), np.float32(16)) / np.float32(4)
    bal = np.abs(4 * A * (1 - s * M)).astype(np.float32) / T32
    f[:, 4] = np.minimum(bal, np.float32(64)) / np.float32(16)
    age = np.minimum(t - np.asarray(last_flip, dtype=np.int64), 255).astype(np.float32)
    f[:, 5] = age / np.float32(64)
    return bf16(f)


def heuristic_skip(last_flip, t: int, k: int) -> np.ndarray:
    """Nodes whose last flip is at least k sweeps before sweep t."""
    return (t - np.asarray(last_flip, dtype=np.int64)) >= k


# ---------------------------------------------------------------- network, kernel precision
def _fma32(a, b, c):
    """FP32 fused multiply-add: a*b is exact in FP64, one rounding of the sum to FP32."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def mlp_logits_f32(w, X) -> np.ndarray:
    """Logits in the kernels' precision and FP32 operation order.

    Layer 1: BF16 products summed exactly, rounded once to FP32, + b1 in FP32,
    ReLU, rounded to BF16. Layer 2: four 16-input partial sums (exact), each added
    to the FP32 accumulator with one rounding, + b2, ReLU. Output: for each of the
    four row groups g, a running FP32 fused multiply-add over hidden units 16m + 4g
    + i (m outer, i inner), then (p0 + p1) + (p2 + p3) + b3.
    """
    P = unflatten(w)
    Xb = bf16(np.asarray(X, dtype=np.float32)[:, :6]).astype(np.float64)
    W1 = bf16(P["w1"].astype(np.float32)).astype(np.float64)
    W2 = bf16(P["w2"].astype(np.float32)).astype(np.float64)
    b1 = P["b1"].astype(np.float32)
    b2 = P["b2"].astype(np.float32)
    w3 = P["w3"].astype(np.float32)
    b3 = np.float32(P["b3"])
    pre1 = (Xb @ W1.T).astype(np.float32) + b1
    h1 = bf16(np.maximum(pre1, np.float32(0))).astype(np.float64)
    acc = np.zeros((Xb.shape[0], 64), dtype=np.float32)
    for kb in range(4):
        part = h1[:, 16 * kb:16 * kb + 16] @ W2[:, 16 * kb:16 * kb + 16].T
        acc = (acc.astype(np.float64) + part).astype(np.float32)
    h2 = np.maximum(acc + b2, np.float32(0))
    parts = []
    for g in range(4):
        p = np.zeros(Xb.shape[0], dtype=np.float32)
        for m in range(4):
            for i in range(4):
                u = 16 * m + 4 * g + i
                p = _fma32(np.full_like(p, w3[u]), h2[:, u], p)
        parts.append(p)
    return ((parts[0] + parts[1]) + (parts[2] + parts[3])) + b3


def threshold_logit(p: float) -> np.float32:
    """logit(p) in FP32: log(p / (1 - p)) with p, 1 - p and the quotient in FP32."""
    p32 = np.float32(p)
    return np.float32(np.log(p32 / (np.float32(1) - p32)))


# ---------------------------------------------------------------- network, FP64 reference
def _forward64(P, X, round_points):
    r = (lambda a: bf16(a.astype(np.float32)).astype(np.float64)) if round_points else (lambda a: a)
    x = r(np.asarray(X, dtype=np.float64)[:, :6])
    W1, W2 = r(P["w1"]), r(P["w2"])
    pre1 = x @ W1.T + P["b1"]
    h1 = r(np.maximum(pre1, 0.0))
    pre2 = h1 @ W2.T + P["b2"]
    h2 = np.maximum(pre2, 0.0)
    z = h2 @ P["w3"] + P["b3"]
    return r, x, W1, W2, h1, pre2, h2, z


def mlp_logits(w, X, round_points: bool = True) -> np.ndarray:
    """Logits z = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 in FP64 (BF16 storage points optional)."""
    return _forward64(unflatten(w), X, round_points)[-1]


def mlp_loss_grad(w, X, y, round_points: bool = True):
    """Mean logistic loss of the network on rows X (n x 6) with labels y, and its
    gradient with respect to the flat parameters, in FP64.

    z = w3 . relu(W2 h1 + b2) + b3, h1 = relu(W1 x + b1); loss = mean(softplus(z)
    - y z). With round_points, x, W1, W2 and h1 are rounded to BF16 as stored by
    the kernels, and the back-propagated dPre2 (for dH1 and dW2) and dPre1 (for
    dW1) are rounded to BF16 where the kernels round them.
    """
    P = unflatten(w)
    y = np.asarray(y, dtype=np.float64)
    r, x, W1, W2, h1, pre2, h2, z = _forward64(P, X, round_points)
    n = x.shape[0]
    loss = np.mean(np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z))) - y * z)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g = {"b3": dz.sum(), "w3": h2.T @ dz}
    dpre2 = np.where(pre2 > 0, dz[:, None] * P["w3"][None, :], 0.0)
    g["b2"] = dpre2.sum(axis=0)
    dp2 = r(dpre2)
    g["w2"] = dp2.T @ h1
    dh1 = dp2 @ W2
    dpre1 = np.where(h1 > 0, dh1, 0.0)
    g["b1"] = dpre1.sum(axis=0)
    g["w1"] = r(dpre1).T @ x
    return float(loss), flatten(g)


# ---------------------------------------------------------------- the learned schedule
def learned_anneal(g, temps, seed: int, k_full: int, proposal: str = "none", weights=None, p: float = 0.5,
                   heuristic_k: int = 1, A: int = 1, B: int = 1, replica: int = 0, mode: int = 0,
                   start_sweep: int = 0, init=None, n_threads: int = 0, learn_from: int = 0) -> dict:
    """The annealing schedule: sweeps start_sweep .. b0-1 plain (b0 = max(start_sweep,
    learn_from)), then a full sweep at b0, b0 + k_full, ... and the proposal's skip set
    applied to the sweeps in between.

    Returns spins, M, cut, masks (one row per full sweep, original order; a full
    sweep with no masked sweeps after it has an all-zero row) and, for the network
    proposal, logits (one row per full sweep with masked sweeps after it) and margins =
    min |logit - logit(p)| per row.
    """
    T = np.ascontiguousarray(temps, dtype=np.float64)
    S = T.size
    n = g.n
    lf = np.full(n, start_sweep - 1, dtype=np.int32)
    spins = None if init is None else np.asarray(init, dtype=np.int8)
    b0 = min(S, max(start_sweep, learn_from))
    rows = (S - b0 + k_full - 1) // k_full
    masks = np.zeros((rows, n), dtype=np.uint8)
    margins, logits = [], []
    kw = dict(A=A, B=B, replica=replica, mode=mode, n_threads=n_threads)
    M = None
    res = None
    thr = threshold_logit(p) if proposal == "network" else None
    if b0 > start_sweep:
        res = oracle_anneal(g, T[:b0], seed, start_sweep=start_sweep, init=spins, last_flip=lf, **kw)
        spins = res["spins"]
    for row, b in enumerate(range(b0, S, k_full)):
        res = oracle_anneal(g, T[:b + 1], seed, start_sweep=b, init=spins, last_flip=lf, **kw)
        spins, M = res["spins"], res["M"]
        if b + 1 >= S:
            break
        end = min(b + k_full, S)
        if proposal == "none":
            skip = np.zeros(n, dtype=bool)
        elif proposal == "heuristic":
            skip = heuristic_skip(lf, b, heuristic_k)
        elif proposal == "network":
            z = mlp_logits_f32(weights, features(g, spins, lf, b, T[b], A, B, M))
            skip = z > thr
            logits.append(z)
            margins.append(float(np.min(np.abs(z.astype(np.float64) - np.float64(thr)))))
        else:
            raise ValueError(proposal)
        masks[row] = skip
        res = oracle_anneal(g, T[:end], seed, start_sweep=b + 1, init=spins, skip=skip, last_flip=lf, **kw)
        spins, M = res["spins"], res["M"]
    if res is None:  # start_sweep == S: nothing runs
        res = oracle_anneal(g, T, seed, start_sweep=S, init=init, **kw)
        spins = res["spins"]
    return dict(spins=spins, M=res["M"], cut=res["cut"], masks=masks, margins=margins, logits=logits,
                threshold=thr, last_flip=lf)


def trace_dataset(g, temps, seed: int, every: int, k_label: int, max_snapshots: int, A: int = 1, B: int = 1,
                  replica: int = 0, mode: int = 0):
    """Training rows of a plain anneal: after sweeps t_s = every-1, 2 every-1, ... with
    t_s + k_label < S, the features of every node and the label 1 if it does not flip in
    sweeps t_s+1 .. t_s+k_label. Returns (X: rows x 6 BF16-valued FP32, y: uint8)."""
    T = np.ascontiguousarray(temps, dtype=np.float64)
    S = T.size
    lf = np.full(g.n, -1, dtype=np.int32)
    spins, t_cur = None, 0
    Xs, ys = [], []
    ts = every - 1
    while ts + k_label < S and len(Xs) < max_snapshots:
        r = oracle_anneal(g, T[:ts + 1], seed, start_sweep=t_cur, init=spins, last_flip=lf, A=A, B=B,
                          replica=replica, mode=mode)
        spins = r["spins"]
        Xs.append(features(g, spins, lf, ts, T[ts], A, B, r["M"]))
        r = oracle_anneal(g, T[:ts + k_label + 1], seed, start_sweep=ts + 1, init=spins, last_flip=lf, A=A, B=B,
                          replica=replica, mode=mode)
        spins = r["spins"]
        ys.append((lf <= ts).astype(np.uint8))
        t_cur = ts + k_label + 1
        ts += every
    if not Xs:
        return np.zeros((0, 6), np.float32), np.zeros(0, np.uint8)
    return np.concatenate(Xs), np.concatenate(ys)
