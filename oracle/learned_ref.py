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

Precision. The network is defined with BF16 storage points: features, W1, W2 and
the first hidden layer H1 hold BF16 values, everything else is exact. ``mlp_logits``
and ``mlp_loss_grad`` evaluate that definition in FP64 (with rounding off, the
gradient is pinned by finite differences and autograd). A device computes the same
definition in FP32; ``mlp_error_model`` bounds how far any FP32 evaluation may land
from the FP64 one: every short dot product (at most 67 terms) by the worst-case
bound gamma_k = k u / (1 - k u), every sum over minibatch rows by the probabilistic
bound lambda sqrt(N) u of Higham and Mary (SIAM J. Sci. Comput. 41(5), 2019) with
lambda = 8, and every BF16 storage point by rounding both ends of the value's
interval (rounding is monotone), so that a value near a BF16 rounding boundary
carries the full width of the two candidates. u is taken as 2^-23 (twice FP32's
unit roundoff), which also covers accumulators that round less carefully than
round-to-nearest. A skip decision is the FP64 one, skip iff z > logit(p); it is
fixed only where |z - logit(p)| exceeds the logit's bound plus the error of an FP32
evaluation of logit(p) -- nodes inside that band may go either way.

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


# ---------------------------------------------------------------- decision threshold
def threshold_logit(p: float) -> float:
    """logit(p) = log(p / (1 - p)) in FP64 for the FP32 value of p (skip iff sigmoid(z) > p)."""
    p64 = float(np.float32(p))
    return float(np.log(p64 / (1.0 - p64)))


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


# ---------------------------------------------------------------- error model of an FP32 evaluation
U_FP32 = 2.0 ** -23   # twice FP32's unit roundoff (see the module docstring)
LAMBDA = 8.0          # probabilistic bound: fails with probability <= 2 exp(-LAMBDA^2 / 2) per sum


def _gamma(k: int) -> float:
    """Worst-case relative error of a k-term FP32 sum or dot product (Higham, Thm. 3.1)."""
    return k * U_FP32 / (1.0 - k * U_FP32)


def _gamma_rows(n: int) -> float:
    """Probabilistic relative error of a sum over n rows (Higham and Mary 2019, Thm. 3.1)."""
    return LAMBDA * np.sqrt(n) * U_FP32 + n * U_FP32 ** 2


def _w32(w) -> dict:
    """The FP32 master weights a device holds, as FP64 values."""
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in unflatten(w).items()}


def _bf16_64(a):
    """Round FP64 values to FP32, then to BF16 (the storage a device applies to an FP32 value)."""
    return bf16(np.asarray(a, dtype=np.float64).astype(np.float32)).astype(np.float64)


def _bf16_spread(v, e):
    """Largest distance between bf16(v) and bf16 of any value within e of v (monotone rounding)."""
    c = _bf16_64(v)
    return np.maximum(_bf16_64(v + e) - c, c - _bf16_64(v - e))


def mlp_error_model(w, X, y=None) -> dict:
    """The FP64 definition of the network on rows X (n x 6) with FP32 master weights w,
    and bounds on how far an FP32 evaluation with the same BF16 storage points may be
    from it.

    Returns z (logits) and z_bound; with labels y also loss, loss_bound, grad (flat,
    gdi_mlp_weights order) and grad_bound (flat, elementwise).
    """
    P = _w32(w)
    x = bf16(np.asarray(X, dtype=np.float32)[:, :6]).astype(np.float64)
    W1, W2 = _bf16_64(P["w1"]), _bf16_64(P["w2"])
    b1, b2, w3, b3 = P["b1"], P["b2"], P["w3"], float(P["b3"])
    n = x.shape[0]
    # layer 1: six exact products and the bias per hidden unit, then ReLU and BF16 storage
    pre1 = x @ W1.T + b1
    e1 = _gamma(8) * (np.abs(x) @ np.abs(W1).T + np.abs(b1))
    h1 = _bf16_64(np.maximum(pre1, 0.0))
    dh1 = _bf16_spread(np.maximum(pre1, 0.0), e1)
    h1_lo = _bf16_64(np.maximum(pre1 - e1, 0.0))
    amb1 = (h1_lo == 0.0) & (_bf16_64(np.maximum(pre1 + e1, 0.0)) > 0.0)  # ReLU gate undecided
    # layer 2: 64 exact BF16 products and the bias, ReLU (1-Lipschitz), kept unrounded
    pre2 = h1 @ W2.T + b2
    e2 = _gamma(66) * ((h1 + dh1) @ np.abs(W2).T + np.abs(b2)) + dh1 @ np.abs(W2).T
    h2 = np.maximum(pre2, 0.0)
    dh2 = e2
    # output: 64 FP32 products and the bias
    z = h2 @ w3 + b3
    ez = _gamma(67) * ((h2 + dh2) @ np.abs(w3) + abs(b3)) + dh2 @ np.abs(w3)
    out = dict(z=z, z_bound=ez)
    if y is None:
        return out
    y = np.asarray(y, dtype=np.float64)
    gN = _gamma_rows(n)
    sig = 1.0 / (1.0 + np.exp(-z))
    sig_lo, sig_hi = 1.0 / (1.0 + np.exp(-(z - ez))), 1.0 / (1.0 + np.exp(-(z + ez)))
    # sigmoid through exp, an addition and a division: eight roundings' worth of slack
    dsig = np.maximum(sig_hi - sig, sig - sig_lo) + 8 * U_FP32 * sig_hi
    dz = (sig - y) / n
    ddz = (dsig + 3 * U_FP32 * (np.abs(sig - y) + dsig)) / n
    # loss: softplus(z) - y z per row, mean over rows
    terms = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z))) - y * z
    dterm = np.abs(sig - y) * ez + ez ** 2 + 8 * U_FP32 * (np.abs(terms) + np.abs(y * z) + np.abs(z))
    out["loss"] = float(np.mean(terms))
    out["loss_bound"] = float((np.sum(dterm) + gN * np.sum(np.abs(terms) + dterm)) / n)
    # backward through the output layer
    gw3 = h2.T @ dz
    gw3_b = (ddz @ (h2 + dh2) + np.abs(dz) @ dh2 + U_FP32 * (np.abs(dz) @ (h2 + dh2))
             + gN * ((np.abs(dz) + ddz) @ (h2 + dh2)))
    gb3 = float(dz.sum())
    gb3_b = float(ddz.sum() + gN * np.sum(np.abs(dz) + ddz))
    amb2 = np.abs(pre2) <= e2  # ReLU gate of layer 2 undecided
    dzw = dz[:, None] * w3[None, :]
    dpre2 = np.where(pre2 > 0, dzw, 0.0)
    ddpre2 = ddz[:, None] * np.abs(w3)[None, :] + U_FP32 * np.abs(dzw)
    ddpre2 = np.where(amb2, ddpre2 + np.abs(dzw), np.where(pre2 > 0, ddpre2, 0.0))
    gb2 = dpre2.sum(axis=0)
    gb2_b = ddpre2.sum(axis=0) + gN * (np.abs(dpre2) + ddpre2).sum(axis=0)
    dp2 = _bf16_64(dpre2)
    ddp2 = _bf16_spread(dpre2, ddpre2)
    gw2 = dp2.T @ h1
    gw2_b = ddp2.T @ (h1 + dh1) + np.abs(dp2).T @ dh1 + gN * ((np.abs(dp2) + ddp2).T @ (h1 + dh1))
    # back into layer 1
    dH1 = dp2 @ W2
    ddH1 = ddp2 @ np.abs(W2) + _gamma(65) * ((np.abs(dp2) + ddp2) @ np.abs(W2))
    dpre1 = np.where(h1 > 0, dH1, 0.0)
    ddpre1 = np.where((h1 > 0) | amb1, ddH1, 0.0) + np.where(amb1, np.abs(dH1), 0.0)
    gb1 = dpre1.sum(axis=0)
    gb1_b = ddpre1.sum(axis=0) + gN * (np.abs(dpre1) + ddpre1).sum(axis=0)
    dp1 = _bf16_64(dpre1)
    ddp1 = _bf16_spread(dpre1, ddpre1)
    gw1 = dp1.T @ x
    gw1_b = ddp1.T @ np.abs(x) + gN * ((np.abs(dp1) + ddp1).T @ np.abs(x))
    out["grad"] = flatten(dict(w1=gw1, b1=gb1, w2=gw2, b2=gb2, w3=gw3, b3=gb3))
    out["grad_bound"] = flatten(dict(w1=gw1_b, b1=gb1_b, w2=gw2_b, b2=gb2_b, w3=gw3_b, b3=gb3_b))
    return out


def skip_decisions(w, X, p: float):
    """FP64 skip decisions (z > logit(p)) and the nodes an FP32 evaluation could decide
    either way: |z - logit(p)| <= z_bound + the error of an FP32 logit(p) (a division,
    a subtraction and a logarithm: 16 units of roundoff, relative, plus as much absolute)."""
    m = mlp_error_model(w, X)
    thr = threshold_logit(p)
    band = m["z_bound"] + 16 * U_FP32 * (1.0 + abs(thr))
    return m["z"] > thr, np.abs(m["z"] - thr) <= band, m["z"], thr


# ---------------------------------------------------------------- the learned schedule
def learned_anneal(g, temps, seed: int, k_full: int, proposal: str = "none", weights=None, p: float = 0.5,
                   heuristic_k: int = 1, A: int = 1, B: int = 1, replica: int = 0, mode: int = 0,
                   start_sweep: int = 0, init=None, n_threads: int = 0, learn_from: int = 0,
                   replay_masks=None) -> dict:
    """The annealing schedule: sweeps start_sweep .. b0-1 plain (b0 = max(start_sweep,
    learn_from)), then a full sweep at b0, b0 + k_full, ... and the proposal's skip set
    applied to the sweeps in between.

    replay_masks (rows x n, original order) replaces the skip set of every row by the
    given one after the proposal has been evaluated on the schedule's own state: the run
    then follows another implementation's masks, and ``proposed`` holds what the
    proposal itself decided at each row, so that both can be compared row by row even
    after the two have taken different values inside the ambiguity band.

    Returns spins, M, cut, masks (one row per full sweep, original order; a full
    sweep with no masked sweeps after it has an all-zero row) and, for the network
    proposal, logits (FP64, one row per full sweep with masked sweeps after it),
    margins = min |logit - logit(p)| per row, and ambiguous (per row, the nodes whose
    decision an FP32 evaluation could take either way, see skip_decisions).
    """
    T = np.ascontiguousarray(temps, dtype=np.float64)
    S = T.size
    n = g.n
    lf = np.full(n, start_sweep - 1, dtype=np.int32)
    spins = None if init is None else np.asarray(init, dtype=np.int8)
    b0 = min(S, max(start_sweep, learn_from))
    rows = (S - b0 + k_full - 1) // k_full
    masks = np.zeros((rows, n), dtype=np.uint8)
    proposed = np.zeros((rows, n), dtype=np.uint8)
    if replay_masks is not None:
        replay_masks = np.asarray(replay_masks, dtype=np.uint8)
        if replay_masks.shape != (rows, n):
            raise ValueError(f"replay_masks must be {rows} x {n}")
    margins, logits, ambiguous = [], [], []
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
            skip, amb, z, _ = skip_decisions(weights, features(g, spins, lf, b, T[b], A, B, M), p)
            logits.append(z)
            ambiguous.append(amb)
            margins.append(float(np.min(np.abs(z - thr))))
        else:
            raise ValueError(proposal)
        proposed[row] = skip
        if replay_masks is not None:
            skip = replay_masks[row] != 0
        masks[row] = skip
        res = oracle_anneal(g, T[:end], seed, start_sweep=b + 1, init=spins, skip=skip, last_flip=lf, **kw)
        spins, M = res["spins"], res["M"]
    if res is None:  # start_sweep == S: nothing runs
        res = oracle_anneal(g, T, seed, start_sweep=S, init=init, **kw)
        spins = res["spins"]
    return dict(spins=spins, M=res["M"], cut=res["cut"], masks=masks, proposed=proposed, margins=margins,
                logits=logits, ambiguous=ambiguous, threshold=thr, last_flip=lf)


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
