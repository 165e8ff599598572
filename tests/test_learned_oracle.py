"""Pins of the learned-proposal reference (oracle/learned_ref.py) against facts outside it:
torch's BF16 cast, finite differences and torch autograd for the network's gradient,
closed forms of a constant network, an independent FP32 evaluation for the error model,
the oracle's brute-force-pinned flip cost for the features, the pure-Python annealer
for skipped nodes, and the plain schedule for the degenerate proposals."""
import numpy as np
import pytest

import gdi_synth as gs
from oracle import learned_ref as L
from oracle import ref_tiny


def rand_weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    d = dict(w1=rng.normal(0, scale, (64, 6)), b1=rng.normal(0, 0.1, 64), w2=rng.normal(0, scale / 8, (64, 64)),
             b2=rng.normal(0, 0.1, 64), w3=rng.normal(0, scale / 8, 64), b3=float(rng.normal(0, 0.1)))
    return L.flatten(d)


def test_bf16_rounding_matches_torch():
    import torch

    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1.0078125 + 2**-24, 65504.0, -3.0e-39]]
                       ).astype(np.float32)
    # exact ties between two BF16 values go to the even one
    ties = (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(L.bf16(x).view(np.uint32), ref.view(np.uint32))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    w = rand_weights(3)
    X = rng.normal(0, 1, (64, 6))
    y = (rng.random(64) < 0.4).astype(np.float64)
    loss, g = L.mlp_loss_grad(w, X, y, round_points=False)
    idx = np.concatenate([rng.choice(384, 12, replace=False), 384 + rng.choice(64, 6, replace=False),
                          448 + rng.choice(4096, 20, replace=False), 4544 + rng.choice(64, 6, replace=False),
                          4608 + rng.choice(64, 6, replace=False), [4672]])
    eps = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (L.mlp_loss_grad(wp, X, y, False)[0] - L.mlp_loss_grad(wm, X, y, False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    import torch

    rng = np.random.default_rng(4)
    w = rand_weights(5)
    X = rng.normal(0, 1, (200, 6))
    y = (rng.random(200) < 0.5).astype(np.float64)
    loss, g = L.mlp_loss_grad(w, X, y, round_points=False)
    P = {k: torch.tensor(np.asarray(v), dtype=torch.float64, requires_grad=True) for k, v in L.unflatten(w).items()}
    x = torch.tensor(X)
    z = torch.relu(torch.relu(x @ P["w1"].T + P["b1"]) @ P["w2"].T + P["b2"]) @ P["w3"] + P["b3"]
    tl = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(y))
    tl.backward()
    tg = L.flatten({k: v.grad.numpy() for k, v in P.items()})
    assert abs(tl.item() - loss) < 1e-12
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-14)


def test_constant_network_closed_forms():
    """All weights zero except b3: z = b3 for every row, loss = softplus(b3) - mean(y) b3,
    dL/db3 = sigmoid(b3) - mean(y), and every other gradient is zero."""
    w = np.zeros(L.MLP_PARAMS)
    w[-1] = 0.75
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (100, 6))
    y = (rng.random(100) < 0.3).astype(np.float64)
    loss, g = L.mlp_loss_grad(w, X, y)
    assert np.isclose(loss, np.log1p(np.exp(0.75)) - y.mean() * 0.75, rtol=1e-14)
    assert np.isclose(g[-1], 1 / (1 + np.exp(-0.75)) - y.mean(), rtol=1e-14)
    assert not np.any(g[:-1])
    assert np.all(L.mlp_logits(w, X) == 0.75)
    m = L.mlp_error_model(w, X.astype(np.float32), y)
    assert np.all(m["z"] == 0.75) and np.allclose(m["z_bound"], L._gamma(67) * 0.75, rtol=1e-12)


def fp32_network(w, X, y):
    """The network evaluated in FP32 with numpy's float32 matrix products (BLAS order, not
    any device's) and BF16 storage at the definition's points: a second, independent FP32
    evaluation for checking the error model. Returns logits, loss and flat gradient."""
    P = {k: np.asarray(v, dtype=np.float32) for k, v in L.unflatten(w).items()}
    f32 = np.float32
    x = L.bf16(np.asarray(X, np.float32)[:, :6])
    W1, W2 = L.bf16(P["w1"]), L.bf16(P["w2"])
    h1 = L.bf16(np.maximum(x @ W1.T + P["b1"], f32(0)))
    pre2 = h1 @ W2.T + P["b2"]
    h2 = np.maximum(pre2, f32(0))
    z = h2 @ P["w3"] + f32(P["b3"])
    n = x.shape[0]
    yf = np.asarray(y, np.float32)
    sig = f32(1) / (f32(1) + np.exp(-z))
    loss = np.sum(np.maximum(z, f32(0)) + np.log1p(np.exp(-np.abs(z))) - yf * z, dtype=np.float32) / f32(n)
    dz = (sig - yf) * (f32(1) / f32(n))
    dpre2 = np.where(pre2 > 0, dz[:, None] * P["w3"][None, :], f32(0))
    dp2 = L.bf16(dpre2)
    dpre1 = np.where(h1 > 0, dp2 @ W2, f32(0))
    g = dict(w1=L.bf16(dpre1).T @ x, b1=dpre1.sum(axis=0), w2=dp2.T @ h1, b2=dpre2.sum(axis=0),
             w3=h2.T @ dz, b3=dz.sum())
    return z.astype(np.float64), float(loss), L.flatten({k: np.asarray(v, np.float64) for k, v in g.items()})


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_error_model_contains_an_fp32_evaluation(seed):
    """An FP32 evaluation of the network in another summation order (numpy's float32
    BLAS) lands within the error model's bounds of the FP64 definition, for every logit and
    every gradient element; and the bounds are not vacuous."""
    rng = np.random.default_rng(seed)
    w = rand_weights(seed + 10).astype(np.float32)
    X = L.bf16(rng.normal(0, 1, (3000, 6)).astype(np.float32))
    y = (rng.random(3000) < 0.4).astype(np.uint8)
    m = L.mlp_error_model(w, X, y)
    z32, loss32, g32 = fp32_network(w, X, y)
    assert np.all(np.abs(z32 - m["z"]) <= m["z_bound"])
    assert abs(loss32 - m["loss"]) <= m["loss_bound"]
    assert np.all(np.abs(g32 - m["grad"]) <= m["grad_bound"])
    # the FP64 definition is the reference's: same loss and gradient as mlp_loss_grad
    loss64, g64 = L.mlp_loss_grad(w.astype(np.float32).astype(np.float64), X, y, round_points=True)
    assert m["loss"] == pytest.approx(loss64, rel=1e-12) and np.allclose(m["grad"], g64, rtol=1e-12, atol=1e-18)
    # not vacuous: logit bounds below 1e-3 (1 + |z|) at the median, gradient bounds a few
    # per mille of each tensor's largest entry
    assert np.median(m["z_bound"] / (1 + np.abs(m["z"]))) < 1e-3
    gu, bu = L.unflatten(m["grad"]), L.unflatten(m["grad_bound"])
    for k in ("w1", "b1", "w2", "b2", "w3"):
        assert bu[k].max() < 2e-2 * np.abs(gu[k]).max(), k


def test_skip_decisions_band():
    """Nodes outside the band are decided by the FP64 logit; the band is the logit bound
    plus the threshold's FP32 error, and an FP32 evaluation never contradicts a decision
    outside it."""
    rng = np.random.default_rng(12)
    w = rand_weights(13).astype(np.float32)
    X = L.bf16(rng.normal(0, 1, (20000, 6)).astype(np.float32))
    skip, amb, z, thr = L.skip_decisions(w, X, 0.5)
    assert thr == 0.0 and np.array_equal(skip, z > 0)
    z32 = fp32_network(w, X, np.zeros(20000))[0]
    thr32 = np.log(np.float32(0.5) / (np.float32(1) - np.float32(0.5)))
    assert np.array_equal((z32 > thr32)[~amb], skip[~amb])
    assert amb.mean() < 1e-2


def test_features_against_flip_cost_and_cut():
    """With T = 1 and unit-scale inputs the features hold exact integers: 4 f3 = B s h and
    16 f4 = |4A(1 - s M)|, whose signed sum is the single-flip energy change of eq. 6
    (the oracle's flip_delta, pinned by brute force); sum_i deg_i f2_i counts every cut
    edge twice."""
    import oracle

    g = gs.er_graph(150, 0.03, 31, "unit")
    rng = np.random.default_rng(9)
    s = np.where(rng.random(g.n) < 0.5, 1, -1).astype(np.int8)
    M = int(s.astype(np.int64).sum())
    lf = rng.integers(-1, 40, g.n).astype(np.int32)
    A, B = 1, 1
    f = L.features(g, s, lf, 40, 1.0, A, B, M).astype(np.float64)
    deg = np.diff(g.row_ptr)
    assert np.array_equal(f[:, 0] * 16, deg) and np.array_equal(f[:, 1] * 16, deg)
    for i in range(g.n):
        sh, bal = 4 * f[i, 3], 16 * f[i, 4]
        if abs(sh) < 16 and bal < 64:
            sign = 1 if 1 - s[i] * M >= 0 else -1
            assert sh + sign * bal == oracle.flip_delta(g, s, A, B, i), i
    crossing = oracle.cut(g, s)[1]
    assert np.isclose(np.sum(deg * f[:, 2]), 2 * crossing, rtol=1e-2)
    assert np.array_equal(f[:, 5], L.bf16(np.minimum(40 - lf, 255) / np.float32(64)))


def test_skipped_nodes_match_pure_python_annealer():
    """The C oracle's skip set against the independent pure-Python annealer."""
    import oracle

    for k in range(6):
        g = gs.er_graph(60, 0.08, 40 + k, "pm1" if k % 2 else "unit")
        T = gs.geometric_temps(2.0, 0.2, 8)
        rng = np.random.default_rng(k)
        skip = rng.random(g.n) < 0.4
        edges = [(i, int(g.col[q]), int(g.w[q])) for i in range(g.n)
                 for q in range(g.row_ptr[i], g.row_ptr[i + 1]) if g.col[q] > i]
        lf_c = np.full(g.n, -1, dtype=np.int32)
        r = oracle.anneal(g, T, 70 + k, skip=skip, last_flip=lf_c, mode=k % 2)
        lf_p = [-1] * g.n
        s, M, cut = ref_tiny.anneal(g.n, edges, list(T), 70 + k, gated=(k % 2 == 0),
                                    skip=np.flatnonzero(skip).tolist(), last_flip=lf_p)
        assert list(r["spins"]) == s and (r["M"], r["cut"]) == (M, cut)
        assert list(lf_c) == lf_p
        # skipped nodes keep their initial spins
        init = oracle.anneal(g, T[:1], 70 + k, start_sweep=1)["spins"]
        assert np.array_equal(r["spins"][skip], init[skip])


def test_degenerate_proposals_reduce_to_the_plain_schedule():
    import oracle

    g = gs.rgg_graph(1500, 8.0, 41)
    T = gs.geometric_temps(2.5, 0.05, 37)
    plain = oracle.anneal(g, T, 12)
    for kw in (dict(k_full=5, proposal="none"), dict(k_full=1, proposal="heuristic", heuristic_k=1),
               dict(k_full=6, proposal="heuristic", heuristic_k=1000)):
        r = L.learned_anneal(g, T, 12, **kw)
        assert np.array_equal(r["spins"], plain["spins"]) and r["cut"] == plain["cut"], kw
    # a proposal that starts only after the last sweep never skips anything
    r = L.learned_anneal(g, T, 12, k_full=3, proposal="heuristic", heuristic_k=1, learn_from=T.size)
    assert np.array_equal(r["spins"], plain["spins"]) and r["masks"].shape == (0, g.n)
    # the same with a resumed start
    head = oracle.anneal(g, T[:10], 12)
    r = L.learned_anneal(g, T, 12, k_full=4, proposal="none", start_sweep=10, init=head["spins"])
    assert np.array_equal(r["spins"], plain["spins"])


def test_skip_everything_runs_only_the_full_sweeps():
    """A network whose logit is always above the threshold skips every node in the masked
    sweeps: the result equals running only sweeps 0, k, 2k, ... (one-sweep oracle calls)."""
    import oracle

    g = gs.er_graph(700, 0.01, 42, "pm1")
    T = gs.geometric_temps(2.0, 0.1, 21)
    w = np.zeros(L.MLP_PARAMS)
    w[-1] = 5.0
    r = L.learned_anneal(g, T, 3, k_full=4, proposal="network", weights=w, p=0.5)
    spins = None
    for b in range(0, 21, 4):
        spins = oracle.anneal(g, T[:b + 1], 3, start_sweep=b, init=spins)["spins"]
    assert np.array_equal(r["spins"], spins)
    assert r["masks"][:-1].all() and not r["masks"][-1].any()


def test_mask_replay():
    """Replaying a run's own masks reproduces it; replaying the all-skip masks with a
    network that never skips runs only the full sweeps while ``proposed`` still holds
    the network's own (all-zero) decisions."""
    import oracle

    g = gs.er_graph(700, 0.01, 42, "pm1")
    T = gs.geometric_temps(2.0, 0.1, 21)
    w = np.zeros(L.MLP_PARAMS)
    w[-1] = -5.0  # never skips
    own = L.learned_anneal(g, T, 3, k_full=4, proposal="network", weights=w, p=0.5)
    again = L.learned_anneal(g, T, 3, k_full=4, proposal="network", weights=w, p=0.5, replay_masks=own["masks"])
    assert np.array_equal(again["spins"], own["spins"]) and again["cut"] == own["cut"]
    assert not own["masks"].any() and np.array_equal(again["proposed"], own["masks"])
    forced = np.ones_like(own["masks"])
    forced[-1] = 0
    r = L.learned_anneal(g, T, 3, k_full=4, proposal="network", weights=w, p=0.5, replay_masks=forced)
    spins = None
    for b in range(0, 21, 4):
        spins = oracle.anneal(g, T[:b + 1], 3, start_sweep=b, init=spins)["spins"]
    assert np.array_equal(r["spins"], spins) and not r["proposed"].any()
    with pytest.raises(ValueError):
        L.learned_anneal(g, T, 3, k_full=4, proposal="network", weights=w, p=0.5, replay_masks=forced[:-1])


def test_trace_labels_follow_per_sweep_states():
    """Label 1 iff the spin does not change in any of the k_label sweeps that follow the
    snapshot (a node decides once per sweep; checked with one-sweep oracle calls)."""
    import oracle

    g = gs.rgg_graph(900, 10.0, 43, "pm1")
    T = gs.geometric_temps(3.0, 0.8, 30)
    X, y = L.trace_dataset(g, T, 5, every=10, k_label=4, max_snapshots=5)
    assert X.shape == (2 * g.n, 6) and y.shape == (2 * g.n,)  # snapshots after sweeps 9 and 19
    states = [None]
    for t in range(30):
        states.append(oracle.anneal(g, T[:t + 1], 5, start_sweep=t, init=states[-1])["spins"])
    for snap, ts in enumerate((9, 19)):
        still = np.all(np.stack([states[ts + 1 + j] == states[ts + 2 + j] for j in range(4)]), axis=0)
        assert np.array_equal(y[snap * g.n:(snap + 1) * g.n], still.astype(np.uint8))
        assert 0 < still.mean() < 1
