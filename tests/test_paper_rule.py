"""Pins of the paper's acceptance rule (Sec. V, Alg. 2 and 3: the energy-minimising
value, then a random flip with probability P_f) in the oracle, against facts outside
it: the independent pure-Python annealer, closed forms with A = B = 0, greedy descent
with P_f = 0, and the brute-force-pinned single-flip energy change."""
import numpy as np
import pytest

import gdi_synth as gs
import oracle
from oracle import ref_tiny


def edges_of(g):
    return [(i, int(g.col[q]), int(g.w[q])) for i in range(g.n)
            for q in range(g.row_ptr[i], g.row_ptr[i + 1]) if g.col[q] > i]


@pytest.mark.parametrize("gated", [True, False])
def test_matches_pure_python_annealer(gated):
    for k in range(5):
        g = gs.er_graph(70, 0.07, 90 + k, "pm1" if k % 2 else "unit")
        pf = gs.geometric_temps(0.3, 0.01, 9)
        r = oracle.anneal(g, pf, 40 + k, mode=0 if gated else 1, rule=oracle.RULE_PAPER, A=1, B=2)
        s, M, cut = ref_tiny.anneal(g.n, edges_of(g), list(pf), 40 + k, A=1, B=2, gated=gated, paper_rule=True)
        assert list(r["spins"]) == s and (r["M"], r["cut"]) == (M, cut)


def test_zero_coefficients_leave_only_the_random_flips():
    """A = B = 0: dE = 0, the argmin keeps every spin, so node i ends as its initial spin
    times (-1)^(number of sweeps t with x0(i, t) < floor(2^32 P_f(t)))."""
    g = gs.rgg_graph(300, 6.0, 91)
    pf = np.array([0.5, 0.25, 0.9, 0.0, 1.0, 0.125, 0.7])
    seed = 17
    r = oracle.anneal(g, pf, seed, A=0, B=0, rule=oracle.RULE_PAPER)
    init = oracle.anneal(g, pf[:1], seed, start_sweep=1)["spins"].astype(np.int64)
    expect = []
    for i in range(g.n):
        flips = sum(ref_tiny.philox4x32_10(seed, (i, t, 0, 0))[0] < ref_tiny.flip_threshold(p) for t, p in enumerate(pf))
        expect.append(init[i] * (-1) ** flips)
    assert np.array_equal(r["spins"], np.array(expect, dtype=np.int8))


def test_zero_flip_probability_is_greedy_descent():
    """P_f = 0 and A = 0: each phase flips exactly the class members whose flip lowers
    the cut, so the cut never rises, and the end state is a local minimum of the cut
    (no single flip lowers it, by the brute-force-pinned flip cost)."""
    g = gs.rgg_graph(2000, 8.0, 92, "pm1")
    pf = np.zeros(30)
    r = oracle.anneal(g, pf, 3, A=0, B=1, rule=oracle.RULE_PAPER, phase_trace=True)
    cuts = r["phase_cut"].ravel()
    assert np.all(np.diff(cuts) <= 0)
    s = r["spins"]
    for i in range(0, g.n, 7):
        assert oracle.flip_delta(g, s, 0, 1, i) >= 0


def test_certain_flip_alternates():
    """P_f = 1 with A = B = 0: the threshold is 2^32 - 1, so every spin flips in every
    sweep unless x0 = 2^32 - 1."""
    g = gs.er_graph(200, 0.05, 93)
    pf = np.ones(6)
    init = oracle.anneal(g, pf[:1], 5, start_sweep=1)["spins"]
    r = oracle.anneal(g, pf, 5, A=0, B=0, rule=oracle.RULE_PAPER)
    assert np.array_equal(r["spins"], init)  # six flips


def test_rejects_probabilities_outside_unit_interval():
    g = gs.er_graph(50, 0.1, 94)
    for bad in (np.array([0.5, 1.5]), np.array([-0.1]), np.array([np.nan])):
        with pytest.raises(RuntimeError):
            oracle.anneal(g, bad, 1, rule=oracle.RULE_PAPER)
