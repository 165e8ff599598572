"""Pins of the paper's acceptance rule (Sec. V, Alg. 2 and 3: the energy-minimising
value, a random value on a tie, then a random flip with probability P_f) in the
oracle, against facts outside it: the independent pure-Python annealer, closed forms
with A = B = 0, ties on an alternating cycle, greedy descent with P_f = 0, and the
brute-force-pinned single-flip energy change."""
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


def test_zero_coefficients_leave_only_the_random_values():
    """A = B = 0: every dE is 0, so in every sweep the energy-minimising value is a tie
    and the spin takes a random value (Sec. III: +1 iff Philox word x2 is odd), which the
    random flip then inverts when x0 < floor(2^32 P_f). Hence node i ends as
    v(x2(i, S-1)) * (-1)^[x0(i, S-1) < floor(2^32 P_f(S-1))], whatever came before."""
    g = gs.rgg_graph(300, 6.0, 91)
    seed = 17
    for pf in (np.array([0.5, 0.25, 0.9, 0.0, 1.0, 0.125, 0.7]), np.array([0.3, 0.0]), np.array([1.0])):
        r = oracle.anneal(g, pf, seed, A=0, B=0, rule=oracle.RULE_PAPER)
        last = pf.size - 1
        expect = []
        for i in range(g.n):
            x = ref_tiny.philox4x32_10(seed, (i, last, 0, 0))
            value = 1 if x[2] & 1 else -1
            expect.append(-value if x[0] < ref_tiny.flip_threshold(pf[last]) else value)
        assert np.array_equal(r["spins"], np.array(expect, dtype=np.int8))
    # the tie's values are fair coins: about half of the spins end +1 with P_f = 0
    g = gs.rgg_graph(20_000, 6.0, 95)
    r = oracle.anneal(g, np.zeros(3), 8, A=0, B=0, rule=oracle.RULE_PAPER)
    assert abs(float(np.mean(r["spins"] > 0)) - 0.5) < 4 * 0.5 / np.sqrt(g.n)


def test_tie_takes_a_random_value_not_the_old_one():
    """A node whose local energy is the same for both values (dE = 0: zero local field of
    eq. 2, Sec. III) takes a random value; with the value kept instead, a greedy schedule
    (P_f = 0, A = 0) could never move such a node. On a cycle of length 4k with spins
    + + - - + + - - ..., every node has one neighbour of each sign, so h = 0 and every node
    of the first phase sees dE = 0."""
    n = 40
    g = gs.from_edges(n, np.arange(n), (np.arange(n) + 1) % n, np.ones(n, np.int64))
    init = np.where(np.arange(n) % 4 < 2, 1, -1).astype(np.int8)
    seed = 5
    r = oracle.anneal(g, np.zeros(1), seed, A=0, B=1, rule=oracle.RULE_PAPER, init=init, phase_spins=True)
    col, C = oracle.colour(g)
    assert C == 2  # first fit on an even cycle: even ids colour 0, odd ids colour 1
    after0 = r["phase_spins"][0, 0]
    for i in np.flatnonzero(col == 0):
        x = ref_tiny.philox4x32_10(seed, (int(i), 0, 0, 0))
        assert after0[i] == (1 if x[2] & 1 else -1)
    assert np.any(after0[col == 0] != init[col == 0])  # some tied nodes moved


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


def test_certain_flip_inverts_the_tie_value():
    """P_f = 1 with A = B = 0: the threshold is 2^32 - 1, so each spin ends as the
    opposite of its last tie value unless x0 = 2^32 - 1."""
    g = gs.er_graph(200, 0.05, 93)
    pf = np.ones(6)
    r = oracle.anneal(g, pf, 5, A=0, B=0, rule=oracle.RULE_PAPER)
    expect = []
    for i in range(g.n):
        x = ref_tiny.philox4x32_10(5, (i, 5, 0, 0))
        value = 1 if x[2] & 1 else -1
        expect.append(value if x[0] == 0xFFFFFFFF else -value)
    assert np.array_equal(r["spins"], np.array(expect, dtype=np.int8))


def test_rejects_probabilities_outside_unit_interval():
    g = gs.er_graph(50, 0.1, 94)
    for bad in (np.array([0.5, 1.5]), np.array([-0.1]), np.array([np.nan])):
        with pytest.raises(RuntimeError):
            oracle.anneal(g, bad, 1, rule=oracle.RULE_PAPER)
