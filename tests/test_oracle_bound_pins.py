"""Equality pins for the walk bounds, chi and rho-hat of the TGT+ oracle.

Lemma 4.3 bounds the score sum of any walk of length l; Eq. 17 (and Eq. 15
for gamma = 0) turns the bounds into the range width chi of X * d_i (Eq. 11);
Algorithm 3 replaces rho_i (Eq. 16) by rho-hat.  Validity (bound <= truth)
would also hold for looser formulas, so these tests check equality: on two
small graphs with hand-set score vectors q, built so that the extreme walks
realise the bounds (the first step goes to the best neighbour, every later
pair of consecutive nodes is the best edge of Eq. 16, the walk ends on the
best node of V), the bounds equal the extremes found by enumerating every
walk, and chi equals the exact width of S_i - S_j.  Rho-hat is checked in
both branches of Algorithm 3 against the brute-force rho and a hand-computed
value.  A second set of tests plants plausible mistakes in copies of the
oracle functions and shows that the equality pins reject each of them.
"""
import itertools

import numpy as np
import pytest

import graphgen as gg
from oracle import tgt


def graph_a():
    """7 nodes, triangle 0-1-2: i = 0, j = 1, best neighbour 2 of both,
    global maximum 3 (edge 2-3 is the best edge), worst neighbour 4 of both,
    global minimum 5 (edge 4-5).  Bounds are exact at l = 2."""
    u = np.array([0, 0, 1, 2, 0, 1, 4, 3, 5])
    v = np.array([1, 2, 2, 3, 4, 4, 5, 6, 6])
    q = np.array([0.30, 0.20, 0.50, 0.90, 0.10, 0.05, 0.25])
    return tgt.Graph(7, u, v), q


def graph_b():
    """Same shape; the maximum is held by the adjacent pair 2, 3 and the
    minimum by the adjacent pair 4, 5, so the extreme walks alternate on
    those pairs and every bound is exact at every l."""
    u = np.array([0, 0, 1, 2, 0, 1, 4, 3, 5])
    v = np.array([1, 2, 2, 3, 4, 4, 5, 6, 6])
    q = np.array([0.30, 0.20, 0.60, 0.60, 0.05, 0.05, 0.25])
    return tgt.Graph(7, u, v), q


def graph_c():
    """As graph_a with a different worst neighbour for j: N(0) has its minimum
    at 4 and N(1) at 6, both adjacent to the global minimum 5, so the lower
    bounds of i and j differ and both are exact at l = 2."""
    u = np.array([0, 0, 1, 2, 0, 4, 1, 5, 3])
    v = np.array([1, 2, 2, 3, 4, 5, 6, 6, 4])
    q = np.array([0.30, 0.20, 0.50, 0.90, 0.10, 0.05, 0.15])
    return tgt.Graph(7, u, v), q


def walk_sums(G, q, start, length):
    """Score sums of every walk of `length` steps from `start` (start excluded)."""
    sums = []

    def rec(node, left, acc):
        if left == 0:
            sums.append(acc)
            return
        for x in G.nbr[G.indptr[node]: G.indptr[node + 1]]:
            rec(int(x), left - 1, acc + q[x])

    rec(start, length, 0.0)
    return np.array(sums)


def check_bounds_exact(G, q, start, length):
    rho = tgt.rho_bruteforce(G, q)
    s = walk_sums(G, q, start, length)
    lb, ub = tgt.walk_bounds(G, q, start, length, rho)
    assert lb == pytest.approx(s.min(), abs=1e-14), (start, length, lb, s.min())
    assert ub == pytest.approx(s.max(), abs=1e-14), (start, length, ub, s.max())


def check_chi_exact(G, q, i, j, length, gamma):
    si = walk_sums(G, q, i, length)
    sj = walk_sums(G, q, j, length)
    width = (si.max() - sj.min()) - (si.min() - sj.max())
    chi = tgt.chi_value(G, q, i, j, length, gamma)
    assert chi == pytest.approx(width, abs=1e-13), (i, j, length, gamma, chi, width)


def pins_a():
    for G, q in (graph_a(), graph_c()):
        for start in (0, 1):
            check_bounds_exact(G, q, start, 2)
        check_chi_exact(G, q, 0, 1, 2, 10)
        check_chi_exact(G, q, 1, 0, 2, 3)


def pins_b():
    G, q = graph_b()
    for length in (1, 2, 3, 4):
        for start in (0, 1):
            check_bounds_exact(G, q, start, length)
        check_chi_exact(G, q, 0, 1, length, 0)          # Eq. 15
        check_chi_exact(G, q, 0, 1, length, 2)          # Eq. 17


def test_lemma_4_3_bounds_equal_enumerated_extremes():
    pins_a()
    pins_b()


def test_hand_values_graph_a():
    # LB(0, 2) = min_{N(0)} q + 1 * min_V q = 0.10 + 0.05
    # UB(0, 2) = 0.50/2 + 0.90/2 + 1 * 1.40/2 = 1.40 (rho = q2 + q3 = 1.40)
    G, q = graph_a()
    lb, ub = tgt.walk_bounds(G, q, 0, 2, 1.40)
    assert lb == pytest.approx(0.15, abs=1e-15)
    assert ub == pytest.approx(1.40, abs=1e-15)
    # chi (Eq. 17) = 2 * 1.40 - 2 * 0.15; Eq. 15 at l = 2: 2 * 2 * (0.90 - 0.05)
    assert tgt.chi_value(G, q, 0, 1, 2, 10) == pytest.approx(2.5, abs=1e-14)
    assert tgt.chi_value(G, q, 0, 1, 2, 0) == pytest.approx(3.4, abs=1e-14)
    # graph_c: LB(1, 2) = 0.15 + 0.05, so chi = 2 * 1.40 - 0.15 - 0.20
    G, q = graph_c()
    assert tgt.chi_value(G, q, 0, 1, 2, 10) == pytest.approx(2.45, abs=1e-14)


def test_lemma_4_3_bounds_valid_on_random_graphs():
    rng = np.random.default_rng(5)
    for seed in range(6):
        n, u, v = gg.random_small_connected(9, 14, seed)
        G = tgt.Graph(n, u, v)
        q = rng.random(n) ** 2
        rho = tgt.rho_bruteforce(G, q)
        for start in range(n):
            for length in (1, 2, 3, 4):
                s = walk_sums(G, q, start, length)
                lb, ub = tgt.walk_bounds(G, q, start, length, rho)
                assert lb <= s.min() + 1e-15 and s.max() <= ub + 1e-15


def test_rho_hat_candidate_pair_branch_is_exact():
    # Algorithm 3 lines 3-4: C = {3, 2, 0} holds the edges 2-3 and 0-2; the best
    # is 2-3 with 1.40, which is rho itself (q[c1] + q[c3] = 1.20 is smaller)
    G, q = graph_a()
    assert tgt.rho_hat(G, q, 3) == pytest.approx(1.40, abs=1e-15)
    assert tgt.rho_bruteforce(G, q) == pytest.approx(1.40, abs=1e-15)


def test_rho_hat_no_candidate_edge_branch():
    # Algorithm 3 line 5: C = {3, 5, 0} (q .7, .5, .4) has no edge inside, so
    # rho-hat = q[c1] + q[c3] = 1.1; the true rho (edge 2-3) is 0.9
    G, _ = graph_a()
    q = np.array([0.40, 0.10, 0.20, 0.70, 0.15, 0.50, 0.05])
    assert tgt.rho_hat(G, q, 3) == pytest.approx(1.10, abs=1e-15)
    assert tgt.rho_bruteforce(G, q) == pytest.approx(0.90, abs=1e-15)


def test_chi_width_contains_every_estimator_value():
    # X * d_i over every pair of walks lies inside a window of width chi
    G, q = graph_a()
    for length in (1, 2, 3):
        si = walk_sums(G, q, 0, length)
        sj = walk_sums(G, q, 1, length)
        diffs = (si[:, None] - sj[None, :]).ravel()
        for gamma in (0, 2, 10):
            assert diffs.max() - diffs.min() <= tgt.chi_value(G, q, 0, 1, length, gamma) + 1e-14


# ---------------------------------------------------------------- planted mistakes

def _bounds_ub_no_half(G, q, node, length, rho):
    nq = q[G.nbr[G.indptr[node]: G.indptr[node + 1]]]
    return nq.min() + (length - 1) * q.min(), nq.max() / 2 + q.max() / 2 + (length - 1) * rho


def _bounds_max_over_v(G, q, node, length, rho):
    nq = q[G.nbr[G.indptr[node]: G.indptr[node + 1]]]
    return nq.min() + (length - 1) * q.min(), q.max() / 2 + q.max() / 2 + (length - 1) * rho / 2


def _bounds_min_over_v(G, q, node, length, rho):
    nq = q[G.nbr[G.indptr[node]: G.indptr[node + 1]]]
    return q.min() + (length - 1) * q.min(), nq.max() / 2 + q.max() / 2 + (length - 1) * rho / 2


def _bounds_l_for_l_minus_1(G, q, node, length, rho):
    nq = q[G.nbr[G.indptr[node]: G.indptr[node + 1]]]
    return nq.min() + length * q.min(), nq.max() / 2 + q.max() / 2 + length * rho / 2


def _bounds_first_node_included(G, q, node, length, rho):
    lb, ub = tgt.__dict__["_orig_walk_bounds"](G, q, node, length, rho)
    return lb + q[node], ub + q[node]


@pytest.mark.parametrize("mutant", [_bounds_ub_no_half, _bounds_max_over_v, _bounds_min_over_v,
                                    _bounds_l_for_l_minus_1, _bounds_first_node_included])
def test_planted_bound_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setitem(tgt.__dict__, "_orig_walk_bounds", tgt.walk_bounds)
    monkeypatch.setattr(tgt, "walk_bounds", mutant)
    with pytest.raises(AssertionError):
        pins_a()
        pins_b()


def _chi_eq15_one_sided(G, q, i, j, length, gamma, rho=None):
    if gamma == 0:
        return length * (q.max() - q.min())
    return tgt.__dict__["_orig_chi_value"](G, q, i, j, length, gamma, rho)


def _chi_j_bounds_from_i(G, q, i, j, length, gamma, rho=None):
    if gamma == 0:
        return 2.0 * length * (q.max() - q.min())
    rho = tgt.rho_hat(G, q, gamma) if rho is None else rho
    lbi, ubi = tgt.walk_bounds(G, q, i, length, rho)
    return 2 * (ubi - lbi)


@pytest.mark.parametrize("mutant", [_chi_eq15_one_sided, _chi_j_bounds_from_i])
def test_planted_chi_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setitem(tgt.__dict__, "_orig_chi_value", tgt.chi_value)
    monkeypatch.setattr(tgt, "chi_value", mutant)
    with pytest.raises(AssertionError):
        pins_a()
        pins_b()


def _rho_pairs_only(G, q, gamma):
    C = tgt.top_candidates(q, gamma)
    best = -np.inf
    for a, b in itertools.combinations(C, 2):
        if G.adjacent(a, b):
            best = max(best, q[a] + q[b])
    return best if best > -np.inf else q[C[0]] + q[C[-1]]


def test_planted_unsafe_rho_reading_is_caught():
    # the candidate-pair edge alone (Q7 reading rejected) falls below rho on
    # the counterexample of four nodes
    G = tgt.Graph(4, np.array([1, 0]), np.array([2, 3]))
    q = np.array([0.5, 0.1, 0.09, 0.08])
    assert _rho_pairs_only(G, q, 3) < tgt.rho_bruteforce(G, q)
    assert tgt.rho_hat(G, q, 3) >= tgt.rho_bruteforce(G, q)
