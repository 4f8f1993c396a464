"""Pins for the per-source switch step of Eq. 14 (oracle.tgt.switch_step) and
the adaptive TGT+ built on it (Algorithm 4 with tilde_tau chosen per source).

* a worked example on K_4 computed by hand from Lemma 4.3, Eq. 13, Eq. 14,
  Eq. 17 and Algorithm 3: the two sides of Eq. 14 at l = 0, 1, 2 and the
  resulting tilde_tau = 2 with one walk pair per half;
* when walks are never cheaper (tiny eps: huge walk counts) every source
  traverses to max_j tau_ij and adaptive TGT+ equals TGT exactly;
* rule 1 (walk steps) never switches earlier than rule 0 (walk pairs): its
  right-hand side is at least as large at every l;
* the estimate is within eps of the exact SC (Theorem 4.4 with delta = 1/n);
* planted mistakes (support size instead of volume, a one-sided Eq. 13
  constant) change the hand-computed trace.
"""
import math

import numpy as np
import pytest

import graphgen as gg
from oracle import exact as ex
from oracle import tgt


def k4_trace(fn=None):
    n, u, v = gg.complete_graph(4)
    G = tgt.Graph(n, u, v)
    H = G.halves_of([0])
    trace = []
    tt, nr = (fn or tgt.switch_step)(G, 0, np.full(len(H), 5), 0.9, 0.25, 10, 0, trace)
    return tt, nr, trace


def test_k4_worked_example():
    # K_4, source 0, tau = 5 on every edge, eps = 0.9, delta = 1/4, gamma = 10:
    # Eq. 13 constant 8 ln(2m/delta) / (d^2 eps^2) = 8 ln 48 / (9 * 0.81) = 4.2482.
    # l = 0: q = e_0; chi = UB_0 + UB_j = (0 + 1/2 + 4/2) + (1/2 + 1/2 + 4/2) = 5.5
    #        -> n_r = ceil(4.2482 * 30.25) = 129 per half, Eq. 14: 3 > 387 fails.
    # l = 1: q = (0, 1/3, 1/3, 1/3), rho = 2/3, L' = 4;
    #        UB_0 = 1/6 + 1/6 + 1 = 4/3, LB_0 = 1/3, UB_j = 4/3, LB_j = 0
    #        chi = 7/3 -> n_r = ceil(4.2482 * 49/9) = 24, Eq. 14: 9 > 72 fails.
    # l = 2: q = (1/3, 2/9, 2/9, 2/9), rho = 5/9, L' = 3;
    #        UB_0 = 1/9 + 1/6 + 5/9 = 5/6, LB_0 = 2/3, UB_j = 8/9, LB_j = 2/3
    #        chi = 7/18 -> n_r = ceil(0.6425) = 1, Eq. 14: 12 > 3 holds.
    c = 8 * math.log(48) / (9 * 0.81)
    assert math.ceil(c * 5.5 ** 2) == 129
    assert math.ceil(c * (7 / 3) ** 2) == 24
    assert math.ceil(c * (7 / 18) ** 2) == 1
    tt, nr, trace = k4_trace()
    assert tt == 2
    assert list(nr) == [1, 1, 1]
    assert [(l, a, b) for l, a, b in trace] == [(0, 3.0, 387.0), (1, 9.0, 72.0), (2, 12.0, 3.0)]


def _switch_count_support(g, i, tau_half_i, eps, delta, gamma, rule=0, trace=None):
    # planted mistake: the left side counts support nodes instead of their degrees
    H = g.halves_of([i])
    hj = g.hdst[H]
    tau_h = np.asarray(tau_half_i)
    x = np.zeros(g.n)
    x[i] = 1.0
    ell = 0
    while True:
        lhs = float((x != 0).sum())
        nr = np.zeros(len(H), dtype=np.int64)
        for k in range(len(H)):
            length = int(tau_h[k] - ell)
            if length > 0:
                nr[k] = tgt.walk_count(tgt.chi_value(g, x, i, int(hj[k]), length, gamma),
                                       g.degf[i], eps, g.m, delta)
        rhs = float(nr.sum())
        if trace is not None:
            trace.append((ell, lhs, rhs))
        if lhs > rhs:
            return ell, nr
        x = g.P @ x
        ell += 1


def test_planted_volume_mistake_changes_trace():
    with pytest.raises(AssertionError):
        _, _, trace = k4_trace(_switch_count_support)
        assert [(l, a, b) for l, a, b in trace] == [(0, 3.0, 387.0), (1, 9.0, 72.0),
                                                    (2, 12.0, 3.0)]


def test_planted_walk_count_mistake_changes_trace(monkeypatch):
    # Eq. 13 with eps instead of eps^2 in the denominator
    orig = tgt.walk_count

    def wrong(chi, deg_i, eps, m, delta):
        return orig(chi, deg_i, math.sqrt(eps), m, delta)

    monkeypatch.setattr(tgt, "walk_count", wrong)
    _, _, trace = k4_trace()
    assert [(l, a, b) for l, a, b in trace] != [(0, 3.0, 387.0), (1, 9.0, 72.0), (2, 12.0, 3.0)]


@pytest.mark.parametrize("graph", [gg.tree_plus_gnp(60, 6.0, 3), gg.barabasi_albert(70, 3, 4)])
def test_tiny_eps_traverses_to_the_end_and_equals_tgt(graph):
    n, u, v = graph
    G = tgt.Graph(n, u, v)
    tau = np.full(len(u), 5)
    s, tilde, nr_uv, nr_vu = tgt.tgt_plus_adaptive(G, tau, 1e-7, 1.0 / n, 10, seed=3)
    assert np.all(tilde == 5)
    assert nr_uv.sum() == 0 and nr_vu.sum() == 0
    np.testing.assert_allclose(s, tgt.truncated_sc(G, tau), atol=1e-14)


def test_step_rule_switches_no_earlier():
    n, u, v = gg.barabasi_albert(120, 3, 5)
    G = tgt.Graph(n, u, v)
    lam = ex.lambda_star(n, u, v)
    eps = 0.02
    tau = tgt.tau_lambda_bound(G.degf[u], G.degf[v], eps / 2, lam)
    tau_half = np.concatenate([tau, tau])
    for i in range(0, n, 7):
        H = G.halves_of([i])
        t0, _ = tgt.switch_step(G, i, tau_half[H], eps, 1.0 / n, 10, 0)
        t1, _ = tgt.switch_step(G, i, tau_half[H], eps, 1.0 / n, 10, 1)
        assert t1 >= t0
        assert t0 >= 1            # at l = 0 every half needs >= 1 walk: d_i > d_i fails


@pytest.mark.parametrize("rule", [0, 1])
def test_adaptive_tgt_plus_within_eps(rule):
    n, u, v = gg.tree_plus_gnp(50, 6.0, 7)
    G = tgt.Graph(n, u, v)
    eps = 0.05
    lam = ex.lambda_star(n, u, v)
    tau = tgt.tau_lambda_bound(G.degf[u], G.degf[v], eps / 2, lam)
    s, tilde, _, _ = tgt.tgt_plus_adaptive(G, tau, eps, 1.0 / n, 10, seed=11, rule=rule)
    assert np.abs(s - ex.sc_pinv(n, u, v)).max() <= eps
    assert tilde.min() >= 1 and np.all(tilde <= tau.max())
