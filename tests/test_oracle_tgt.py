"""Pins for the method oracle (oracle.tgt, oracle.philox).

Each check is against something the paper or mathematics fixes independently
of the code under test:

* the truncated series against its spectral closed form (Eq. 18 summed to tau);
* s_0 and s_1 as stated in the proof of Theorem 3.2;
* the trace identity sum_e s_tau(e) = n - tr(P^(tau+1)) (telescoping Eq. 2
  over all edges) and Foster in the limit;
* odd-tau monotonicity and the lambda* tail bound (proof of Theorem 3.2);
* reversibility p_l(i,j)/d_j = p_l(j,i)/d_i (Eq. 4);
* Lemma 4.1 (head + tail split) with the tail computed from rows of P^l;
* unbiasedness of X (Eq. 11) and the walk bounds of Lemma 4.3 on sampled walks;
* rho-hat >= rho (Eq. 16) and the counterexample to the unsafe reading;
* Philox4x32-10 known-answer vectors.
"""
import math
import os

import numpy as np
import pytest

import graphgen as gg
from oracle import exact as ex
from oracle import tgt
from oracle.philox import philox4x32_10, pick_index

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_graphs():
    return [
        gg.petersen_graph(),
        gg.triangle_pendant(),
        gg.two_triangles_bridge(),
        gg.tree_plus_gnp(120, 6.0, 11),
        gg.barabasi_albert(150, 3, 12),
        gg.king_grid(90),
    ]


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("tau", [0, 1, 3, 8, 15])
def test_traversal_matches_spectral_closed_form(gi, tau):
    n, u, v = small_graphs()[gi]
    s = tgt.truncated_sc(tgt.Graph(n, u, v), np.full(len(u), tau))
    np.testing.assert_allclose(s, ex.s_tau_eigen(n, u, v, tau), atol=1e-13)


def test_per_edge_truncation_matches_closed_form():
    n, u, v = gg.tree_plus_gnp(150, 7.0, 3)
    rng = np.random.default_rng(0)
    tau = 2 * rng.integers(0, 6, size=len(u)) + 1
    s = tgt.truncated_sc(tgt.Graph(n, u, v), tau)
    np.testing.assert_allclose(s, ex.s_tau_eigen(n, u, v, tau), atol=1e-13)


def test_first_two_terms_as_in_theorem_3_2_proof():
    n, u, v = gg.barabasi_albert(200, 4, 9)
    d = ex.degree_vector(n, u, v)
    G = tgt.Graph(n, u, v)
    s0 = tgt.truncated_sc(G, np.zeros(len(u), int))
    s1 = tgt.truncated_sc(G, np.ones(len(u), int))
    np.testing.assert_allclose(s0, 1 / d[u] + 1 / d[v], atol=1e-15)
    np.testing.assert_allclose(s1, 1 / d[u] + 1 / d[v] - 2 / (d[u] * d[v]), atol=1e-15)


@pytest.mark.parametrize("tau", [1, 2, 5, 9])
def test_trace_identity(tau):
    n, u, v = gg.tree_plus_gnp(200, 8.0, 4)
    s = tgt.truncated_sc(tgt.Graph(n, u, v), np.full(len(u), tau))
    # trace from an independent route: matrix power of the dense P
    a = ex.adjacency_dense(n, u, v)
    P = a / a.sum(1, keepdims=True)
    tr = np.trace(np.linalg.matrix_power(P, tau + 1))
    assert abs(s.sum() - (n - tr)) < 1e-10


def test_foster_limit_and_odd_monotonicity_and_lambda_bound():
    n, u, v = gg.tree_plus_gnp(150, 6.0, 8)
    G = tgt.Graph(n, u, v)
    s = ex.sc_pinv(n, u, v)
    lam = ex.lambda_star(n, u, v)
    d = ex.degree_vector(n, u, v)
    num = 1 / d[u] + 1 / d[v] - 2 / (d[u] * d[v])
    prev = None
    for tau in range(1, 30, 2):
        st = tgt.truncated_sc(G, np.full(len(u), tau))
        assert np.all(st <= s + 1e-13)
        if prev is not None:
            assert np.all(st >= prev - 1e-13)
        bound = lam ** (tau + 1) / (1 - lam ** 2) * num
        assert np.all(s - st <= bound + 1e-13)
        prev = st
    far = tgt.truncated_sc(G, np.full(len(u), 801))
    assert abs(far.sum() - (n - 1)) < 1e-8


def test_tau_lambda_bound_is_minimal_and_sufficient():
    n, u, v = gg.tree_plus_gnp(300, 10.0, 2)
    s = ex.sc_pinv(n, u, v)
    lam = ex.lambda_star(n, u, v)
    d = ex.degree_vector(n, u, v)
    for eps in (1e-1, 1e-2, 1e-3):
        tau = tgt.tau_lambda_bound(d[u], d[v], eps, lam)
        assert np.all(tau % 2 == 1)
        num = 1 / d[u] + 1 / d[v] - 2 / (d[u] * d[v])
        bnd = lam ** (tau + 1) / (1 - lam ** 2) * num
        assert np.all(bnd <= eps * (1 + 1e-12))
        big = tau >= 3
        prev = lam ** (tau[big] - 1) / (1 - lam ** 2) * num[big]
        assert np.all(prev > eps)
        st = tgt.truncated_sc(tgt.Graph(n, u, v), tau)
        assert np.abs(st - s).max() <= eps


def test_reversibility_of_recorded_probabilities():
    n, u, v = gg.barabasi_albert(120, 3, 5)
    G = tgt.Graph(n, u, v)
    m = len(u)
    _, _, diag, off = tgt.traversal(G, np.full(m, 5), record=6)
    d = G.degf
    # off[h] = p_l(j, i) for h = (i -> j); the reverse half holds p_l(i, j)
    np.testing.assert_allclose(off[:m] / d[u][:, None], off[m:] / d[v][:, None], atol=1e-15)
    # series terms from the recordings match Eq. 18
    t = tgt.series_terms(diag, off, G.degf[G.hsrc], G.degf[G.hdst], m)
    for ell in range(7):
        np.testing.assert_allclose(t[:, ell], ex.series_term_eigen(n, u, v, ell), atol=1e-14)


def test_lemma_4_1_head_plus_tail():
    n, u, v = gg.tree_plus_gnp(80, 6.0, 21)
    G = tgt.Graph(n, u, v)
    tau, tt = 9, 3
    g_full = tgt.traversal(G, np.full(len(u), tau))[0]
    g_head = tgt.traversal(G, np.full(len(u), tt))[0]
    for e in range(0, len(u), 5):
        i, j = int(u[e]), int(v[e])
        q = tgt.column_at(G, i, tt)
        tail = tgt.tail_exact(G, q, i, j, tau - tt)
        assert abs(g_head[e] + tail - g_full[e]) < 1e-14


# ------------------------------------------------------------------ walks and estimator

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        w = [int(x, 16) for x in r]
        out = philox4x32_10(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]


def test_pick_index_range_and_uniformity():
    rng = np.random.default_rng(1)
    words = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64)
    for deg in (1, 2, 3, 7, 1000):
        k = pick_index(words, deg)
        assert k.min() >= 0 and k.max() < deg
        if deg <= 7:
            cnt = np.bincount(k.astype(np.int64), minlength=deg)
            assert np.all(np.abs(cnt / len(words) - 1 / deg) < 0.01)
    assert int(pick_index(np.uint64(2 ** 32 - 1), 5)) == 4
    assert int(pick_index(np.uint64(0), 5)) == 0


def test_walks_follow_edges_and_are_reproducible():
    n, u, v = gg.barabasi_albert(100, 3, 2)
    G = tgt.Graph(n, u, v)
    w = tgt.walks(G, 5, int(G.nbr[G.indptr[5]]), np.arange(50), 0, 9, seed=77)
    prev = np.full(50, 5)
    for t in range(9):
        for a, b in zip(prev, w[:, t]):
            assert G.adjacent(a, b)
        prev = w[:, t]
    w2 = tgt.walks(G, 5, int(G.nbr[G.indptr[5]]), np.arange(50), 0, 9, seed=77)
    assert np.array_equal(w, w2)
    w3 = tgt.walks(G, 5, int(G.nbr[G.indptr[5]]), np.arange(50), 0, 9, seed=78)
    assert not np.array_equal(w, w3)


def test_walk_step_distribution_is_uniform_over_neighbours():
    n, u, v = gg.complete_graph(6)
    G = tgt.Graph(n, u, v)
    w = tgt.walks(G, 0, 1, np.arange(30000), 0, 1, seed=3)
    cnt = np.bincount(w[:, 0], minlength=6)
    assert cnt[0] == 0
    assert np.all(np.abs(cnt[1:] / 30000 - 0.2) < 0.012)


def test_estimator_is_unbiased():
    n, u, v = gg.tree_plus_gnp(40, 5.0, 13)
    G = tgt.Graph(n, u, v)
    tt, length = 2, 5
    for e in (0, 7, 20):
        i, j = int(u[e]), int(v[e])
        q = tgt.column_at(G, i, tt)
        xs = tgt.estimator_samples(G, q, i, j, 40000, length, seed=1234 + e)
        exact = tgt.tail_exact(G, q, i, j, length)
        se = xs.std() / math.sqrt(len(xs))
        assert abs(xs.mean() - exact) < 5 * se + 1e-15


def test_walk_sums_respect_lemma_4_3_bounds():
    n, u, v = gg.barabasi_albert(200, 4, 6)
    G = tgt.Graph(n, u, v)
    for i in (0, 17, 150):
        q = tgt.column_at(G, i, 2)
        j = int(G.nbr[G.indptr[i]])
        rho = tgt.rho_hat(G, q, 10)
        for length in (1, 2, 5):
            for side, start in ((0, i), (1, j)):
                w = tgt.walks(G, i, j, np.arange(3000), side, length, seed=9)
                S = q[w].sum(1)
                lb, ub = tgt.walk_bounds(G, q, start, length, rho)
                assert np.all(S >= lb - 1e-15) and np.all(S <= ub + 1e-15)
            chi = tgt.chi_value(G, q, i, j, length, 10)
            xs = tgt.estimator_samples(G, q, i, j, 3000, length, seed=9)
            assert xs.max() - xs.min() <= chi / G.degf[i] + 1e-15


def test_rho_hat_bounds_rho_and_catches_unsafe_reading():
    # counterexample: q = (.5, .1, .09, .08) on nodes c1, c2, c3, y with
    # edges c2-c3 and c1-y; with gamma = 3 the candidate-pair edge alone gives .19
    # while rho = .58.
    n = 4
    u = np.array([1, 0])
    v = np.array([2, 3])
    G = tgt.Graph(n, u, v)
    q = np.array([0.5, 0.1, 0.09, 0.08])
    assert tgt.rho_bruteforce(G, q) == pytest.approx(0.58)
    assert tgt.rho_hat(G, q, 3) >= 0.58
    # random score vectors on a real graph
    n, u, v = gg.barabasi_albert(300, 3, 4)
    G = tgt.Graph(n, u, v)
    rng = np.random.default_rng(3)
    for _ in range(30):
        q = rng.random(n) ** 4
        for gamma in (1, 3, 10):
            assert tgt.rho_hat(G, q, gamma) >= tgt.rho_bruteforce(G, q) - 1e-15


def test_walk_count_matches_hoeffding():
    # n_r is the smallest count for which the Hoeffding bound with range width
    # chi/d_i and deviation eps/4 is at most delta/m (Lemma 4.2, proof of Thm 4.4)
    for chi, d, eps, m, delta in [(0.3, 10, 1e-3, 10 ** 6, 1e-5), (0.05, 3, 1e-2, 5000, 1e-3),
                                  (1e-4, 50, 1e-2, 100, 0.1)]:
        nr = tgt.walk_count(chi, d, eps, m, delta)
        hb = lambda k: 2 * math.exp(-2 * k * (eps / 4) ** 2 / (chi / d) ** 2)
        assert hb(nr) <= delta / m * (1 + 1e-9)
        if nr > 1:
            assert hb(nr - 1) > delta / m


def test_replay_with_full_traversal_equals_tgt():
    n, u, v = gg.tree_plus_gnp(60, 6.0, 1)
    G = tgt.Graph(n, u, v)
    tau = np.full(len(u), 7)
    zeros = np.zeros(len(u), int)
    _, _, s = tgt.tgt_plus_replay(G, tau, np.full(n, 7), zeros, zeros, seed=1)
    np.testing.assert_allclose(s, tgt.truncated_sc(G, tau), atol=1e-14)


def test_replay_meets_eps():
    n, u, v = gg.tree_plus_gnp(50, 6.0, 2)
    G = tgt.Graph(n, u, v)
    eps, delta = 0.05, 1.0 / n
    lam = ex.lambda_star(n, u, v)
    tau = tgt.tau_lambda_bound(G.degf[u], G.degf[v], eps / 2, lam)
    tt = 2
    nr = np.zeros(2 * len(u), int)
    for h in range(2 * len(u)):
        i, j = int(G.hsrc[h]), int(G.hdst[h])
        length = int(tau[h % len(u)]) - tt
        if length > 0:
            q = tgt.column_at(G, i, tt)
            nr[h] = tgt.walk_count(tgt.chi_value(G, q, i, j, length, 10), G.degf[i], eps, len(u), delta)
    _, _, s = tgt.tgt_plus_replay(G, tau, np.full(n, tt), nr[: len(u)], nr[len(u):], seed=5)
    assert np.abs(s - ex.sc_pinv(n, u, v)).max() <= eps
