"""Pins for the learned-closure oracle (oracle.closure, oracle.mlp).

* the certified interval of the tail (log-convexity of the pair sums of the
  Eq. 18 series) against exact tails from the Laplacian pseudoinverse;
* feature symmetry under swapping the endpoints;
* all sixteen features equal to their closed forms on distance-regular graphs
  (K_n, odd C_n, Petersen), where the series terms follow from the spectrum
  alone, and a planted swap of two features fails that check;
* the network gradient against central finite differences, and the forward
  pass against a hand-built network with a closed-form output;
* Adam against its first-step closed form (the update is lr * sign(g)).
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import closure as cl
from oracle import exact as ex
from oracle import mlp
from oracle import tgt as otgt


def records(graph):
    n, u, v = graph
    G = otgt.Graph(n, u, v)
    _, _, diag, off = otgt.traversal(G, np.full(len(u), cl.L0), record=cl.L0)
    return G, diag, off


@pytest.mark.parametrize("graph", [gg.tree_plus_gnp(300, 6.0, 3), gg.barabasi_albert(400, 3, 5),
                                   gg.king_grid(200), gg.two_triangles_bridge()])
def test_tail_lies_in_certified_interval(graph):
    n, u, v = graph
    G, diag, off = records(graph)
    lam = ex.lambda_star(n, u, v)
    s = ex.sc_pinv(n, u, v)
    s0, uK, lo, hi = cl.head_and_bounds(diag, off, G.deg, u, v, lam)
    np.testing.assert_allclose(s0, ex.s_tau_eigen(n, u, v, cl.TAU0), atol=1e-13)
    tail = s - s0
    assert np.all(uK >= -1e-15)
    assert np.all(tail >= uK * lo - 1e-12)
    assert np.all(tail <= uK * hi + 1e-12)
    # any clamped prediction is within the certified error
    for z in (lo, hi, (lo + hi) / 2, np.zeros_like(lo), np.full_like(lo, 1e9)):
        est = cl.apply_closure(s0, uK, lo, hi, z)
        assert np.all(np.abs(est - s) <= cl.certified_error(uK, lo, hi) + 1e-12)


def test_features_symmetric_in_endpoints():
    graph = gg.barabasi_albert(300, 4, 2)
    n, u, v = graph
    G, diag, off = records(graph)
    m = len(u)
    F = cl.features(diag, off, G.deg, u, v)
    # swap orientation of every edge: halves exchange places
    sw = np.concatenate([np.arange(m, 2 * m), np.arange(m)])
    F2 = cl.features(diag[sw], off[sw], G.deg, v, u)
    np.testing.assert_allclose(F, F2, rtol=1e-12, atol=1e-15)
    assert F.shape == (m, cl.NFEAT) and np.all(np.isfinite(F))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(37, mlp.D_IN))
    z = rng.normal(size=37)
    th = mlp.init(1) + 0.01 * rng.normal(size=mlp.NPARAM)
    _, g = mlp.loss_and_grad(th, X, z)
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss_and_grad(th + e, X, z)[0] - mlp.loss_and_grad(th - e, X, z)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_mlp_forward_closed_form():
    # W1 = 0, b1 = c -> h1 = silu(c) everywhere; W2 = 0, b2 = c2; y = sum(W3) silu(c2) + b3
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["b1"][:] = 0.3
    p["b2"][:] = -1.2
    p["W3"][:] = 0.5
    p["b3"][:] = 2.0
    th = mlp.pack(p)
    y, _ = mlp.forward(th, np.random.default_rng(1).normal(size=(5, 16)))
    expect = 64 * 0.5 * (-1.2 / (1 + np.exp(1.2))) + 2.0
    np.testing.assert_allclose(y, expect, rtol=1e-14)
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.silu(np.array([40.0])), 40.0, rtol=1e-15)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -2e-3, 0.5])
    th = np.zeros(3)
    new, m1, m2 = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(new, -0.01 * np.sign(g), rtol=1e-12)
    assert mlp.NPARAM == 5313


# ---------------------------------------------------------------- closed-form features
#
# On a distance-regular graph (K_n, odd C_n, Petersen) every node sees the same
# spectrum: with the eigenvalues lambda_k of P and multiplicities mult_k,
# p_l(i,i) = (1/n) sum_k mult_k lambda_k^l, and since all neighbours of i are
# alike, p_l(j,i) = (1/d) sum_{x in N(i)} p_l(x,i) = p_{l+1}(i,i).  The series
# terms are then t_l = (2/d)(p_l(i,i) - p_{l+1}(i,i)) on every edge, with no
# traversal involved; the sixteen features follow from their definitions.

def _drg_spectrum(name, n):
    if name == "K":
        return np.array([1.0, -1.0 / (n - 1)]), np.array([1, n - 1]), n - 1
    if name == "C":
        lam = np.cos(2 * np.pi * np.arange(n) / n)
        return lam, np.ones(n), 2
    assert name == "Petersen"
    return np.array([1.0, 1.0 / 3.0, -2.0 / 3.0]), np.array([1, 5, 4]), 3


def _closed_form_features(name, n, m):
    lam, mult, d = _drg_spectrum(name, n)
    pii = np.array([(mult * lam ** ell).sum() / n for ell in range(cl.L0 + 2)])
    pji = pii[1:]
    t = 2.0 / d * (pii[:-1] - pji)                          # t_0 .. t_8
    u = np.array([t[2 * k] + t[2 * k + 1] for k in range(cl.K + 1)])
    F = np.empty(cl.NFEAT)
    F[0], F[1] = 2.0 / d, 1.0 / d ** 2
    F[2:5] = u[1:4] / u[0:3]
    F[5] = t[8] / u[3]
    F[6:9] = m * 2.0 * pii[6:9] / d
    F[9:12] = m * 2.0 * pji[6:9] / d
    F[12:15] = t[1:4] / t[0]
    F[15] = u[3] / t[0]
    return F


def _drg_graph(name, n):
    if name == "K":
        return gg.complete_graph(n)
    if name == "C":
        return gg.cycle_graph(n)
    return gg.petersen_graph()


DRG_CASES = [("K", 5), ("K", 8), ("C", 7), ("C", 11), ("Petersen", 10)]


def check_features_closed_form(features_fn):
    for name, n in DRG_CASES:
        graph = _drg_graph(name, n)
        G, diag, off = records(graph)
        _, u, v = graph
        F = features_fn(diag, off, G.deg, u, v)
        expect = _closed_form_features(name, n, len(u))
        # t_8 is a difference of two probabilities near 1/n that differ by
        # |lambda|^8 (7^-8 on K_8): the ratios keep ~1e-16 / |lambda|^8 relative rounding
        np.testing.assert_allclose(F, np.broadcast_to(expect, F.shape), rtol=1e-8, atol=1e-13,
                                   err_msg=f"{name}{n}")


def test_features_equal_closed_forms_on_distance_regular_graphs():
    check_features_closed_form(cl.features)


def test_complete_graph_features_by_hand():
    # K_n: lambda = -1/(n-1) (multiplicity n-1), d = n-1, m = n(n-1)/2, and
    # t_l = 2 lambda^l / d, so r_k = lambda^2, t_8/u_3 = lambda^2/(1+lambda),
    # m a_l = 1 + d lambda^l, m b_l = 1 - lambda^l, t_l/t_0 = lambda^l,
    # u_3/t_0 = lambda^6 (1 + lambda)
    n = 6
    lam, d = -1.0 / (n - 1), n - 1
    graph = gg.complete_graph(n)
    G, diag, off = records(graph)
    F = cl.features(diag, off, G.deg, graph[1], graph[2])
    expect = [2.0 / d, 1.0 / d ** 2, lam ** 2, lam ** 2, lam ** 2, lam ** 2 / (1 + lam),
              1 + d * lam ** 6, 1 + d * lam ** 7, 1 + d * lam ** 8,
              1 - lam ** 6, 1 - lam ** 7, 1 - lam ** 8,
              lam, lam ** 2, lam ** 3, lam ** 6 * (1 + lam)]
    np.testing.assert_allclose(F, np.broadcast_to(expect, F.shape), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("swap", [(2, 3), (3, 4), (6, 9), (12, 13), (5, 15)])
def test_planted_feature_swap_is_caught(swap):
    a, b = swap

    def swapped(*args, **kw):
        F = cl.features(*args, **kw)
        F[:, [a, b]] = F[:, [b, a]]
        return F

    with pytest.raises(AssertionError):
        check_features_closed_form(swapped)
