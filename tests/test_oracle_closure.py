"""Pins for the learned-closure oracle (oracle.closure, oracle.mlp).

* the certified interval of the tail (log-convexity of the pair sums of the
  Eq. 18 series) against exact tails from the Laplacian pseudoinverse;
* feature symmetry under swapping the endpoints;
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
