"""Pins of the CalTau oracle (Algorithm 1, Theorem 3.2, Eq. 6-8).

* the guarantee of Theorem 3.2: with the returned tau, the truncated series
  (the oracle's traversal, i.e. matrix powers) is within eps of the exact SC
  (Laplacian pseudoinverse), for several omega including omega = n;
* Eq. 19: sum over k >= 2 of w_k (1 + lambda_k) equals 1/d_i + 1/d_j - 2/(d_i d_j),
  which fixes the scaling of w_k (f_k = sqrt(2m) D^-1/2 phi_k);
* omega = 2 reduces to the lambda*-bound (Algorithm 1 line 1), up to the
  printed loop's extra step when Eq. 6 is an odd integer;
* Eq. 6 special cases, monotonicity in eps, and the size of the gain on a
  slow-mixing king grid.
"""
import math

import numpy as np
import pytest

import graphgen as gg
from oracle import caltau as ct
from oracle import exact as ex
from oracle import tgt as otgt

GRAPHS = {
    "tree_gnp": gg.tree_plus_gnp(120, 6.0, 3),
    "ba": gg.barabasi_albert(150, 3, 2),
    "king": gg.king_grid(225),
    "small": gg.random_small_connected(30, 60, 4),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("omega", [2, 6, 24, None])
@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_theorem_3_2_guarantee(name, omega, eps):
    n, u, v = GRAPHS[name]
    lam, phi = ct.top_spectrum(n, u, v, n if omega is None else omega)
    tau = ct.caltau(n, u, v, eps, lam, phi)
    assert np.all(tau % 2 == 1) and tau.min() >= 1
    s_tau = otgt.truncated_sc(otgt.Graph(n, u, v), tau)
    assert np.abs(ex.sc_pinv(n, u, v) - s_tau).max() <= eps + 1e-12


@pytest.mark.parametrize("name", list(GRAPHS))
def test_eq19_weight_identity(name):
    n, u, v = GRAPHS[name]
    lam, phi = ct.top_spectrum(n, u, v, n)
    d = ex.degree_vector(n, u, v)
    w = (phi[u, 1:] / np.sqrt(d[u])[:, None] - phi[v, 1:] / np.sqrt(d[v])[:, None]) ** 2
    lhs = w @ (1.0 + lam[1:])
    rhs = 1.0 / d[u] + 1.0 / d[v] - 2.0 / (d[u] * d[v])
    np.testing.assert_allclose(lhs, rhs, atol=1e-12, rtol=0)
    # the trivial pair carries no weight: phi_1 / sqrt(d) is constant
    assert abs(lam[0] - 1.0) < 1e-12
    np.testing.assert_allclose(np.abs(phi[:, 0]), np.sqrt(d / d.sum()), atol=1e-12)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-5])
def test_omega_2_is_the_lambda_star_bound(name, eps):
    n, u, v = GRAPHS[name]
    lam, phi = ct.top_spectrum(n, u, v, 2)
    d = ex.degree_vector(n, u, v)
    lam_star = ex.lambda_star(n, u, v)
    assert abs(abs(lam[1]) - lam_star) < 1e-12
    tau = ct.caltau(n, u, v, eps, lam, phi)
    base = otgt.tau_lambda_bound(d[u], d[v], eps, lam_star)
    num = 1.0 / d[u] + 1.0 / d[v] - 2.0 / (d[u] * d[v])
    x = np.log(num / (eps * (1 - lam_star ** 2))) / np.log(1 / lam_star) - 1
    c = np.ceil(x)
    extra = np.where((c >= 1) & (c % 2 == 1), 2, 0)   # t == f: the printed loop steps once more
    np.testing.assert_array_equal(tau, base + extra)


def test_eq6_special_cases():
    assert ct.eq6(0.1, 1e-3, 1e-3, 0.5) == math.inf
    assert ct.eq6(0.1, 1e-3, 2e-3, 0.5) == math.inf
    assert ct.eq6(0.0, 1e-3, 0.0, 0.5) == -math.inf
    assert ct.eq6(-1e-18, 1e-3, 0.0, 0.5) == -math.inf
    # lambda^(x+1) (1/(1-lambda^2)) num = eps at the returned x
    x = ct.eq6(0.2, 1e-3, 0.0, 0.5)
    assert abs(0.5 ** (x + 1) * 0.2 / (1 - 0.25) - 1e-3) < 1e-15
    with pytest.raises(ValueError):
        ct.caltau_edge(3, 3, np.ones(1), np.ones(1), np.ones(1), 1e-2)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_smaller_eps_never_shortens(name):
    n, u, v = GRAPHS[name]
    lam, phi = ct.top_spectrum(n, u, v, 12)
    prev = None
    for eps in (1e-1, 1e-2, 1e-3, 1e-4):
        tau = ct.caltau(n, u, v, eps, lam, phi)
        if prev is not None:
            assert np.all(tau >= prev)
        prev = tau


def test_king_grid_gain():
    # lambda* is close to 1 on grids; the captured eigenpairs carry the slow modes
    n, u, v = GRAPHS["king"]
    d = ex.degree_vector(n, u, v)
    lam_star = ex.lambda_star(n, u, v)
    base = otgt.tau_lambda_bound(d[u], d[v], 1e-2, lam_star)
    lam, phi = ct.top_spectrum(n, u, v, 24)
    tau = ct.caltau(n, u, v, 1e-2, lam, phi)
    assert tau.mean() * 10 < base.mean()


def test_max_L_cap_and_margins():
    n, u, v = GRAPHS["king"]
    lam, phi = ct.top_spectrum(n, u, v, 6)
    margins = []
    tau = ct.caltau(n, u, v, 1e-3, lam, phi, max_L=30, margins=margins)
    assert tau.max() <= 29 and len(margins) == len(u)
    assert all(mg >= 0 for mg in margins)
