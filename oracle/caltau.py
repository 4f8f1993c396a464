"""CalTau (Algorithm 1): per-edge truncation lengths from the omega eigenpairs
of N = D^-1/2 A D^-1/2 of largest |lambda| (Theorem 3.2, Eq. 6-8).

TEST INFRASTRUCTURE: CPU oracle.  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  Nothing here is shared with the
GPU library.

Notation (Section 3.1): eigenpairs (lambda_k, phi_k) of N sorted by |lambda|
descending, lambda_1 = 1 with phi_1 = sqrt(d / 2m); f_k = sqrt(2m) D^-1/2 phi_k
(Lemma 3.1), so (1/2m)(f_k[i] - f_k[j])^2 = (phi_k[i]/sqrt(d_i) - phi_k[j]/sqrt(d_j))^2
=: w_k.  For an edge (i, j):

* Eq. 7:  Upsilon  = sum_{k=2}^{omega-1} w_k (1 + lambda_k)
* Eq. 8:  Delta_t  = sum_{k=2}^{omega-1} w_k lambda_k^(t+1) / (1 - lambda_k)
* Eq. 6:  f = ceil( log( (1/d_i + 1/d_j - 2/(d_i d_j) - Upsilon)
                         / ((eps - Delta_t)(1 - lambda_omega^2)) ) / log(1/|lambda_omega|) - 1 )

Readings (the paper leaves these open):

* Eq. 6 is +infinity when eps <= Delta_t (no t that small can be certified),
  and -infinity when the numerator is <= 0 (the uncaptured eigenpairs carry
  no weight on this edge);
* Algorithm 1 needs omega >= 2 (lambda_omega = lambda_1 = 1 would make the
  logarithm zero); with omega = 2 the sums are empty and lambda_omega is the
  largest non-trivial |lambda| (lambda* of the lambda*-bound);
* the loop is followed as printed: while the current odd t satisfies
  t <= f(Delta_t), t grows by 2; the first t that exceeds f(Delta_t) is
  returned (when t equals f exactly, the printed loop still steps once more).
"""
from __future__ import annotations

import math

import numpy as np

from . import exact


def top_spectrum(n, u, v, omega):
    """The omega eigenpairs of N with largest |lambda| (dense eigensolver),
    lambda_1 = 1 first, then by |lambda| descending (ties by lambda descending).
    Returns lam[omega] and phi[n, omega] (columns are eigenvectors)."""
    lam, phi, _ = exact.spectral(n, u, v)   # descending; lam[0] = 1
    rest = 1 + np.lexsort((-lam[1:], -np.abs(lam[1:])))
    order = np.concatenate([[0], rest])[: min(omega, n)]
    return lam[order], phi[:, order]


def eq6(numerator, eps, delta, lam_omega):
    """Eq. 6 before the ceiling: log(numerator / ((eps - delta)(1 - lam^2))) / log(1/|lam|) - 1,
    with +inf when eps <= delta and -inf when numerator <= 0."""
    if eps - delta <= 0.0:
        return math.inf
    if numerator <= 0.0:
        return -math.inf
    a = abs(lam_omega)
    return math.log(numerator / ((eps - delta) * (1.0 - a * a))) / math.log(1.0 / a) - 1.0


def caltau_edge(d_i, d_j, phi_i, phi_j, lam, eps, t_max=1 << 20, margins=None):
    """Algorithm 1 for the edge (i, j): d_i, d_j degrees, phi_i, phi_j the rows
    of the eigenvector matrix at i and j, lam the omega eigenvalues (index 0 is
    the trivial pair).  Returns tau_ij.  If ``margins`` is a list, the distance
    of every evaluated Eq. 6 value to the nearest integer is appended to it
    (the GPU, summing in another order, may round such a case differently)."""
    omega = len(lam)
    if omega < 2:
        raise ValueError("CalTau needs omega >= 2")
    di, dj = float(d_i), float(d_j)
    num = 1.0 / di + 1.0 / dj - 2.0 / (di * dj)
    lam = np.asarray(lam, dtype=np.float64)
    # line 1: Eq. 6 with lambda_2 and Delta = Upsilon = 0 (overwritten by the loop)
    x1 = eq6(num, eps, 0.0, lam[1])
    tau = math.ceil(x1) if math.isfinite(x1) else x1
    k = slice(1, omega - 1)   # eigenpairs 2 .. omega-1 (1-based)
    w = (np.asarray(phi_i)[k] / math.sqrt(di) - np.asarray(phi_j)[k] / math.sqrt(dj)) ** 2
    lk = lam[k]
    ups = float(np.sum(w * (1.0 + lk)))   # line 2, Eq. 7
    lam_omega = lam[omega - 1]
    t = 1
    while True:
        delta = float(np.sum(w * lk ** (t + 1) / (1.0 - lk)))   # line 4, Eq. 8
        x = eq6(num - ups, eps, delta, lam_omega)                # line 4, Eq. 6
        if margins is not None and math.isfinite(x):
            margins.append(abs(x - round(x)))
        tp = math.ceil(x) if math.isfinite(x) else x
        if t <= tp:                                              # line 5
            tau = tp
            t += 2
            if t > t_max:
                raise RuntimeError("CalTau did not terminate below t_max")
        else:                                                    # line 6
            break
    return t                                                     # line 7


def caltau(n, u, v, eps, lam, phi, max_L=None, margins=None):
    """tau_ij of every edge (u_e, v_e) by Algorithm 1 with the given eigenpairs
    (phi[n, omega]); capped at the odd max_L when given.  ``margins`` (a list)
    receives, per edge, the smallest distance of an evaluated Eq. 6 value to an
    integer."""
    u = np.asarray(u)
    v = np.asarray(v)
    d = exact.degree_vector(n, u, v)
    out = np.empty(len(u), dtype=np.int64)
    for e in range(len(u)):
        mg = [] if margins is not None else None
        t = caltau_edge(d[u[e]], d[v[e]], phi[u[e]], phi[v[e]], lam, eps, margins=mg)
        if max_L is not None:
            cap = max_L if max_L % 2 == 1 else max_L - 1
            t = min(t, cap)
        out[e] = t
        if margins is not None:
            margins.append(min(mg) if mg else math.inf)
    return out
