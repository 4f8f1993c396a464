"""Learned tail closure: features, certified bounds and targets, in float64.

TEST INFRASTRUCTURE: CPU oracle for the learned-closure form of the method.
The paper has no learned component; what is fixed by the paper is the series
structure this closure relies on:

* t_l(e) = sum_{k>=2} w_k lambda_k^l with w_k >= 0 (Eq. 18), hence the pair
  sums u_k = t_{2k} + t_{2k+1} = sum w (1 + lambda) lambda^{2k} are a
  non-negative mixture of geometric sequences in k.  A mixture of geometric
  sequences is log-convex, so r_k = u_k / u_{k-1} is non-decreasing and at
  most lambda*^2;
* therefore, truncating at the odd tau0 = 2K+1, the tail T = s - s_tau0 =
  sum_{k>K} u_k satisfies u_K r_K/(1-r_K) <= T <= u_K lambda*^2/(1-lambda*^2).

The closure predicts z = T / u_K with a small network and clamps it to that
interval, so the error of s_tau0 + u_K clamp(z) is at most u_K (hi - lo)
whatever the network does.  Edges whose interval is too wide for eps fall
back to the full truncated traversal.

Features (16 per edge, symmetric in the two endpoints), from the degrees and
p_l(i,i), p_l(j,j), p_l(j,i) for l = 0..8 (the first L0 = 8 steps):
  0: 1/d_i + 1/d_j            1: 1/(d_i d_j)
  2-4: r_1, r_2, r_3          5: t_8 / u_3
  6-8: m a_l, l = 6,7,8 with a_l = p_l(i,i)/d_i + p_l(j,j)/d_j (-> 1/m as l grows)
  9-11: m b_l, l = 6,7,8 with b_l = 2 p_l(j,i)/d_i (-> 1/m)
  12-14: t_1/t_0, t_2/t_0, t_3/t_0
  15: u_3 / t_0
"""
from __future__ import annotations

import numpy as np

L0 = 8          # traversal steps recorded
TAU0 = 7        # odd truncation the closure starts from (K = 3)
K = 3
NFEAT = 16


def _safe_div(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast(a, b).shape)
    np.divide(a, b, out=out, where=b != 0)
    return out


def edge_series(diag, off, deg, u, v):
    """Per edge: t[e, l] (Eq. 2 terms), a[e, l], b[e, l] for l = 0..L0 from the
    per-half recordings diag[h, l] = p_l(i,i), off[h, l] = p_l(j,i) (half h < m is
    (u_e -> v_e), h >= m is (v_e -> u_e))."""
    m = len(u)
    di = np.asarray(deg, np.float64)[u][:, None]
    dj = np.asarray(deg, np.float64)[v][:, None]
    a = diag[:m] / di + diag[m:] / dj
    b = 2.0 * off[:m] / di
    return a - b, a, b


def features(diag, off, deg, u, v, m_edges=None):
    m = len(u)
    mm = float(m if m_edges is None else m_edges)
    t, a, b = edge_series(diag, off, deg, u, v)
    di = np.asarray(deg, np.float64)[u]
    dj = np.asarray(deg, np.float64)[v]
    uk = t[:, 0:2 * K + 2:2] + t[:, 1:2 * K + 2:2]     # u_0..u_K
    F = np.empty((m, NFEAT))
    F[:, 0] = 1.0 / di + 1.0 / dj
    F[:, 1] = 1.0 / (di * dj)
    F[:, 2] = _safe_div(uk[:, 1], uk[:, 0])
    F[:, 3] = _safe_div(uk[:, 2], uk[:, 1])
    F[:, 4] = _safe_div(uk[:, 3], uk[:, 2])
    F[:, 5] = _safe_div(t[:, 8], uk[:, 3])
    F[:, 6:9] = mm * a[:, 6:9]
    F[:, 9:12] = mm * b[:, 6:9]
    F[:, 12:15] = t[:, 1:4] / t[:, 0:1]
    F[:, 15] = uk[:, 3] / t[:, 0]
    return F


def head_and_bounds(diag, off, deg, u, v, lam_star):
    """s_tau0, u_K and the interval [lo, hi] for z = tail / u_K."""
    t, _, _ = edge_series(diag, off, deg, u, v)
    s0 = t[:, : TAU0 + 1].sum(1)
    uK = t[:, 2 * K] + t[:, 2 * K + 1]
    uKm1 = t[:, 2 * K - 2] + t[:, 2 * K - 1]
    r = np.clip(_safe_div(uK, uKm1), 0.0, lam_star ** 2)
    lo = r / (1.0 - r)
    hi = np.full_like(lo, lam_star ** 2 / (1.0 - lam_star ** 2))
    return s0, uK, lo, hi


def target(s_ref, s0, uK):
    """z = (s_ref - s_tau0) / u_K (0 where u_K = 0)."""
    return _safe_div(s_ref - s0, uK)


def apply_closure(s0, uK, lo, hi, z):
    return s0 + uK * np.clip(z, lo, hi)


def certified_error(uK, lo, hi):
    """Worst-case error of any clamped prediction: u_K (hi - lo)."""
    return uK * (hi - lo)
