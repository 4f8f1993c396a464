"""The TGT / TGT+ method, step by step, on the CPU in float64.

TEST INFRASTRUCTURE: CPU oracle.  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  Nothing here is shared with the
GPU library; the two meet only through the paper and through the walk
definition stated below.

Notation (Table 1, Section 2.1): P = D^-1 A, p_l(x, i) = P^l[x, i].  The
traversal from source i propagates the column p_l(., i) = P p_{l-1}(., i)
(Algorithm 2 lines 6-9 and the proof of Theorem 3.3).

Half-edges: the input edge e = (u_e, v_e) has two halves, (i=u_e, j=v_e) and
(i=v_e, j=u_e).  Per-half results are returned as two arrays ``*_uv`` and
``*_vu`` aligned with the input edge order.

Walk definition (the part of TGT+ the paper leaves to the implementation,
Algorithm 4 lines 15-17):

* the walk pair number r of half-edge (i, j) consists of W_i from i (side 0)
  and W_j from j (side 1), each of L' = tau_ij - tilde_tau_i steps;
* step t (1-based) of side s draws word ((t-1) mod 4) of
  Philox4x32-10(counter = (i, j, r, s*2^31 + (t-1) div 4), key = seed split
  into (low 32 bits, high 32 bits));
* from node v the walk moves to its neighbour number floor(word * d(v) / 2^32)
  in ascending node-id order;
* W holds the L' nodes reached after steps 1..L' (the start node is not
  included: Eq. 10 sums l = 1..tau - tilde_tau, and in the proof of Lemma 4.3
  the first walk node is a neighbour of the start).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_10, seed_key, pick_index


# ------------------------------------------------------------------ graph helpers

class Graph:
    """Adjacency with neighbour lists in ascending id order, plus the half-edge table."""

    def __init__(self, n, u, v):
        self.n = int(n)
        self.u = np.asarray(u, dtype=np.int64)
        self.v = np.asarray(v, dtype=np.int64)
        self.m = len(self.u)
        w = np.ones(self.m)
        a = sp.coo_matrix((w, (self.u, self.v)), shape=(self.n, self.n))
        a = (a + a.T).tocsr()
        a.sort_indices()
        self.A = a
        self.indptr = a.indptr.astype(np.int64)
        self.nbr = a.indices.astype(np.int64)
        self.deg = np.diff(self.indptr)
        self.degf = self.deg.astype(np.float64)
        # P = D^-1 A
        self.P = sp.diags(1.0 / self.degf) @ a
        # half-edges: index h < m is (u_e -> v_e), h >= m is (v_e -> u_e)
        self.hsrc = np.concatenate([self.u, self.v])
        self.hdst = np.concatenate([self.v, self.u])
        order = np.argsort(self.hsrc, kind="stable")
        self.h_by_src = order
        self.h_ptr = np.concatenate([[0], np.cumsum(np.bincount(self.hsrc, minlength=self.n))])

    def halves_of(self, sources):
        """Half-edge ids whose source is in ``sources``."""
        parts = [self.h_by_src[self.h_ptr[s]: self.h_ptr[s + 1]] for s in sources]
        return np.concatenate(parts) if parts else np.zeros(0, np.int64)

    def adjacent(self, a, b):
        lo, hi = self.indptr[a], self.indptr[a + 1]
        k = np.searchsorted(self.nbr[lo:hi], b)
        return k < hi - lo and self.nbr[lo + k] == b


def as_graph(g_or_n, u=None, v=None):
    return g_or_n if isinstance(g_or_n, Graph) else Graph(g_or_n, u, v)


# ------------------------------------------------------------------ truncation lengths (Thm 3.2)

def odd_ceil(x):
    """Smallest odd integer >= x, and at least 1 (Eq. 5 requires tau odd)."""
    k = max(1, int(math.ceil(x)))
    return k if k % 2 == 1 else k + 1


def tau_uniform(L, m):
    """A fixed truncation L for every edge, rounded up to odd (Eq. 5 parity)."""
    return np.full(m, odd_ceil(L), dtype=np.int64)


def tau_lambda_bound(deg_i, deg_j, eps, lam_star):
    """Eq. 6 with Upsilon = Delta_t = 0 and lambda_omega -> lambda* (Algorithm 1
    line 1): the smallest odd tau with
    lambda*^(tau+1) / (1 - lambda*^2) * (1/d_i + 1/d_j - 2/(d_i d_j)) <= eps."""
    di = np.asarray(deg_i, dtype=np.float64)
    dj = np.asarray(deg_j, dtype=np.float64)
    num = 1.0 / di + 1.0 / dj - 2.0 / (di * dj)
    f = np.log(num / (eps * (1.0 - lam_star ** 2))) / np.log(1.0 / lam_star) - 1.0
    f = np.ceil(f)
    out = np.array([odd_ceil(x) for x in np.atleast_1d(f)], dtype=np.int64)
    return out


# ------------------------------------------------------------------ TGT traversal (Alg. 2)

def traversal(g, tau_edge, sources=None, chunk=512, record=None):
    """Truncated graph traversal of Algorithm 2 with a per-edge truncation.

    For each source i: p_0(., i) = e_i; g(i, j) starts at 1/d_i (the l = 0
    term, Algorithm 2 lines 2-3); for l = 1 .. max_j tau_ij the column is
    pushed one hop, p_l = P p_{l-1}, and every half-edge (i, j) with
    l <= tau_ij gains (p_l(i, i) - p_l(j, i)) / d_i (Eq. 9).  Both halves of
    an edge use the same tau_ij.

    Sources are processed ``chunk`` at a time as the columns of one matrix
    (the same per-column arithmetic).  ``record`` (an int L0) additionally
    returns, per half-edge, p_l(i,i) and p_l(j,i) for l = 0..L0.

    Returns g_uv, g_vu (per input edge; NaN for halves whose source was not
    traversed) and, with ``record``, arrays diag[h, l], off[h, l] indexed by
    half-edge id h (h < m: (u->v); h >= m: (v->u))."""
    g = as_graph(g)
    tau_edge = np.asarray(tau_edge, dtype=np.int64)
    tau_half = np.concatenate([tau_edge, tau_edge])
    if sources is None:
        sources = np.arange(g.n)
    sources = np.asarray(sources, dtype=np.int64)
    gh = np.full(2 * g.m, np.nan)
    if record is not None:
        diag = np.full((2 * g.m, record + 1), np.nan)
        off = np.full((2 * g.m, record + 1), np.nan)
    for s0 in range(0, len(sources), chunk):
        S = sources[s0: s0 + chunk]
        k = len(S)
        col_of = {int(s): c for c, s in enumerate(S)}
        H = g.halves_of(S)
        hi, hj = g.hsrc[H], g.hdst[H]
        hc = np.array([col_of[int(x)] for x in hi], dtype=np.int64)
        htau = tau_half[H]
        X = np.zeros((g.n, k))
        X[S, np.arange(k)] = 1.0                      # p_0(., i) = e_i
        acc = 1.0 / g.degf[hi]                        # l = 0 term
        if record is not None:
            diag[H, 0] = X[hi, hc]
            off[H, 0] = X[hj, hc]
        lmax = int(htau.max()) if len(H) else 0
        if record is not None:
            lmax = max(lmax, record)
        for ell in range(1, lmax + 1):
            X = g.P @ X                               # p_l = P p_{l-1}
            pii = X[hi, hc]
            pji = X[hj, hc]
            live = ell <= htau
            acc = acc + np.where(live, (pii - pji) / g.degf[hi], 0.0)
            if record is not None and ell <= record:
                diag[H, ell] = pii
                off[H, ell] = pji
        gh[H] = acc
    res = (gh[: g.m], gh[g.m:])
    if record is not None:
        return res + (diag, off)
    return res


def truncated_sc(g, tau_edge, **kw):
    """s_tau(e_ij) = g_tau(i, j) + g_tau(j, i) (Algorithm 2 line 12, Eq. 2)."""
    g_uv, g_vu = traversal(g, tau_edge, **kw)[:2]
    return g_uv + g_vu


def series_terms(diag, off, deg_src, deg_dst, m):
    """t_l(e) = p_l(i,i)/d_i + p_l(j,j)/d_j - 2 p_l(j,i)/d_i (Eq. 2 with the
    reversibility of Eq. 4), from the per-half recordings of ``traversal``."""
    di = deg_src[:m, None]
    dj = deg_dst[:m, None]
    return diag[:m] / di + diag[m:] / dj - 2.0 * off[:m] / di


# ------------------------------------------------------------------ TGT+ pieces (Section 4)

def column_at(g, source, ell):
    """p_ell(., source) as a dense float64 vector."""
    x = np.zeros(g.n)
    x[source] = 1.0
    for _ in range(ell):
        x = g.P @ x
    return x


def top_candidates(q, gamma):
    """C = the gamma nodes with the largest q, ordered by (value desc, id asc) (Algorithm 3 line 2)."""
    order = np.lexsort((np.arange(len(q)), -q))
    return order[: min(gamma, len(q))]


def rho_hat(g, q, gamma):
    """Upper bound on rho_i = max over edges (x, y) of q_x + q_y (Eq. 16).

    Algorithm 3 lines 2-5 with the safe reading: the best candidate-pair edge
    is combined with q[c_1] + q[c_gamma], which bounds every edge with an
    endpoint outside C.  (Taking the candidate-pair edge alone can fall below
    rho_i when the best edge has one endpoint outside C.)"""
    C = top_candidates(q, gamma)
    bound = q[C[0]] + q[C[-1]]
    in_c = np.zeros(g.n, dtype=bool)
    in_c[C] = True
    both = in_c[g.u] & in_c[g.v]          # the edges of C x C
    best = float(np.max(q[g.u[both]] + q[g.v[both]])) if both.any() else -np.inf
    return max(best, bound)


def rho_bruteforce(g, q):
    """rho_i of Eq. 16 by scanning every edge."""
    return float(np.max(q[g.u] + q[g.v]))


def walk_bounds(g, q, node, length, rho):
    """LB(node, length) and UB(node, length) of Lemma 4.3 for walks from ``node``
    scored with q = p_tilde_tau(., i)."""
    nq = q[g.nbr[g.indptr[node]: g.indptr[node + 1]]]
    lb = nq.min() + (length - 1) * q.min()
    ub = nq.max() / 2.0 + q.max() / 2.0 + (length - 1) * rho / 2.0
    return lb, ub


def chi_value(g, q, i, j, length, gamma, rho=None):
    """chi for half-edge (i, j) (Algorithm 3).

    gamma > 0: Eq. 17, UB(i)+UB(j)-LB(i)-LB(j) with rho_i replaced by its
    bound; gamma = 0: Eq. 15, 2 * length * (max q - min q).  For the walk from
    j the bounds use the same score vector q (the source is i)."""
    if gamma == 0:
        return 2.0 * length * (q.max() - q.min())
    if rho is None:
        rho = rho_hat(g, q, gamma)
    lbi, ubi = walk_bounds(g, q, i, length, rho)
    lbj, ubj = walk_bounds(g, q, j, length, rho)
    return ubi + ubj - lbi - lbj


NR_CAP = 2 ** 31 - 1   # walk pairs per half-edge are capped (a reading: counts fit 31 bits)


def walk_count(chi, deg_i, eps, m, delta):
    """n_r from Eq. 13: R = 8 chi^2 ln(2m/delta) / (d_i^2 eps^2), rounded up,
    at least one walk pair (the estimator needs one sample)."""
    r = 8.0 * chi ** 2 * math.log(2.0 * m / delta) / (deg_i ** 2 * eps ** 2)
    return max(1, int(math.ceil(r)))


def walks(g, i, j, r_ids, side, length, seed):
    """Node sequences of walks (see the module docstring); returns int array
    [len(r_ids), length]."""
    key = seed_key(seed)
    r_ids = np.asarray(r_ids, dtype=np.int64)
    start = i if side == 0 else j
    pos = np.full(len(r_ids), start, dtype=np.int64)
    out = np.empty((len(r_ids), length), dtype=np.int64)
    words = None
    for t in range(1, length + 1):
        if (t - 1) % 4 == 0:
            ctr = np.stack([np.full(len(r_ids), i), np.full(len(r_ids), j), r_ids,
                            np.full(len(r_ids), (side << 31) + (t - 1) // 4)], axis=-1)
            words = philox4x32_10(ctr, key)
        w = words[:, (t - 1) % 4]
        k = pick_index(w, g.deg[pos]).astype(np.int64)
        pos = g.nbr[g.indptr[pos] + k]
        out[:, t - 1] = pos
    return out


def estimator_samples(g, q, i, j, n_r, length, seed):
    """X_r of Eq. 11 for r = 0..n_r-1: (sum over W_i of q - sum over W_j of q) / d_i."""
    r = np.arange(n_r)
    wi = walks(g, i, j, r, 0, length, seed)
    wj = walks(g, i, j, r, 1, length, seed)
    return (q[wi].sum(1) - q[wj].sum(1)) / g.degf[i]


def tail_exact(g, q, i, j, length):
    """E[X] computed exactly: (1/d_i) sum_{l=1..length} sum_x (p_l(i,x) - p_l(j,x)) q[x],
    i.e. g_{tilde_tau -> tau}(i, j) of Eq. 10 (rows of P^l by repeated products)."""
    ri = np.zeros(g.n)
    ri[i] = 1.0
    rj = np.zeros(g.n)
    rj[j] = 1.0
    tot = 0.0
    PT = g.P.T.tocsr()
    for _ in range(length):
        ri = PT @ ri          # row vector e_i^T P^l, stored as a column
        rj = PT @ rj
        tot += (ri - rj) @ q
    return tot / g.degf[i]


def tgt_plus_replay(g, tau_edge, tilde_tau, nr_uv, nr_vu, seed, sources=None):
    """Algorithm 4 with tilde_tau (per source) and n_r (per half-edge) given.

    For each source i: traverse to tilde_tau_i collecting g_{tilde_tau} (Alg. 2
    with every half truncated at min(tilde_tau_i, tau_ij)), keep
    q = p_{tilde_tau_i}(., i); for every half (i, j) with
    L' = tau_ij - tilde_tau_i > 0 add the mean of n_r samples of X (Eq. 11).
    Returns g_uv, g_vu and s = g_uv + g_vu (Algorithm 4 line 18).  With
    ``sources`` only those sources' halves are computed (others are NaN)."""
    g = as_graph(g)
    tau_edge = np.asarray(tau_edge, dtype=np.int64)
    tilde_tau = np.asarray(tilde_tau, dtype=np.int64)
    nr = np.concatenate([np.asarray(nr_uv, np.int64), np.asarray(nr_vu, np.int64)])
    tau_half = np.concatenate([tau_edge, tau_edge])
    gh = np.full(2 * g.m, np.nan)
    src = range(g.n) if sources is None else [int(x) for x in sources]
    for i in src:
        H = g.halves_of([i])
        if len(H) == 0:
            continue
        tt = int(tilde_tau[i])
        x = np.zeros(g.n)
        x[i] = 1.0
        acc = np.full(len(H), 1.0 / g.degf[i])
        hj = g.hdst[H]
        for ell in range(1, tt + 1):
            x = g.P @ x
            live = ell <= tau_half[H]
            acc += np.where(live, (x[i] - x[hj]) / g.degf[i], 0.0)
        for k, h in enumerate(H):
            length = int(tau_half[h]) - tt
            if length > 0:
                xs = estimator_samples(g, x, i, int(hj[k]), int(nr[h]), length, seed)
                acc[k] += xs.mean()
        gh[H] = acc
    return gh[: g.m], gh[g.m:], gh[: g.m] + gh[g.m:]


# ------------------------------------------------------------------ per-source switch (Eq. 14)

def switch_step(g, i, tau_half_i, eps, delta, gamma, rule=0, trace=None):
    """Algorithm 4 lines 3-11 for source i with the adaptive switch of Section
    4.2.1: starting at l = 0 with p_0(., i) = e_i, stop at the first l where
    Eq. 14 holds,

        sum of d(v) over the nodes with p_l(v, i) != 0
            >  sum over the halves (i, j) of R(e_ij, tau_ij - l),

    R from Eq. 13 with chi from Algorithm 3 at q = p_l(., i) (n_r = 0 where
    tau_ij - l <= 0, so the loop also ends at l = max_j tau_ij); otherwise push
    one step and continue.  rule = 1 weighs each walk pair by its
    2 (tau_ij - l) single-walk steps (the right-hand side then counts walk
    steps, not walk pairs).  ``tau_half_i`` lists tau_ij over the halves of i in
    the order of ``g.halves_of([i])``.  Returns (tilde_tau, n_r per half of i);
    ``trace`` (a list) receives (l, left side, right side) per test."""
    g = as_graph(g)
    H = g.halves_of([i])
    hj = g.hdst[H]
    tau_h = np.asarray(tau_half_i, dtype=np.int64)
    x = np.zeros(g.n)
    x[i] = 1.0
    ell = 0
    while True:
        lhs = float(g.degf[x != 0].sum())
        nr = np.zeros(len(H), dtype=np.int64)
        live = tau_h - ell > 0
        if live.any():
            rho = rho_hat(g, x, gamma) if gamma > 0 else None
            for k in np.nonzero(live)[0]:
                length = int(tau_h[k] - ell)
                chi = chi_value(g, x, i, int(hj[k]), length, gamma, rho)
                nr[k] = min(walk_count(chi, g.degf[i], eps, g.m, delta), NR_CAP)
        rhs = float(nr.sum()) if rule == 0 else float((2 * nr * np.maximum(tau_h - ell, 0)).sum())
        if trace is not None:
            trace.append((ell, lhs, rhs))
        if lhs > rhs:
            return ell, nr
        x = g.P @ x
        ell += 1


def tgt_plus_adaptive(g, tau_edge, eps, delta, gamma, seed, rule=0, sources=None):
    """Algorithm 4 with a switch step per source by Eq. 14 (``switch_step``):
    the decisions (tilde_tau per source, n_r per half-edge) are taken first and
    the estimate is then ``tgt_plus_replay`` with them.  Returns
    (s, tilde_tau[n], nr_uv, nr_vu) with -1 / 0 for sources not computed."""
    g = as_graph(g)
    tau_edge = np.asarray(tau_edge, dtype=np.int64)
    tau_half = np.concatenate([tau_edge, tau_edge])
    tilde = np.full(g.n, -1, dtype=np.int64)
    nr = np.zeros(2 * g.m, dtype=np.int64)
    src = range(g.n) if sources is None else [int(x) for x in sources]
    for i in src:
        H = g.halves_of([i])
        if len(H) == 0:
            continue
        tilde[i], nr[H] = switch_step(g, i, tau_half[H], eps, delta, gamma, rule)
    tt = np.where(tilde < 0, 0, tilde)
    _, _, s = tgt_plus_replay(g, tau_edge, tt, nr[: g.m], nr[g.m:], seed, sources=sources)
    return s, tilde, nr[: g.m], nr[g.m:]
