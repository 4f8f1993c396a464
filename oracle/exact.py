"""Exact spanning centrality: the plain definitions the method approximates.

TEST INFRASTRUCTURE: this module is the CPU oracle.  Only tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library
never calls it.  Everything is float64.

Graphs are ``(n, u, v)`` with int edge arrays (simple, undirected).  Results
are per input edge, in input order.

Definitions followed:

* spanning centrality s(e) = fraction of spanning trees containing e
  (Definition 2.1);
* s(e_ij) equals the effective resistance
  r(i,j) = L+[i,i] + L+[j,j] - 2 L+[i,j], with L = D - A and L+ its
  pseudoinverse (Section 2.3; Section 6);
* spectral form (Lemma 3.1, Eq. 4, and Eq. 18 in the proof of Theorem 3.2):
  with N = D^-1/2 A D^-1/2 = sum_k lambda_k phi_k phi_k^T, the l-th series
  term of edge (i,j) is sum_{k>=2} w_k lambda_k^l where
  w_k = (phi_k[i]/sqrt(d_i) - phi_k[j]/sqrt(d_j))^2.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _as_graph(n, u, v):
    return int(n), np.asarray(u, dtype=np.int64), np.asarray(v, dtype=np.int64)


def degree_vector(n, u, v):
    n, u, v = _as_graph(n, u, v)
    return (np.bincount(u, minlength=n) + np.bincount(v, minlength=n)).astype(np.float64)


def adjacency_dense(n, u, v):
    n, u, v = _as_graph(n, u, v)
    a = np.zeros((n, n))
    a[u, v] = 1.0
    a[v, u] = 1.0
    return a


def adjacency_sparse(n, u, v):
    n, u, v = _as_graph(n, u, v)
    w = np.ones(len(u))
    a = sp.coo_matrix((w, (u, v)), shape=(n, n))
    return (a + a.T).tocsr()


# ------------------------------------------------------------------ Definition 2.1

def sc_kirchhoff(n, u, v):
    """Spanning centrality by enumerating every spanning tree (Definition 2.1).

    Every (n-1)-subset of the edges is tested with union-find; the count of
    trees containing each edge is divided by the number of trees.  Tiny graphs
    only (the enumeration is C(m, n-1))."""
    n, u, v = _as_graph(n, u, v)
    m = len(u)
    if m > 24:
        raise ValueError("enumeration is for tiny graphs only")
    hits = np.zeros(m, dtype=np.int64)
    trees = 0
    for subset in itertools.combinations(range(m), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        ok = True
        for e in subset:
            a, b = find(int(u[e])), find(int(v[e]))
            if a == b:
                ok = False
                break
            parent[a] = b
        if ok:
            trees += 1
            for e in subset:
                hits[e] += 1
    return hits / trees, trees


def reduced_laplacian_det(n, u, v):
    """det of the Laplacian with row/column 0 removed: the number of spanning
    trees by the matrix-tree theorem (cited in Section 1)."""
    a = adjacency_dense(n, u, v)
    lap = np.diag(a.sum(1)) - a
    return float(np.linalg.det(lap[1:, 1:]))


# ------------------------------------------------------------------ Section 2.3 / 6: L+

def sc_pinv(n, u, v):
    """Effective resistance of every edge from the Laplacian pseudoinverse.

    For a connected graph L + J/n is symmetric positive definite and its
    inverse is L+ + J/n; the J/n part cancels in L+ii + L+jj - 2 L+ij, so the
    Cholesky inverse of L + J/n is used directly."""
    n, u, v = _as_graph(n, u, v)
    a = adjacency_dense(n, u, v)
    lap = np.diag(a.sum(1)) - a
    mat = lap + np.full((n, n), 1.0 / n)
    c = sla.cho_factor(mat, lower=True)
    minv = sla.cho_solve(c, np.eye(n))
    return minv[u, u] + minv[v, v] - 2.0 * minv[u, v]


# ------------------------------------------------------------------ Lemma 3.1 spectral forms

def spectral(n, u, v):
    """Eigenpairs of N = D^-1/2 A D^-1/2 (the symmetric matrix similar to P),
    eigenvalues in descending order."""
    a = adjacency_dense(n, u, v)
    d = a.sum(1)
    s = 1.0 / np.sqrt(d)
    lam, phi = np.linalg.eigh(s[:, None] * a * s[None, :])
    order = np.argsort(-lam)
    return lam[order], phi[:, order], d


def edge_weights(n, u, v, lam=None, phi=None, d=None):
    """w[e, k] = (phi_k[i]/sqrt(d_i) - phi_k[j]/sqrt(d_j))^2 for k >= 2 (Eq. 18 with f_k = sqrt(2m) D^-1/2 phi_k)."""
    n, u, v = _as_graph(n, u, v)
    if lam is None:
        lam, phi, d = spectral(n, u, v)
    g = phi / np.sqrt(d)[:, None]
    w = (g[u, 1:] - g[v, 1:]) ** 2
    return w, lam[1:]


def sc_eigen(n, u, v):
    """s(e) = sum_{k>=2} w_k / (1 - lambda_k): the full series of Eq. 18 summed."""
    w, lam = edge_weights(n, u, v)
    return w @ (1.0 / (1.0 - lam))


def s_tau_eigen(n, u, v, tau):
    """Truncated series s_tau(e) = sum_{l=0..tau} t_l(e) in closed form:
    sum_{k>=2} w_k (1 - lambda_k^(tau+1)) / (1 - lambda_k)."""
    w, lam = edge_weights(n, u, v)
    tau = np.asarray(tau)
    if tau.ndim == 0:
        return w @ ((1.0 - lam ** (int(tau) + 1)) / (1.0 - lam))
    out = np.empty(len(w))
    for e in range(len(w)):
        out[e] = w[e] @ ((1.0 - lam ** (int(tau[e]) + 1)) / (1.0 - lam))
    return out


def series_term_eigen(n, u, v, ell):
    """t_l(e) = sum_{k>=2} w_k lambda_k^l (Eq. 18)."""
    w, lam = edge_weights(n, u, v)
    return w @ (lam ** int(ell))


def lambda_star(n, u, v):
    """max_{k>=2} |lambda_k| of D^-1/2 A D^-1/2 (dense eigensolver)."""
    lam, _, _ = spectral(n, u, v)
    return float(np.max(np.abs(lam[1:])))


def trace_p_power(n, u, v, k):
    """tr(P^k) = sum_k lambda^k over the spectrum of D^-1/2 A D^-1/2 (similar to P)."""
    lam, _, _ = spectral(n, u, v)
    return float(np.sum(lam ** int(k)))


# ------------------------------------------------------------------ sampled exact ER (large graphs)

def _laplacian_apply(lap, spmm):
    """y = L x for a block x: scipy's sparse product, or PyTorch's CPU CSR
    product (a library matmul that uses every host core) for large graphs."""
    if spmm == "scipy":
        return lambda x: lap @ x
    import torch
    t = torch.sparse_csr_tensor(torch.from_numpy(lap.indptr.astype(np.int64)),
                                torch.from_numpy(lap.indices.astype(np.int64)),
                                torch.from_numpy(lap.data.astype(np.float64)), size=lap.shape)
    return lambda x: (t @ torch.from_numpy(np.ascontiguousarray(x))).numpy()


def sc_sampled_pcg(n, u, v, edge_ids, tol=1e-12, max_iter=5000, block=256, spmm="scipy"):
    """Effective resistance of selected edges by Jacobi-preconditioned block CG.

    Solves L x = e_i - e_j (consistent: the right-hand side sums to zero) for
    each selected edge and returns r = x_i - x_j.  Residuals stay orthogonal to
    the all-ones null vector, so CG on the semidefinite system converges; the
    constant component of x is irrelevant to x_i - x_j.  Convergence is checked on the true residual
    ||L x - b|| <= tol * ||b||.  Used where a dense L+ does not fit."""
    n, u, v = _as_graph(n, u, v)
    a = adjacency_sparse(n, u, v)
    d = np.asarray(a.sum(1)).ravel()
    lap = (sp.diags(d) - a).tocsr()
    apply = _laplacian_apply(lap, spmm)
    edge_ids = np.asarray(edge_ids, dtype=np.int64)
    out = np.empty(len(edge_ids))
    dinv = 1.0 / d
    for s in range(0, len(edge_ids), block):
        ids = edge_ids[s: s + block]
        k = len(ids)
        b = np.zeros((n, k))
        b[u[ids], np.arange(k)] = 1.0
        b[v[ids], np.arange(k)] = -1.0
        x = np.zeros((n, k))
        r = b.copy()
        z = dinv[:, None] * r
        p = z.copy()
        rz = np.einsum("ij,ij->j", r, z)
        bnorm = np.linalg.norm(b, axis=0)
        for _ in range(max_iter):
            ap = apply(p)
            pap = np.einsum("ij,ij->j", p, ap)
            alpha = np.where(pap > 0, rz / np.where(pap > 0, pap, 1.0), 0.0)
            x += alpha * p
            r -= alpha * ap
            if np.all(np.linalg.norm(r, axis=0) <= tol * bnorm):
                true_r = b - apply(x)
                if np.all(np.linalg.norm(true_r, axis=0) <= 10 * tol * bnorm):
                    break
            z = dinv[:, None] * r
            rz_new = np.einsum("ij,ij->j", r, z)
            beta = np.where(rz > 0, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
            p = z + beta * p
            rz = rz_new
        else:
            raise RuntimeError("block PCG did not converge")
        out[s: s + k] = x[u[ids], np.arange(k)] - x[v[ids], np.arange(k)]
    return out
