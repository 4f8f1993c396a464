"""Seeded generators for the graph families the method is evaluated on.

The paper evaluates on heavy-tailed social/collaboration graphs (its Table 3)
and on Erdos-Renyi graphs (its scalability tables).  Those files are not
available here; these generators produce synthetic stand-ins of the same
shape: Barabasi-Albert (heavy tail), G(n,p) with a spanning tree (ER-like),
2-D king grids (slow mixing) and R-MAT (skewed, large).

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64), which
is stable across platforms and numpy versions, so a (family, params, seed)
triple names one graph everywhere.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


# ---------------------------------------------------------------- utilities

def canonical_edges(n: int, u, v):
    """Drop self-loops and duplicates, orient u < v, sort by (u, v)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * np.int64(n) + b)
    return key // n, key % n


def degrees(n: int, u, v) -> np.ndarray:
    return np.bincount(np.asarray(u), minlength=n) + np.bincount(np.asarray(v), minlength=n)


def _adj(n, u, v):
    w = np.ones(len(u), dtype=np.int8)
    a = sp.coo_matrix((w, (u, v)), shape=(n, n))
    return (a + a.T).tocsr()


def is_connected(n: int, u, v) -> bool:
    if n <= 1:
        return True
    ncomp, _ = csg.connected_components(_adj(n, u, v), directed=False)
    return ncomp == 1


def is_bipartite(n: int, u, v) -> bool:
    """BFS 2-colouring from every component root; bipartite iff no edge joins equal colours."""
    a = _adj(n, u, v)
    colour = np.full(n, -1, dtype=np.int64)
    for root in range(n):
        if colour[root] >= 0:
            continue
        order, pred = csg.breadth_first_order(a, root, directed=False, return_predecessors=True)
        colour[root] = 0
        for x in order[1:]:
            colour[x] = 1 - colour[pred[x]]
    return bool(np.all(colour[np.asarray(u)] != colour[np.asarray(v)]))


def _largest_component(n, u, v):
    ncomp, lab = csg.connected_components(_adj(n, u, v), directed=False)
    if ncomp == 1:
        return n, u, v, np.arange(n)
    big = np.argmax(np.bincount(lab))
    nodes = np.flatnonzero(lab == big)
    remap = np.full(n, -1, dtype=np.int64)
    remap[nodes] = np.arange(len(nodes))
    keep = (lab[u] == big)
    return len(nodes), remap[u[keep]], remap[v[keep]], nodes


# ---------------------------------------------------------------- tiny named graphs

def complete_graph(n: int):
    i, j = np.triu_indices(n, 1)
    return n, i.astype(np.int64), j.astype(np.int64)


def cycle_graph(n: int):
    i = np.arange(n, dtype=np.int64)
    return (n,) + canonical_edges(n, i, (i + 1) % n)


def petersen_graph():
    outer = [(k, (k + 1) % 5) for k in range(5)]
    spokes = [(k, k + 5) for k in range(5)]
    inner = [(5 + k, 5 + (k + 2) % 5) for k in range(5)]
    e = np.array(outer + spokes + inner, dtype=np.int64)
    return (10,) + canonical_edges(10, e[:, 0], e[:, 1])


def triangle_pendant():
    """Triangle 0-1-2 with pendant vertex 3 hanging off 0 (edge 0-3 is a bridge)."""
    e = np.array([(0, 1), (1, 2), (0, 2), (0, 3)], dtype=np.int64)
    return (4,) + canonical_edges(4, e[:, 0], e[:, 1])


def two_triangles_bridge():
    """Triangles 0-1-2 and 3-4-5 joined by the bridge 2-3."""
    e = np.array([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)], dtype=np.int64)
    return (6,) + canonical_edges(6, e[:, 0], e[:, 1])


def random_small_connected(n: int, m: int, seed: int, max_tries: int = 1000):
    """Random simple connected non-bipartite graph with exactly m edges (m >= n)."""
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n, 1)
    for _ in range(max_tries):
        pick = rng.choice(len(i), size=m, replace=False)
        u, v = canonical_edges(n, i[pick], j[pick])
        if is_connected(n, u, v) and not is_bipartite(n, u, v):
            return n, u, v
    raise RuntimeError("no connected non-bipartite sample found")


# ---------------------------------------------------------------- workload families

def _random_tree(n, rng):
    """Uniform random recursive tree laid on a random permutation of the nodes."""
    perm = rng.permutation(n)
    k = np.arange(1, n)
    parent_pos = (rng.random(n - 1) * k).astype(np.int64)
    return perm[1:], perm[parent_pos]


def _gnp_pairs(n, p, rng):
    """G(n,p) edge set: Binomial(C(n,2), p) distinct uniform pairs."""
    total = n * (n - 1) // 2
    k = int(rng.binomial(total, p))
    return _distinct_pairs(n, k, rng)


def _distinct_pairs(n, k, rng):
    """k distinct node pairs (a < b) drawn uniformly from the C(n,2) pairs."""
    total = n * (n - 1) // 2
    if k == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    got = np.zeros(0, dtype=np.int64)
    while len(got) < k:
        draw = rng.integers(0, total, size=int((k - len(got)) * 1.1) + 16, dtype=np.int64)
        got = np.unique(np.concatenate([got, draw]))
    got = rng.permutation(got)[:k]
    # unrank pair index -> (a, b), a < b, row-major over the upper triangle
    # index(a, b) = a*n - a*(a+1)/2 + (b - a - 1)
    a = np.floor(((2 * n - 1) - np.sqrt((2.0 * n - 1) ** 2 - 8.0 * got)) / 2).astype(np.int64)
    a = np.clip(a, 0, n - 2)
    start = a * n - a * (a + 1) // 2
    # fix floating error in a
    over = got < start
    while np.any(over):
        a[over] -= 1
        start = a * n - a * (a + 1) // 2
        over = got < start
    nxt = (a + 1) * n - (a + 1) * (a + 2) // 2
    under = got >= nxt
    while np.any(under):
        a[under] += 1
        start = a * n - a * (a + 1) // 2
        nxt = (a + 1) * n - (a + 1) * (a + 2) // 2
        under = got >= nxt
    b = got - start + a + 1
    return a, b


def tree_plus_gnp(n: int, avg_deg: float, seed: int):
    """Random spanning tree union G(n,p) with p set so the expected edge count is avg_deg*n/2."""
    rng = np.random.default_rng(seed)
    tu, tv = _random_tree(n, rng)
    target_m = avg_deg * n / 2.0
    p = (target_m - (n - 1)) / (n * (n - 1) / 2.0)
    gu, gv = _gnp_pairs(n, p, rng)
    u, v = canonical_edges(n, np.concatenate([tu, gu]), np.concatenate([tv, gv]))
    return n, u, v


def gnp_connected(n: int, avg_deg: float, seed: int):
    """G(n,p) with p = avg_deg/(n-1); each non-giant component is linked to the
    giant one by one random edge."""
    rng = np.random.default_rng(seed)
    u, v = _gnp_pairs(n, avg_deg / (n - 1), rng)
    u, v = canonical_edges(n, u, v)
    ncomp, lab = csg.connected_components(_adj(n, u, v), directed=False)
    if ncomp > 1:
        big = np.argmax(np.bincount(lab))
        giant = np.flatnonzero(lab == big)
        extra_u, extra_v = [], []
        for c in range(ncomp):
            if c == big:
                continue
            members = np.flatnonzero(lab == c)
            extra_u.append(members[rng.integers(0, len(members))])
            extra_v.append(giant[rng.integers(0, len(giant))])
        u, v = canonical_edges(n, np.concatenate([u, extra_u]), np.concatenate([v, extra_v]))
    return n, u, v


def erdos_renyi_nm(n: int, m: int, seed: int):
    """Uniform G(n, m): m distinct pairs drawn uniformly.  Each component other
    than the giant one is joined to it by one random edge (so m grows by the
    number of such components, none at the densities used here)."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of node pairs")
    rng = np.random.default_rng(seed)
    u, v = _distinct_pairs(n, m, rng)
    u, v = canonical_edges(n, u, v)
    ncomp, lab = csg.connected_components(_adj(n, u, v), directed=False)
    if ncomp > 1:
        big = np.argmax(np.bincount(lab))
        giant = np.flatnonzero(lab == big)
        extra_u, extra_v = [], []
        for c in range(ncomp):
            if c == big:
                continue
            members = np.flatnonzero(lab == c)
            extra_u.append(members[rng.integers(0, len(members))])
            extra_v.append(giant[rng.integers(0, len(giant))])
        u, v = canonical_edges(n, np.concatenate([u, extra_u]), np.concatenate([v, extra_v]))
    return n, u, v


# Scalability series of Erdos-Renyi graphs: n fixed at 10^4 with m varied, and
# m fixed at 10^6 with n varied (the sizes of the paper's scalability tables).
ER_EDGES_SERIES = [(10_000, m) for m in (200_000, 500_000, 1_000_000, 2_000_000, 5_000_000)]
ER_NODES_SERIES = [(n, 1_000_000) for n in (2_000, 5_000, 10_000, 20_000, 50_000)]


def barabasi_albert(n: int, m_attach: int, seed: int, progress=None):
    """Preferential attachment: a seed clique on m_attach+1 nodes, then every new
    node joins m_attach distinct targets drawn with probability proportional to degree.
    ``progress`` (optional) is called with the number of nodes placed every 2^19 nodes."""
    rng = np.random.default_rng(seed)
    k0 = m_attach + 1
    ci, cj = np.triu_indices(k0, 1)
    m_total = len(ci) + (n - k0) * m_attach
    eu = np.empty(m_total, dtype=np.int64)
    ev = np.empty(m_total, dtype=np.int64)
    eu[: len(ci)] = ci
    ev[: len(ci)] = cj
    pool = np.empty(2 * m_total, dtype=np.int64)   # every edge endpoint once
    pool[0: 2 * len(ci): 2] = ci
    pool[1: 2 * len(ci): 2] = cj
    plen = 2 * len(ci)
    ecount = len(ci)
    batch = rng.random(4 * m_attach * (n - k0) + 64)
    bpos = 0
    for new in range(k0, n):
        if progress is not None and new % (1 << 19) == 0:
            progress(new)
        chosen = set()
        while len(chosen) < m_attach:
            if bpos >= len(batch):
                batch = rng.random(4 * m_attach * 1024)
                bpos = 0
            t = int(pool[int(batch[bpos] * plen)])
            bpos += 1
            chosen.add(t)
        for t in sorted(chosen):
            eu[ecount] = t
            ev[ecount] = new
            pool[plen] = t
            pool[plen + 1] = new
            plen += 2
            ecount += 1
    u, v = canonical_edges(n, eu, ev)
    return n, u, v


def king_grid(n: int):
    """Row-major r x c grid (r = floor(sqrt n), c = ceil(n/r)) truncated to n nodes,
    with horizontal, vertical and both diagonal edges."""
    r = int(np.floor(np.sqrt(n)))
    c = int(np.ceil(n / r))
    idx = np.arange(n, dtype=np.int64)
    row, col = idx // c, idx % c
    us, vs = [], []
    for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
        rr, cc = row + dr, col + dc
        ok = (cc >= 0) & (cc < c)
        tgt = rr * c + cc
        ok &= tgt < n
        us.append(idx[ok])
        vs.append(tgt[ok])
    u, v = canonical_edges(n, np.concatenate(us), np.concatenate(vs))
    return n, u, v


def rmat_lcc(scale: int, edge_factor: int, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 22):
    """R-MAT (no noise) with 2^scale nodes and edge_factor*2^scale generated edges;
    symmetrised, self-loops dropped, deduplicated; a seeded random relabelling is
    applied and the largest connected component is kept (relabelled 0..n-1)."""
    rng = np.random.default_rng(seed)
    nn = 1 << scale
    ne = edge_factor * nn
    a, b, c, _ = abcd
    u = np.zeros(ne, dtype=np.int64)
    v = np.zeros(ne, dtype=np.int64)
    chunk = 1 << 22
    for s in range(0, ne, chunk):
        e = min(ne, s + chunk)
        uu = np.zeros(e - s, dtype=np.int64)
        vv = np.zeros(e - s, dtype=np.int64)
        for lvl in range(scale):
            r = rng.random(e - s)
            bit = np.int64(1) << (scale - 1 - lvl)
            right = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            down = r >= a + b
            vv += np.where(right, bit, 0)
            uu += np.where(down, bit, 0)
        u[s:e] = uu
        v[s:e] = vv
    perm = rng.permutation(nn)
    u, v = canonical_edges(nn, perm[u], perm[v])
    n2, u2, v2, _ = _largest_component(nn, u, v)
    u2, v2 = canonical_edges(n2, u2, v2)
    return n2, u2, v2


# ---------------------------------------------------------------- named workloads

def mixed_batch(count: int, n_lo: int, n_hi: int, seed: int):
    """Many graphs of uneven size: n_k uniform in [n_lo, n_hi], family k mod 3 =
    G(n,p) with average degree 8 (components linked to the giant), Barabasi-Albert
    with 5 edges per new node, king grid.  Per-graph seeds come from the master seed."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    seeds = rng.integers(1, 2**31 - 1, size=count)
    out = []
    for k in range(count):
        n = int(sizes[k])
        fam = k % 3
        if fam == 0:
            out.append(gnp_connected(n, 8.0, int(seeds[k])))
        elif fam == 1:
            out.append(barabasi_albert(n, 5, int(seeds[k])))
        else:
            out.append(king_grid(n))
    return out


def workload(name: str, seed: int = 1):
    """The evaluation workloads, by name.

    * ``tree_gnp_1k``  : n=1,000, random spanning tree + G(n,p), average degree 10.
    * ``ba_100k``      : Barabasi-Albert, n=100,000, 10 edges per new node.
    * ``ba_small``     : Barabasi-Albert, n=2,000, 10 edges per new node (parity size).
    * ``rmat_s22``     : R-MAT scale 22, edge factor 16, LCC.
    * ``batch_256``    : 256 graphs, n uniform in [200, 20,000], G(n,p) deg 8 /
                         BA m = 5 / king grid in turn (a list of graphs).
    """
    if name == "tree_gnp_1k":
        return tree_plus_gnp(1000, 10.0, seed)
    if name == "ba_100k":
        return barabasi_albert(100_000, 10, seed)
    if name == "ba_small":
        return barabasi_albert(2_000, 10, seed)
    if name == "batch_256":
        return mixed_batch(256, 200, 20_000, seed)
    if name == "rmat_s22":
        return rmat_lcc(22, 16, seed=seed)
    raise KeyError(name)
