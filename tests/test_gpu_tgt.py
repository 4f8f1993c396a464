"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

* TGT (Algorithm 2) against the oracle's truncated traversal, element by
  element, FP64 to 1e-12 and FP32 to 2e-5 (FP32 rounding of probabilities
  that are summed over at most L+1 steps; every term is below 1);
* the GPU's truncation lengths against the lambda*-bound of Theorem 3.2;
* TGT+ (Algorithm 4) against the oracle's replay with the GPU's recorded
  tilde_tau and n_r: the walks are the same Philox walks, so only rounding
  differs; the GPU's n_r against the oracle's own chi / Eq. 13;
* accuracy against the exact SC (Laplacian pseudoinverse) within eps;
* edge cases: tiny graphs, partial blocks, rows split into chunks, all block
  widths, tilde_tau of 0 and 1, gamma = 0, duplicates, device pointers,
  determinism and error paths; source blocks skipped for having nothing to
  traverse; 2, 3, 4 and 7 blocks around the three-deep block pipeline.
"""
import math

import numpy as np
import pytest

import graphgen as gg
from oracle import exact as ex
from oracle import tgt as otgt

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-5


@pytest.fixture(scope="module")
def sc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_16086_amd import sc as scmod
    return scmod


def run(sc, graph, eps, L, flags=0, **opt):
    n, u, v = graph
    print(f"[gpu] n={n} m={len(u)} eps={eps} L={L} opt={opt}", flush=True)
    g = sc.sc_build_graph(n, u, v, flags)
    o = sc.sc_default_options(**opt)
    tau = np.empty(g.m, np.int32)
    tt = np.empty(n, np.int32)
    nr = np.empty(2 * g.m, np.int64)
    out, st = sc.sc_all_edges_ex(g, eps, L, o, tau_out=tau, tilde_tau_out=tt, nr_out=nr)
    g.free()
    return out, st, tau, tt, nr


# ------------------------------------------------------------------ TGT

@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("precision", [1, 0])
def test_tgt_tree_gnp_1k_auto_L(sc, seed, precision):
    graph = gg.workload("tree_gnp_1k", seed)
    n, u, v = graph
    eps = 1e-2
    out, st, tau, _, _ = run(sc, graph, eps, 0, method=sc.SC_TGT, precision=precision)
    G = otgt.Graph(n, u, v)
    lam = ex.lambda_star(n, u, v)
    assert lam - 1e-12 <= st["lambda_star"] <= lam + 1e-7
    tau_or = otgt.tau_lambda_bound(G.degf[u], G.degf[v], eps, lam)
    assert np.all(tau >= tau_or)
    assert np.mean(tau == tau_or) >= 0.999
    ref = otgt.truncated_sc(G, tau)
    tol = FP64_TOL if precision == 1 else FP32_TOL
    np.testing.assert_allclose(out, ref, atol=tol, rtol=0)
    assert np.abs(out - ex.sc_pinv(n, u, v)).max() <= eps


@pytest.mark.parametrize("L", [1, 2, 3, 8, 15])
def test_tgt_fixed_L_matches_closed_form(sc, L):
    graph = gg.barabasi_albert(600, 4, 7)
    out, st, tau, _, _ = run(sc, graph, 0.1, L, method=sc.SC_TGT, precision=1)
    todd = L if L % 2 else L + 1
    assert np.all(tau == todd) and st["L_used"] == todd
    np.testing.assert_allclose(out, ex.s_tau_eigen(*graph, todd), atol=FP64_TOL, rtol=0)


@pytest.mark.parametrize("block", [16, 32, 64])
@pytest.mark.parametrize("precision", [1, 0])
def test_block_widths_heavy_rows_ragged(sc, block, precision):
    # n = 3001 is not a multiple of any block width; hubs exceed the 256-slot chunk
    graph = gg.barabasi_albert(3001, 10, 5)
    d = gg.degrees(*graph)
    assert d.max() > 256
    out, _, tau, _, _ = run(sc, graph, 0.1, 5, method=sc.SC_TGT, precision=precision, block=block)
    ref = otgt.truncated_sc(otgt.Graph(*graph), tau)
    np.testing.assert_allclose(out, ref, atol=FP64_TOL if precision else FP32_TOL, rtol=0)


TINY = {
    "petersen": gg.petersen_graph(),
    "tri_pendant": gg.triangle_pendant(),
    "two_tri_bridge": gg.two_triangles_bridge(),
    "K5": gg.complete_graph(5),
    "C7": gg.cycle_graph(7),
    "triangle": gg.complete_graph(3),
}


@pytest.mark.parametrize("name", list(TINY))
@pytest.mark.parametrize("method", [0, 1])
def test_tiny_graphs_within_eps(sc, name, method):
    graph = TINY[name]
    eps = 1e-3
    out, _, tau, _, _ = run(sc, graph, eps, 0, method=method, precision=1)
    exact = ex.sc_pinv(*graph)
    assert np.abs(out - exact).max() <= eps
    if method == 0:
        np.testing.assert_allclose(out, otgt.truncated_sc(otgt.Graph(*graph), tau), atol=FP64_TOL)


@pytest.mark.parametrize("graph", [gg.tree_plus_gnp(500, 6.0, 9), gg.barabasi_albert(800, 3, 2),
                                   gg.king_grid(400)])
def test_lambda_star(sc, graph):
    g = sc.sc_build_graph(*graph)
    lam = sc.sc_lambda_star(g)
    ref = ex.lambda_star(*graph)
    assert ref - 1e-12 <= lam <= ref + 1e-7


# ------------------------------------------------------------------ TGT+

def oracle_nr(G, tau, tilde, eps, delta, gamma, halves):
    out = {}
    for h in halves:
        i, j = int(G.hsrc[h]), int(G.hdst[h])
        length = int(tau[h % G.m]) - tilde
        if length <= 0:
            out[h] = 0
            continue
        q = otgt.column_at(G, i, tilde)
        chi = otgt.chi_value(G, q, i, j, length, gamma)
        out[h] = otgt.walk_count(chi, G.degf[i], eps, G.m, delta)
    return out


@pytest.mark.parametrize("precision,tilde,gamma", [(1, 2, 10), (0, 2, 10), (1, 3, 0), (1, 1, 10),
                                                   (1, 0, 10), (0, 4, 3)])
def test_tgt_plus_replay_parity(sc, precision, tilde, gamma):
    graph = gg.barabasi_albert(300, 3, 4)
    n, u, v = graph
    eps = 0.2 if tilde >= 2 else 0.5
    out, st, tau, tt, nr = run(sc, graph, eps, 7, method=sc.SC_TGT_PLUS, precision=precision,
                               tilde_tau=tilde, gamma=gamma, seed=12345)
    G = otgt.Graph(n, u, v)
    m = len(u)
    assert st["tilde_tau"] == tilde and np.all(tt == tilde)
    assert np.all(nr[np.concatenate([tau, tau]) <= tilde] == 0)
    assert np.all(nr[np.concatenate([tau, tau]) > tilde] >= 1)
    assert st["walks"] == nr.sum()
    _, _, ref = otgt.tgt_plus_replay(G, tau, tt, nr[:m], nr[m:], seed=12345)
    np.testing.assert_allclose(out, ref, atol=FP64_TOL if precision else FP32_TOL, rtol=0)
    # the GPU's walk counts against the oracle's chi and Eq. 13 (FP64 q)
    rng = np.random.default_rng(0)
    halves = rng.choice(2 * m, size=60, replace=False)
    want = oracle_nr(G, tau, tilde, eps, 1.0 / n, gamma, halves)
    for h in halves:
        # FP64: the two sides differ only in the order of the sums inside chi, which
        # can move Eq. 13's ceiling by one walk; FP32 q also rounds chi itself
        tol = 1 if precision else max(1, 1e-5 * want[h])
        assert abs(int(nr[h]) - want[h]) <= tol, (h, nr[h], want[h])


def test_walk_trace_equals_oracle_walks(sc):
    """The walk stream itself: the nodes a walk pair visits on the GPU (the walk
    kernels' counters and neighbour pick) equal the oracle's Philox walks node by
    node, across Philox word boundaries, from hubs and at the largest r."""
    graph = gg.barabasi_albert(400, 3, 9)
    n, u, v = graph
    G = otgt.Graph(n, u, v)
    g = sc.sc_build_graph(n, u, v)
    hub = int(np.argmax(G.deg))
    cases = [(int(u[0]), int(v[0]), 0, 1, 1), (int(u[5]), int(v[5]), 7, 9, 0x5C5C),
             (hub, int(G.nbr[G.indptr[hub]]), 123456, 37, 2**63 + 12345),
             (int(v[100]), int(u[100]), 2**32 - 1, 64, 99), (3, 250, 5, 23, 7)]
    for i, j, r, length, seed in cases:
        a, b = sc.sc_walk_trace(g, i, j, r, length, seed)
        np.testing.assert_array_equal(a, otgt.walks(G, i, j, [r], 0, length, seed)[0])
        np.testing.assert_array_equal(b, otgt.walks(G, i, j, [r], 1, length, seed)[0])
    for bad in ((n, 0, 0, 4), (0, -1, 0, 4), (0, 1, 2**32, 4), (0, 1, 0, -1)):
        with pytest.raises(sc.ScError) as e:
            sc.sc_walk_trace(g, *bad, 1)
        assert e.value.code == sc.SC_EINVAL
    g.free()


def test_tgt_plus_walks_without_chunk_buffer_match(sc, monkeypatch):
    """Blocks whose walk chunks do not fit the chunk-sum buffer run the per-slot
    walk kernel: same walks, other summation order."""
    graph = gg.barabasi_albert(300, 3, 4)
    n, u, v = graph
    kw = dict(method=sc.SC_TGT_PLUS, precision=1, tilde_tau=2, gamma=10, seed=777)
    flat, st1, tau, tt, nr = run(sc, graph, 0.2, 7, **kw)
    monkeypatch.setenv("SC_WALK_CHUNK_CAPACITY", "1")
    slot, st2, tau2, tt2, nr2 = run(sc, graph, 0.2, 7, **kw)
    np.testing.assert_array_equal(nr, nr2)
    np.testing.assert_allclose(slot, flat, atol=1e-12, rtol=0)
    G = otgt.Graph(n, u, v)
    m = len(u)
    _, _, ref = otgt.tgt_plus_replay(G, tau, tt, nr[:m], nr[m:], seed=777)
    np.testing.assert_allclose(slot, ref, atol=FP64_TOL, rtol=0)


def test_tgt_plus_auto_meets_eps_on_tree_gnp_1k(sc):
    graph = gg.workload("tree_gnp_1k", 2)
    eps = 1e-2
    out, st, tau, tt, nr = run(sc, graph, eps, 0, method=sc.SC_TGT_PLUS, precision=0)
    assert np.abs(out - ex.sc_pinv(*graph)).max() <= eps
    assert 2 <= st["tilde_tau"] <= st["L_used"]


def test_deterministic_rerun(sc):
    graph = gg.barabasi_albert(2000, 5, 3)
    a = run(sc, graph, 0.05, 7, method=sc.SC_TGT_PLUS, precision=0, tilde_tau=3)[0]
    b = run(sc, graph, 0.05, 7, method=sc.SC_TGT_PLUS, precision=0, tilde_tau=3)[0]
    assert np.array_equal(a, b)


def test_device_pointers_and_stream(sc):
    import torch
    graph = gg.barabasi_albert(1500, 4, 8)
    n, u, v = graph
    host = run(sc, graph, 0.05, 5, method=sc.SC_TGT, precision=0)[0]
    g = sc.sc_build_graph(n, u, v)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = torch.full((g.m,), -1.0, dtype=torch.float64, device="cuda")
        tau = torch.zeros(g.m, dtype=torch.int32, device="cuda")
        o = sc.sc_default_options(method=sc.SC_TGT, precision=0)
        sc.sc_all_edges_ex(g, 0.05, 5, o, out=out, tau_out=tau)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), host)
    assert torch.all(tau == 5).item()


def test_merge_duplicates(sc):
    n, u, v = gg.tree_plus_gnp(300, 6.0, 4)
    base = run(sc, (n, u, v), 0.05, 5, method=sc.SC_TGT, precision=1)[0]
    u2 = np.concatenate([u, v[:10]])
    v2 = np.concatenate([v, u[:10]])
    dup = run(sc, (n, u2, v2), 0.05, 5, flags=sc.SC_MERGE_DUPS, method=sc.SC_TGT, precision=1)[0]
    np.testing.assert_array_equal(dup[: len(u)], base)
    np.testing.assert_array_equal(dup[len(u):], base[:10])


def test_error_paths_leave_out_untouched(sc):
    graph = gg.tree_plus_gnp(200, 6.0, 1)
    g = sc.sc_build_graph(*graph)
    out = np.full(g.m, 7.0)
    bad = [(0.0, 3, {}), (1.0, 3, {}), (0.1, -1, {}), (0.1, 3, {"block": 48}),
           (0.1, 3, {"gamma": 17, "method": 1}), (0.1, 3, {"precision": 2}), (0.1, 3, {"method": 5})]
    for eps, L, kw in bad:
        with pytest.raises(sc.ScError) as ei:
            sc.sc_all_edges_ex(g, eps, L, sc.sc_default_options(**kw), out=out)
        assert ei.value.code == sc.SC_EINVAL
        assert np.all(out == 7.0)


# ------------------------------------------------------------------ full-size bench workload

def test_ba_100k_tgt_plus_sampled(sc):
    """The benchmark configuration (BA n=100k, 10 edges per node, TGT+, FP32,
    eps=1e-3, automatic truncation, block 64) checked on sampled edges: exact SC
    by block-PCG within eps, and oracle replay of the same walks."""
    graph = gg.workload("ba_100k", 1)
    n, u, v = graph
    m = len(u)
    eps = 1e-3
    out, st, tau, tt, nr = run(sc, graph, eps, 0, method=sc.SC_TGT_PLUS, precision=0, block=64)
    assert np.all(np.isfinite(out)) and out.min() > 0 and out.max() <= 1 + eps
    rng = np.random.default_rng(11)
    ids = rng.choice(m, size=96, replace=False)
    exact = ex.sc_sampled_pcg(n, u, v, ids)
    assert np.abs(out[ids] - exact).max() <= eps
    G = otgt.Graph(n, u, v)
    sub = ids[:24]
    srcs = np.unique(np.concatenate([u[sub], v[sub]]))
    _, _, ref = otgt.tgt_plus_replay(G, tau, tt, nr[:m], nr[m:], seed=0x5C5C, sources=srcs)
    np.testing.assert_allclose(out[sub], ref[sub], atol=FP32_TOL, rtol=0)


@pytest.mark.parametrize("precision", [1, 0])
def test_dense_erdos_renyi_rows(sc, precision):
    """G(n, m) with n = 700, m = 105,000 (degrees 250-340: most rows are
    workgroup tasks): TGT against the oracle's truncated traversal on every
    edge, and TGT+ against the oracle's replay of the same walks on the edges
    of 12 sources."""
    graph = gg.erdos_renyi_nm(700, 105_000, 2)
    n, u, v = graph
    m = len(u)
    G = otgt.Graph(n, u, v)
    tol = FP64_TOL if precision else FP32_TOL
    out, st, tau, _, _ = run(sc, graph, 1e-3, 0, method=sc.SC_TGT, precision=precision)
    np.testing.assert_allclose(out, otgt.truncated_sc(G, tau), atol=tol, rtol=0)
    out, st, tau, tt, nr = run(sc, graph, 0.3, 7, method=sc.SC_TGT_PLUS, precision=precision,
                               tilde_tau=2, seed=99)
    srcs = np.arange(0, n, 59)[:12]
    _, _, ref = otgt.tgt_plus_replay(G, tau, tt, nr[:m], nr[m:], seed=99, sources=srcs)
    both = np.isin(u, srcs) & np.isin(v, srcs)   # both halves replayed
    assert both.sum() > 0
    np.testing.assert_allclose(out[both], ref[both], atol=tol, rtol=0)


@pytest.mark.parametrize("precision,block", [(1, 64), (0, 64), (0, 16)])
def test_giant_and_heavy_rows(sc, precision, block):
    """A hub with 5,500 neighbours (cut into workgroup chunks and a fix-up
    pass) and hubs with a few hundred (one workgroup each)."""
    n0, u0, v0 = gg.tree_plus_gnp(6000, 6.0, 17)
    rng = np.random.default_rng(5)
    hub = 6000
    spokes = rng.choice(6000, size=5500, replace=False)
    mids = [(6001 + k, rng.choice(6000, size=300 + 40 * k, replace=False)) for k in range(3)]
    u = np.concatenate([u0, np.full(5500, hub)] + [np.full(len(t), h) for h, t in mids])
    v = np.concatenate([v0, spokes] + [t for _, t in mids])
    graph = (6004,) + gg.canonical_edges(6004, u, v)
    d = gg.degrees(*graph)
    assert d.max() > 4096 and np.sum((d > 256) & (d <= 4096)) >= 3
    out, _, tau, _, _ = run(sc, graph, 0.1, 5, method=sc.SC_TGT, precision=precision, block=block)
    ref = otgt.truncated_sc(otgt.Graph(*graph), tau)
    np.testing.assert_allclose(out, ref, atol=FP64_TOL if precision else FP32_TOL, rtol=0)


def two_density_graph(seed=3):
    """Nodes 0-191: G(n, p = 0.8); nodes 192-791: G(n, p) of mean degree 24;
    2,400 random edges join nodes 128-191 to the sparse part.  At eps = 0.05
    the lambda*-bound gives tau = 1 on every edge of nodes 0-127 (two whole
    source blocks of 64 with no traversal) and tau = 7-11 elsewhere."""
    rng = np.random.default_rng(seed)
    nd, ns = 192, 600
    iu = np.triu_indices(nd, 1)
    keep = rng.random(len(iu[0])) < 0.8
    _, u2, v2 = gg.gnp_connected(ns, 24.0, seed)
    a = rng.integers(128, nd, size=2400)
    b = rng.integers(nd, nd + ns, size=2400)
    u = np.concatenate([iu[0][keep], u2 + nd, a])
    v = np.concatenate([iu[1][keep], v2 + nd, b])
    return (nd + ns,) + gg.canonical_edges(nd + ns, u, v)


@pytest.mark.parametrize("precision", [1, 0])
def test_blocks_without_traversal_are_skipped_correctly(sc, precision):
    graph = two_density_graph()
    n, u, v = graph
    m = len(u)
    G = otgt.Graph(n, u, v)
    tol = FP64_TOL if precision else FP32_TOL
    eps = 0.05
    out, st, tau, _, _ = run(sc, graph, eps, 0, method=sc.SC_TGT, precision=precision)
    d = ex.degree_vector(n, u, v)
    want_tau = otgt.tau_lambda_bound(d[u], d[v], eps, ex.lambda_star(n, u, v))
    np.testing.assert_array_equal(tau, want_tau)
    low = (u < 128) & (v < 128)
    assert np.all(tau[(u < 128) | (v < 128)] == 1) and tau.max() >= 7 and low.sum() > 5000
    np.testing.assert_allclose(out, otgt.truncated_sc(G, tau), atol=tol, rtol=0)
    # TGT+ at 2 eps (it truncates at eps / 2, so tau is the same): with
    # tilde = 2 the first two blocks have neither traversal nor walks (replayed
    # on sources from both kinds of block); with tilde = 0 they have walks only
    # (replayed on sources of the first block: their walks have one step)
    cases = {2: np.concatenate([np.arange(0, 6), np.arange(130, 136), np.arange(300, 306)]),
             0: np.arange(0, 8)}
    for tilde, srcs in cases.items():
        both = np.isin(u, srcs) & np.isin(v, srcs)
        assert both[low].sum() > 0 and (tilde == 0 or both[~low].sum() > 0)
        out, st, tau2, tt, nr = run(sc, graph, 2 * eps, 0, method=sc.SC_TGT_PLUS,
                                    precision=precision, tilde_tau=tilde, seed=31)
        np.testing.assert_array_equal(tau2, tau)
        assert st["tilde_tau"] == tilde
        _, _, ref = otgt.tgt_plus_replay(G, tau, tt, nr[:m], nr[m:], seed=31, sources=srcs)
        np.testing.assert_allclose(out[both], ref[both], atol=tol, rtol=0)


@pytest.mark.parametrize("nblocks", [2, 3, 4, 7, 13, 26])
def test_tgt_plus_pipeline_depths(sc, nblocks):
    """The two streams meet once per group of four blocks and the groups cycle
    through three sets of four state pairs, a set reused once the tails of the
    group three back are done: graphs of 2 to 26 blocks (within one group, one
    set, past the first reuse at 13, several reuses and a ragged last group at
    26; the last block ragged at 7 and 26) against the oracle's replay on every
    edge."""
    n = 64 * nblocks - (17 if nblocks in (7, 26) else 0)
    graph = gg.barabasi_albert(n, 3, 40 + nblocks)
    n, u, v = graph
    m = len(u)
    out, st, tau, tt, nr = run(sc, graph, 0.2, 7, method=sc.SC_TGT_PLUS, precision=1,
                               tilde_tau=3, seed=2024)
    assert st["walks"] > 0
    _, _, ref = otgt.tgt_plus_replay(otgt.Graph(n, u, v), tau, tt, nr[:m], nr[m:], seed=2024)
    np.testing.assert_allclose(out, ref, atol=FP64_TOL, rtol=0)
