"""GPU checks of the node orders SC_DEGREE_ORDER and SC_BFS_ORDER: a handle that
stores the graph with its nodes renumbered by descending degree (ties by id),
or in breadth-first order from the highest-degree node.

The flagged handle must compute exactly what an unflagged handle computes on
the renumbered edge list (same CSR, same sums, same walks), while every node
id at the interface stays the caller's:

* TGT and TGT+ (dense blocks, FP32 and FP64) and per-source TGT+: outputs,
  tau and n_r traces and statistics bit for bit; tilde_tau_out per node in
  the caller's ids (host and device outputs);
* a per-source source list in the caller's ids;
* the allocation-free entry point's device tilde output;
* spectra: a loaded spectrum read back unchanged, a computed one equal to
  the renumbered handle's rows;
* walk traces in the caller's ids;
* the estimate within eps of the exact SC (labelling does not change SC).

The renumbering itself is recomputed here from its definition (numpy stable
argsort of the negated degrees; a plain breadth-first search over sorted
neighbour lists).
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import exact as ex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_16086_amd import sc as scmod
    return scmod


@pytest.fixture(scope="module")
def graph():
    # R-MAT component: randomly labelled, heavy-tailed degrees
    return gg.rmat_lcc(10, 8, seed=3)


def renumbering(n, u, v, kind):
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    if kind == "degree":
        label = np.argsort(-deg, kind="stable")   # stored node y is the caller's label[y]
    else:
        adj = [[] for _ in range(n)]
        for a, b in zip(u.tolist(), v.tolist()):
            adj[a].append(b)
            adj[b].append(a)
        start = int(np.argmax(deg))   # the first of the highest degree
        seen = np.zeros(n, bool)
        seen[start] = True
        order = [start]
        for x in order:               # grows while it is walked
            for y in sorted(adj[x]):
                if not seen[y]:
                    seen[y] = True
                    order.append(y)
        order += [x for x in range(n) if not seen[x]]
        label = np.array(order)
    rank = np.empty(n, np.int64)
    rank[label] = np.arange(n)
    return rank, label


@pytest.fixture(scope="module", params=["degree", "bfs"])
def pair(sc, graph, request):
    n, u, v = graph
    kind = request.param
    rank, label = renumbering(n, u, v, kind)
    assert not np.array_equal(label, np.arange(n))   # the order does change the ids
    print(f"[gpu] node order {kind}: n={n} m={len(u)}", flush=True)
    flag = sc.SC_DEGREE_ORDER if kind == "degree" else sc.SC_BFS_ORDER
    gf = sc.sc_build_graph(n, u, v, flag)
    gr = sc.sc_build_graph(n, rank[u], rank[v])
    yield gf, gr, rank, label
    gf.free()
    gr.free()


def run(sc, g, n, m, eps, L=0, sources=None, **opt):
    o = sc.sc_default_options(seed=91, **opt)
    tau = np.empty(m, np.int32)
    tt = np.empty(n, np.int32)
    nr = np.empty(2 * m, np.int64)
    out, st = sc.sc_all_edges_ex(g, eps, L, o, tau_out=tau, tilde_tau_out=tt, nr_out=nr,
                                 sources=sources)
    return out, st, tau, tt, nr


CASES = [
    ("tgt fp32", 1e-2, 0, dict(method=0, precision=0)),
    ("tgt fp64 L=9", 1e-2, 9, dict(method=0, precision=1)),
    ("tgt+ fp32", 1e-3, 0, dict(method=1, precision=0)),
    # a forced early switch: 1.2e6 walk pairs at eps = 0.05 (2e10 at 1e-3)
    ("tgt+ fp64 tilde 3", 0.05, 0, dict(method=1, precision=1, tilde_tau=3)),
    ("per-source tgt+", 1e-3, 0, dict(method=1, flags=0x20)),
]


@pytest.mark.parametrize("name,eps,L,opt", CASES, ids=[c[0] for c in CASES])
def test_flagged_equals_renumbered_graph(sc, graph, pair, name, eps, L, opt):
    n, u, v = graph
    m = len(u)
    gf, gr, rank, label = pair
    print(f"[gpu] degree order case {name}", flush=True)
    of, sf, tf, ttf, nf = run(sc, gf, n, m, eps, L, **opt)
    orr, sr, tr, ttr, nrr = run(sc, gr, n, m, eps, L, **opt)
    assert np.array_equal(of, orr)
    assert np.array_equal(tf, tr)
    assert np.array_equal(nf, nrr)
    assert np.array_equal(ttf, ttr[rank])   # per node, in the caller's ids
    for k in ("walks", "walk_steps", "L_used", "L_min", "tilde_min", "tilde_max", "push_edges"):
        assert sf[k] == sr[k], k


def test_per_source_list_in_caller_ids(sc, graph, pair):
    import torch
    n, u, v = graph
    m = len(u)
    gf, gr, rank, label = pair
    rng = np.random.default_rng(4)
    src = rng.choice(n, size=97, replace=False).astype(np.int32)
    print("[gpu] degree order: source list", flush=True)
    of, sf, tf, ttf, nf = run(sc, gf, n, m, 1e-3, sources=src, method=1, flags=0x20)
    orr, sr, tr, ttr, nrr = run(sc, gr, n, m, 1e-3, sources=rank[src].astype(np.int32),
                                method=1, flags=0x20)
    assert np.array_equal(of, orr)
    assert np.array_equal(nf, nrr)
    assert np.array_equal(ttf, ttr[rank])
    assert sf["walks"] == sr["walks"]
    # device outputs: the tilde trace gathered on the device
    dev = torch.device("cuda:0")
    od = torch.empty(m, dtype=torch.float64, device=dev)
    ttd = torch.empty(n, dtype=torch.int32, device=dev)
    o = sc.sc_default_options(seed=91, method=1, flags=0x20)
    sc.sc_all_edges_ex(gf, 1e-3, 0, o, out=od, tilde_tau_out=ttd, sources=src)
    torch.cuda.synchronize()
    assert np.array_equal(od.cpu().numpy(), of)
    assert np.array_equal(ttd.cpu().numpy(), ttf)


def test_static_entry_point_tilde_in_caller_ids(sc, graph, pair):
    import torch
    n, u, v = graph
    m = len(u)
    gf, gr, rank, label = pair
    print("[gpu] degree order: static entry point", flush=True)
    of, sf, tf, ttf, nf = run(sc, gf, n, m, 1e-3, method=1, flags=0x20)
    dev = torch.device("cuda:0")
    out = torch.empty(m, dtype=torch.float64, device=dev)
    tt = torch.full((n,), -7, dtype=torch.int32, device=dev)
    nr = torch.empty(2 * m, dtype=torch.int64, device=dev)
    o = sc.sc_default_options(seed=91, method=1)
    sc.sc_all_edges_static(gf, 1e-3, 0, o, out, tilde_tau_out=tt, nr_out=nr)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), of)
    assert np.array_equal(tt.cpu().numpy(), ttf)
    assert np.array_equal(nr.cpu().numpy(), nf)


def test_spectrum_rows_in_caller_ids(sc, graph, pair):
    n, u, v = graph
    gf, gr, rank, label = pair
    print("[gpu] degree order: spectrum", flush=True)
    kf, _ = sc.sc_compute_spectrum(gf, 8)
    kr, _ = sc.sc_compute_spectrum(gr, 8)
    assert kf == kr
    lf, pf = sc.sc_get_spectrum(gf)
    lr, pr = sc.sc_get_spectrum(gr)
    assert np.array_equal(lf, lr)
    assert np.array_equal(pf, pr[rank])
    # a loaded spectrum reads back as given
    rng = np.random.default_rng(8)
    lam = np.concatenate([[1.0], np.sort(rng.uniform(0.1, 0.9, 5))[::-1]])
    phi = rng.standard_normal((n, 6))
    sc.sc_set_spectrum(gf, lam, phi)
    l2, p2 = sc.sc_get_spectrum(gf)
    assert np.array_equal(l2, lam)
    assert np.array_equal(p2, phi)
    # and CalTau on the flagged handle equals CalTau on the renumbered one
    sc.sc_set_spectrum(gr, lam, phi[label])
    m = len(u)
    of, _, tf, _, _ = run(sc, gf, n, m, 1e-2, method=0, flags=sc.SC_TAU_SPECTRAL)
    orr, _, tr, _, _ = run(sc, gr, n, m, 1e-2, method=0, flags=sc.SC_TAU_SPECTRAL)
    assert np.array_equal(tf, tr)
    assert np.array_equal(of, orr)


def test_walk_trace_in_caller_ids(sc, graph, pair):
    n, u, v = graph
    gf, gr, rank, label = pair
    print("[gpu] degree order: walk trace", flush=True)
    rng = np.random.default_rng(2)
    for e in rng.choice(len(u), size=6, replace=False):
        i, j = int(u[e]), int(v[e])
        a_f, b_f = sc.sc_walk_trace(gf, i, j, 5, 23, 0x1234)
        a_r, b_r = sc.sc_walk_trace(gr, int(rank[i]), int(rank[j]), 5, 23, 0x1234)
        assert np.array_equal(a_f, label[a_r])
        assert np.array_equal(b_f, label[b_r])
        # every step moves along an edge of the caller's graph
        adj = set(zip(u.tolist(), v.tolist())) | set(zip(v.tolist(), u.tolist()))
        for path, start in ((a_f, i), (b_f, j)):
            prev = start
            for x in path.tolist():
                assert (prev, x) in adj
                prev = x


def test_within_eps_of_exact(sc, graph, pair):
    n, u, v = graph
    gf = pair[0]
    print("[gpu] degree order: exact", flush=True)
    exact = ex.sc_pinv(n, u, v)
    for eps, opt in ((1e-2, dict(method=1)), (1e-2, dict(method=1, flags=0x20))):
        out, *_ = run(sc, gf, n, len(u), eps, **opt)
        assert np.abs(out - exact).max() <= eps


def test_learned_closure_and_dataset(sc, graph, pair):
    import torch
    n, u, v = graph
    m = len(u)
    gf, gr, rank, label = pair
    print("[gpu] degree order: learned closure", flush=True)
    data = []
    for g in (gf, gr):
        X = torch.empty(m * 16, dtype=torch.float32, device="cuda")
        z = torch.empty(m, dtype=torch.float32, device="cuda")
        w = torch.empty(m, dtype=torch.float32, device="cuda")
        sc.sc_closure_dataset(g, 41, 1, X, z, w)
        torch.cuda.synchronize()
        data.append([t.cpu().numpy() for t in (X, z, w)])
    for a, b in zip(*data):   # per edge, input order
        assert np.array_equal(a, b)
    net = sc.sc_mlp_create(5)
    outs = []
    for g in (gf, gr):
        o = sc.sc_default_options(method=sc.SC_LEARNED, precision=0, mlp=net.handle.value)
        out, st = sc.sc_all_edges_ex(g, 1e-2, 0, o)
        outs.append((out, st["fallback_edges"]))
    net.free()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
