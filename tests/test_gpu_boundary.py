"""GPU tests of the boundary's reporting and resource paths.

* lambda* (Lemma 3.1's max_{k>=2} |lambda_k|, the rate of Theorem 3.2) from the
  two device Lanczos runs against a dense or sparse eigensolver on graphs up to
  n = 5,000, with the convergence flag set;
* L_capped: the count of edges whose automatic truncation was cut to max_L,
  against the oracle's lambda*-bound (Theorem 3.2) with the same lambda*, for
  one graph and for a batch; zero when nothing is cut;
* batches with CalTau (Algorithm 1): every graph holding a spectrum equals its
  single-graph CalTau run bit for bit (FP64, same block width), nothing is
  capped, and every graph is within eps of the exact SC;
* the network file: save / load round trip, and a corrupted or truncated file
  refused;
* the device-memory budget: an out-of-memory failure leaves the output
  untouched, and the next call within budget succeeds.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import graphgen as gg
from oracle import caltau as ct
from oracle import exact as ex
from oracle import tgt as otgt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_16086_amd import sc as scmod
    return scmod


def lambda_star_sparse(n, u, v):
    """max_{k>=2} |lambda_k| of D^-1/2 A D^-1/2 by ARPACK (both ends)."""
    a = sp.coo_matrix((np.ones(len(u)), (u, v)), shape=(n, n))
    a = (a + a.T).tocsr()
    d = np.asarray(a.sum(1)).ravel()
    s = sp.diags(1.0 / np.sqrt(d))
    N = s @ a @ s
    top = sla.eigsh(N, k=2, which="LA", return_eigenvectors=False, tol=1e-12)
    bot = sla.eigsh(N, k=1, which="SA", return_eigenvectors=False, tol=1e-12)
    return max(sorted(top)[0], -bot[0])


@pytest.mark.parametrize("name", ["ba5000", "gnp3000", "king2500", "tree1000"])
def test_lambda_star_against_eigensolver(sc, name):
    graph = {"ba5000": lambda: gg.barabasi_albert(5000, 4, 3),
             "gnp3000": lambda: gg.gnp_connected(3000, 8.0, 4),
             "king2500": lambda: gg.king_grid(2500),
             "tree1000": lambda: gg.tree_plus_gnp(1000, 10.0, 1)}[name]()
    n, u, v = graph
    print(f"[gpu] lambda* {name} n={n} m={len(u)}", flush=True)
    want = ex.lambda_star(n, u, v) if n <= 2500 else lambda_star_sparse(n, u, v)
    g = sc.sc_build_graph(n, u, v)
    o = sc.sc_default_options(method=sc.SC_TGT, max_L=9)
    _, st = sc.sc_all_edges_ex(g, 0.05, 0, o)
    got = sc.sc_lambda_star(g)
    g.free()
    assert st["lambda_converged"] == 1
    assert st["lambda_star"] == got
    # the extreme Ritz value plus its residual: at least the true value, and close
    assert got >= want - 1e-9, (got, want)
    assert got <= want + 1e-6, (got, want)


def test_lambda_converged_is_minus_one_when_given(sc):
    n, u, v = gg.barabasi_albert(300, 3, 1)
    g = sc.sc_build_graph(n, u, v)
    _, st = sc.sc_all_edges_ex(g, 0.05, 0, sc.sc_default_options(lambda_star=0.6))
    assert st["lambda_converged"] == -1 and st["lambda_star"] == 0.6
    _, st = sc.sc_all_edges_ex(g, 0.05, 5, sc.sc_default_options())
    assert st["lambda_converged"] == -1 and st["L_capped"] == 0
    g.free()


# TGT+ only with short caps: the grid's walk counts at long truncations are huge
@pytest.mark.parametrize("method,max_L", [(0, 3), (0, 7), (0, 255), (1, 3), (1, 7)])
def test_L_capped_counts_cut_edges(sc, method, max_L):
    n, u, v = gg.king_grid(400)
    eps = 1e-2
    print(f"[gpu] L_capped king400 method={method} max_L={max_L}", flush=True)
    g = sc.sc_build_graph(n, u, v)
    tau = np.empty(len(u), np.int32)
    o = sc.sc_default_options(method=method, max_L=max_L)
    _, st = sc.sc_all_edges_ex(g, eps, 0, o, tau_out=tau)
    lam = st["lambda_star"]
    g.free()
    G = otgt.Graph(n, u, v)
    eps_tau = eps / 2 if method == 1 else eps
    raw = otgt.tau_lambda_bound(G.degf[u], G.degf[v], eps_tau, lam)
    want = int((raw > max_L).sum())
    assert st["L_capped"] == want
    np.testing.assert_array_equal(tau, np.minimum(raw, max_L))
    if max_L <= 7:
        assert want > 0


def test_L_capped_zero_on_fast_mixing_graph(sc):
    n, u, v = gg.barabasi_albert(2000, 10, 1)
    g = sc.sc_build_graph(n, u, v)
    _, st = sc.sc_all_edges_ex(g, 1e-3, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS))
    g.free()
    assert st["L_capped"] == 0 and st["lambda_converged"] == 1


def batch_graphs():
    return [gg.king_grid(300), gg.barabasi_albert(400, 5, 2), gg.king_grid(529),
            gg.gnp_connected(350, 8.0, 3), gg.king_grid(150)]


def test_batch_L_capped_matches_single_runs(sc):
    graphs = batch_graphs()
    b = sc.sc_build_batch(graphs)
    eps, max_L = 1e-2, 15
    o = sc.sc_default_options(method=sc.SC_TGT, precision=1, block=16, max_L=max_L)
    _, st = sc.sc_batch_all_edges(b, eps, None, o)
    total = 0
    for i in range(len(graphs)):
        _, s1 = sc.sc_all_edges_ex(b.graphs[i], eps, 0, o)
        total += s1["L_capped"]
    b.free()
    assert total > 0
    assert st["L_capped"] == total


@pytest.mark.parametrize("block", [16, 64])
def test_batch_caltau_equals_single_graph_caltau(sc, block):
    graphs = batch_graphs()
    b = sc.sc_build_batch(graphs)
    eps = 1e-2
    omega = 64
    kings = [0, 2, 4]
    for i in kings:    # grids: repeated eigenvalues, so the exact pairs are loaded
        n, u, v = graphs[i]
        lam, phi = ct.top_spectrum(n, u, v, omega)
        sc.sc_set_spectrum(b.graphs[i], lam, phi)
    print(f"[gpu] batch CalTau block={block}", flush=True)
    o = sc.sc_default_options(method=sc.SC_TGT, precision=1, block=block,
                              flags=sc.SC_TAU_SPECTRAL)
    outs, st = sc.sc_batch_all_edges(b, eps, None, o)
    capped = 0
    plain = sc.sc_default_options(method=sc.SC_TGT, precision=1, block=block)
    for i, (n, u, v) in enumerate(graphs):
        tau = np.empty(len(u), np.int32)
        # graphs without a spectrum take the lambda*-bound in the batch as well
        one, s1 = sc.sc_all_edges_ex(b.graphs[i], eps, 0, o if i in kings else plain, tau_out=tau)
        capped += s1["L_capped"]
        np.testing.assert_array_equal(outs[i], one)
        err = np.abs(outs[i] - ex.sc_pinv(n, u, v)).max()
        assert err <= eps, (i, err)
        if i in kings:
            # CalTau with the given pairs: the oracle's lengths (Eq. 6-8)
            lam, phi = ct.top_spectrum(n, u, v, omega)
            margins = []
            want = ct.caltau(n, u, v, eps, lam, phi, max_L=255, margins=margins)
            bad = tau != want
            assert np.all(np.asarray(margins)[bad] < 1e-9) if bad.any() else True
    b.free()
    assert st["L_capped"] == 0 and capped == 0


def test_mlp_file_round_trip(sc, tmp_path):
    import torch
    net = sc.sc_mlp_create(7)
    rng = np.random.default_rng(0)
    norm = np.concatenate([rng.normal(size=16), 1.0 + rng.random(16)]).astype(np.float32)
    rg = np.concatenate([-1 - rng.random(16), 1 + rng.random(16)]).astype(np.float32)
    sc.sc_mlp_set(net, norm=norm, range_=rg)
    path = str(tmp_path / "net.bin")
    sc.sc_mlp_save(net, path)
    back = sc.sc_mlp_load(path)
    for a, c in zip(sc.sc_mlp_get(net), sc.sc_mlp_get(back)):
        np.testing.assert_array_equal(a, c)
    X = torch.tensor(rng.normal(size=(1000, 16)), dtype=torch.float32, device="cuda")
    y1 = torch.empty(1000, dtype=torch.float32, device="cuda")
    y2 = torch.empty_like(y1)
    sc.sc_mlp_predict(net, X, 1, y1)
    sc.sc_mlp_predict(back, X, 1, y2)
    assert torch.equal(y1, y2)
    back.free()
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0x40
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(sc.ScError) as e:
        sc.sc_mlp_load(bad)
    assert e.value.code == sc.SC_EINVAL and "checksum" in str(e.value)
    short = str(tmp_path / "short.bin")
    open(short, "wb").write(bytes(raw[:-9]))
    with pytest.raises(sc.ScError):
        sc.sc_mlp_load(short)
    with pytest.raises(sc.ScError):
        sc.sc_mlp_load(str(tmp_path / "missing.bin"))
    net.free()


@pytest.mark.parametrize("method", [0, 1])
def test_out_of_memory_leaves_output_untouched(sc, method, monkeypatch):
    n, u, v = gg.barabasi_albert(3000, 5, 9)
    g = sc.sc_build_graph(n, u, v)       # graph memory is allocated before the budget is set
    lam = sc.sc_lambda_star(g)
    out = np.full(len(u), -7.0)
    monkeypatch.setenv("SC_DEVICE_BYTES_LIMIT", "1")
    o = sc.sc_default_options(method=method, lambda_star=lam)
    with pytest.raises(sc.ScError) as e:
        sc.sc_all_edges_ex(g, 1e-2, 0, o, out=out)
    assert e.value.code == sc.SC_ENOMEM
    assert np.all(out == -7.0)
    monkeypatch.delenv("SC_DEVICE_BYTES_LIMIT")
    res, _ = sc.sc_all_edges_ex(g, 1e-2, 0, o, out=out)
    g.free()
    assert np.all(np.isfinite(res)) and np.all(res > 0)
