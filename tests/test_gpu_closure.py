"""GPU checks of the learned tail closure against the CPU oracle.

* features, s_7, u_3 and the certified interval against oracle.closure on the
  oracle's own recordings of the first 8 steps;
* the FP32 training gradient against the float64 reference network;
* BF16 MFMA inference against FP32 inference and the reference forward pass;
* end to end: trained on small BA and G(n,p) graphs with L = 201 targets,
  evaluated on a held-out BA graph: every edge within eps of the exact SC
  (certified interval + fallback), smaller error than the truncation s_7 and
  than the midpoint of the interval, and forcing the fallback reproduces TGT.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import closure as cl
from oracle import exact as ex
from oracle import mlp as omlp
from oracle import tgt as otgt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_16086_amd import sc
    return sc, torch


def test_closure_features_match_oracle(env):
    sc, torch = env
    graph = gg.barabasi_albert(1500, 4, 21)
    n, u, v = graph
    m = len(u)
    print(f"[gpu] closure features n={n} m={m}", flush=True)
    g = sc.sc_build_graph(n, u, v)
    X = torch.empty(m * 16, dtype=torch.float32, device="cuda")
    s0, uK, lo, hi = (torch.empty(m, dtype=torch.float64, device="cuda") for _ in range(4))
    sc.sc_closure_features(g, 1, X, s0, uK, lo, hi)
    lam_gpu = sc.sc_lambda_star(g)
    G = otgt.Graph(n, u, v)
    _, _, diag, off = otgt.traversal(G, np.full(m, 8), record=8)
    F = cl.features(diag, off, G.deg, u, v)
    os0, ouK, olo, ohi = cl.head_and_bounds(diag, off, G.deg, u, v, lam_gpu)
    Xg = X.cpu().numpy().reshape(m, 16)
    np.testing.assert_allclose(Xg, F, rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(s0.cpu().numpy(), os0, atol=1e-13)
    np.testing.assert_allclose(uK.cpu().numpy(), ouK, atol=1e-14)
    np.testing.assert_allclose(lo.cpu().numpy(), olo, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(hi.cpu().numpy(), ohi, rtol=1e-12)


def test_mlp_gradient_matches_float64_reference(env):
    sc, torch = env
    rng = np.random.default_rng(3)
    N = 333
    Xh = rng.normal(size=(N, 16)).astype(np.float32)
    zh = rng.normal(size=N).astype(np.float32)
    wh = (rng.random(N) > 0.2).astype(np.float32)
    net = sc.sc_mlp_create(5)
    ident = np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32)
    sc.sc_mlp_set(net, norm=ident)
    th, _, _ = sc.sc_mlp_get(net)
    X = torch.from_numpy(Xh).cuda().reshape(-1)
    z = torch.from_numpy(zh).cuda()
    w = torch.from_numpy(wh).cuda()
    gg_, loss = sc.sc_mlp_grad(net, X, z, w)
    # reference: weighted mean squared error over N (weights 0/1)
    keep = wh > 0
    ref_loss, ref_g = omlp.loss_and_grad(th.astype(np.float64), Xh[keep].astype(np.float64),
                                         zh[keep].astype(np.float64))
    scale = keep.sum() / N
    ref_loss *= scale
    ref_g *= scale
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    np.testing.assert_allclose(gg_, ref_g, rtol=1e-4, atol=1e-5 * np.abs(ref_g).max())


def test_bf16_inference_matches_fp32_and_reference(env):
    sc, torch = env
    rng = np.random.default_rng(4)
    N = 1000 + 7    # not a multiple of the 16-sample tile
    Xh = rng.normal(size=(N, 16)).astype(np.float32)
    net = sc.sc_mlp_create(9)
    norm = np.concatenate([rng.normal(size=16) * 0.1, 1 + 0.1 * rng.random(16)]).astype(np.float32)
    sc.sc_mlp_set(net, norm=norm)
    th, _, _ = sc.sc_mlp_get(net)
    X = torch.from_numpy(Xh).cuda().reshape(-1)
    y32 = sc.sc_mlp_predict(net, X, bf16=0).cpu().numpy()
    y16 = sc.sc_mlp_predict(net, X, bf16=1).cpu().numpy()
    Xn = (Xh.astype(np.float64) - norm[:16]) * norm[16:]
    ref, _ = omlp.forward(th.astype(np.float64), Xn)
    np.testing.assert_allclose(y32, ref, rtol=1e-4, atol=1e-5)
    scale = np.abs(ref).max()
    assert np.abs(y16 - ref).max() <= 2e-2 * scale


def _dataset(sc, torch, graph, L_ref=201):
    n, u, v = graph
    g = sc.sc_build_graph(n, u, v)
    m = len(u)
    X = torch.empty(m * 16, dtype=torch.float32, device="cuda")
    z = torch.empty(m, dtype=torch.float32, device="cuda")
    w = torch.empty(m, dtype=torch.float32, device="cuda")
    sc.sc_closure_dataset(g, L_ref, 1, X, z, w)
    return g, X, z, w


def test_learned_closure_end_to_end(env):
    sc, torch = env
    train = [gg.barabasi_albert(3000, 4, 101), gg.barabasi_albert(2500, 6, 102),
             gg.tree_plus_gnp(3000, 8.0, 103), gg.gnp_connected(2500, 10.0, 104)]
    Xs, zs, ws = [], [], []
    for graph in train:
        print(f"[gpu] dataset n={graph[0]} m={len(graph[1])}", flush=True)
        _, X, z, w = _dataset(sc, torch, graph)
        Xs.append(X)
        zs.append(z)
        ws.append(w)
    X = torch.cat(Xs)
    z = torch.cat(zs)
    w = torch.cat(ws)
    net = sc.sc_mlp_create(11)
    losses = sc.sc_mlp_train(net, X, z, w, sc.sc_default_train_options(epochs=30, batch=2048))
    assert losses[-1] < losses[0]
    # held-out graph
    graph = gg.barabasi_albert(3000, 5, 999)
    n, u, v = graph
    g = sc.sc_build_graph(n, u, v)
    exact = ex.sc_pinv(n, u, v)
    eps = 1e-3
    o = sc.sc_default_options(method=sc.SC_LEARNED, precision=0, mlp=net.handle.value)
    out, st = sc.sc_all_edges_ex(g, eps, 0, o)
    err = np.abs(out - exact)
    assert err.max() <= eps
    # baselines from the oracle: plain truncation at 7 and the interval midpoint
    G = otgt.Graph(n, u, v)
    _, _, diag, off = otgt.traversal(G, np.full(len(u), 8), record=8)
    s0, uK, lo, hi = cl.head_and_bounds(diag, off, G.deg, u, v, st["lambda_star"])
    mid = cl.apply_closure(s0, uK, lo, hi, (lo + hi) / 2)
    ok = np.ones(len(u), bool)
    print(f"learned mean err {err.mean():.3e} max {err.max():.3e}; s7 mean "
          f"{np.abs(s0 - exact).mean():.3e}; midpoint mean {np.abs(mid - exact).mean():.3e}; "
          f"fallback {st['fallback_edges']}", flush=True)
    assert err[ok].mean() < np.abs(s0 - exact)[ok].mean()
    assert err[ok].mean() < np.abs(mid - exact)[ok].mean()
    # forcing the fallback everywhere is plain TGT at eps
    o2 = sc.sc_default_options(method=sc.SC_LEARNED, precision=0, mlp=net.handle.value,
                               force_fallback=1)
    out2, st2 = sc.sc_all_edges_ex(g, eps, 0, o2)
    plain, _ = sc.sc_all_edges_ex(g, eps, 0, sc.sc_default_options(method=sc.SC_TGT, precision=0))
    assert st2["fallback_edges"] == len(u)
    np.testing.assert_array_equal(out2, plain)
    # narrower source blocks (other row-sum orders, the last recorded step with
    # fewer columns): still certified, the same closure up to rounding
    for blk in (32, 16):
        o3 = sc.sc_default_options(method=sc.SC_LEARNED, precision=0, mlp=net.handle.value,
                                   block=blk)
        out3, st3 = sc.sc_all_edges_ex(g, eps, 0, o3)
        assert np.abs(out3 - exact).max() <= eps
        assert abs(st3["fallback_edges"] - st["fallback_edges"]) <= max(2, len(u) // 100)
        assert np.median(np.abs(out3 - out)) <= 1e-6
