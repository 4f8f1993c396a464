"""GPU parity of the batched persistent launch (many graphs, one launch).

* each graph's batched result equals the single-graph TGT run with the same
  block width bit for bit (B = 16, 32, 64: the batch kernel adds every row in
  the single-graph order), in FP64 and FP32;
* against the oracle's truncated traversal with the GPU's per-edge tau, for
  every block width 1..64 (FP64 to 1e-12, FP32 to 2e-5), including rows of
  more than 256 and more than 4096 neighbours and states too large for LDS
  (device slabs);
* against the exact SC of the mixed-family workload (G(n,p), Barabasi-Albert,
  king grids) within eps, with the automatic truncation capped at max_L;
* hipGraph replay: repeated replays with eager work in between equal the
  eager result; the tuning table round-trips through its JSON file;
* error paths.
"""
import os

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


def small_mix(seed=5):
    # sizes span one to several 64-row groups, ragged tails and block tails
    return [gg.gnp_connected(130, 8.0, seed), gg.barabasi_albert(257, 5, seed + 1),
            gg.king_grid(200), gg.tree_plus_gnp(600, 10.0, seed + 2),
            gg.barabasi_albert(1000, 5, seed + 3), gg.king_grid(431),
            gg.gnp_connected(777, 8.0, seed + 4)]


def single(sc, b, i, eps, L, precision, block):
    o = sc.sc_default_options(method=sc.SC_TGT, precision=precision, block=block)
    tau = np.empty(b.sizes[i][1], np.int32)
    out, st = sc.sc_all_edges_ex(b.graphs[i], eps, L, o, tau_out=tau)
    return out, tau


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("block", [16, 32, 64])
def test_batch_equals_single_graph_bitwise(sc, precision, block):
    graphs = small_mix()
    print(f"[gpu] batch bitwise precision={precision} B={block}", flush=True)
    b = sc.sc_build_batch(graphs)
    o = sc.sc_default_options(method=sc.SC_TGT, precision=precision, block=block)
    outs, st = sc.sc_batch_all_edges(b, 1e-2, None, o)
    assert st["block"] == block
    for i in range(len(graphs)):
        ref, _ = single(sc, b, i, 1e-2, 0, precision, block)
        np.testing.assert_array_equal(outs[i], ref)
    b.free()


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("block", [1, 2, 4, 8, 16, 64])
def test_batch_matches_oracle(sc, precision, block):
    graphs = small_mix(11)
    print(f"[gpu] batch vs oracle precision={precision} B={block}", flush=True)
    b = sc.sc_build_batch(graphs)
    o = sc.sc_default_options(method=sc.SC_TGT, precision=precision, block=block)
    L = [0, 9, 0, 4, 0, 21, 1]   # automatic and fixed (even rounds up)
    outs, st = sc.sc_batch_all_edges(b, 2e-2, L, o)
    tol = FP64_TOL if precision == 1 else FP32_TOL
    for i, (n, u, v) in enumerate(graphs):
        _, tau = single(sc, b, i, 2e-2, L[i], 1, 64)
        if L[i] > 0:
            assert np.all(tau == (L[i] if L[i] % 2 else L[i] + 1))
        ref = otgt.truncated_sc(otgt.Graph(n, u, v), tau)
        np.testing.assert_allclose(outs[i], ref, atol=tol, rtol=0)
    assert st["L_used"] >= 21 and st["L_min"] == 1
    b.free()


def hub_graph(n, hub_deg, seed):
    """Tree + G(n,p) plus node 0 joined to hub_deg other nodes (a heavy row)."""
    n_, u, v = gg.tree_plus_gnp(n, 6.0, seed)
    rng = np.random.default_rng(seed)
    extra = rng.choice(np.arange(1, n), size=hub_deg, replace=False)
    u = np.concatenate([u, np.zeros(hub_deg, np.int64)])
    v = np.concatenate([v, extra.astype(np.int64)])
    u, v = gg.canonical_edges(n, u, v)
    return n, u, v


@pytest.mark.parametrize("precision", [1, 0])
def test_batch_heavy_giant_rows_and_slabs(sc, precision):
    # degrees above 256 and above 4096; B = 64 FP64 states exceed LDS (slabs)
    graphs = [hub_graph(700, 400, 3), hub_graph(5000, 4500, 4), gg.king_grid(300)]
    print(f"[gpu] batch heavy rows precision={precision}", flush=True)
    b = sc.sc_build_batch(graphs)
    for block in (64, 16, 1):
        o = sc.sc_default_options(method=sc.SC_TGT, precision=precision, block=block)
        outs, _ = sc.sc_batch_all_edges(b, 0.05, [7, 5, 9], o)
        for i, (n, u, v) in enumerate(graphs):
            ref_single, tau = single(sc, b, i, 0.05, [7, 5, 9][i], precision, max(block, 16))
            if block >= 16:
                np.testing.assert_array_equal(outs[i], ref_single)
            ref = otgt.truncated_sc(otgt.Graph(n, u, v), tau)
            tol = FP64_TOL if precision == 1 else FP32_TOL
            np.testing.assert_allclose(outs[i], ref, atol=tol, rtol=0)
    b.free()


def test_batch_mixed_families_exact(sc):
    # eps against the exact SC; king grids need the empirical cap max_L
    graphs = gg.mixed_batch(24, 200, 1200, 3)
    print(f"[gpu] mixed batch exact, {len(graphs)} graphs", flush=True)
    b = sc.sc_build_batch(graphs)
    eps = 1e-2
    o = sc.sc_default_options(method=sc.SC_TGT, precision=0, max_L=31)
    outs, st = sc.sc_batch_all_edges(b, eps, None, o)
    assert st["L_used"] <= 31
    worst = 0.0
    for i, (n, u, v) in enumerate(graphs):
        err = np.abs(outs[i] - ex.sc_pinv(n, u, v)).max()
        worst = max(worst, err)
    print(f"max err {worst:.3e}", flush=True)
    assert worst <= eps
    b.free()


def test_batch_device_outputs_and_replay(sc):
    import torch
    graphs = small_mix(21)
    print("[gpu] batch replay", flush=True)
    b = sc.sc_build_batch(graphs)
    o = sc.sc_default_options(method=sc.SC_TGT, precision=0, block=32)
    eager, _ = sc.sc_batch_all_edges(b, 1e-2, None, o)
    o2 = sc.sc_default_options(method=sc.SC_TGT, precision=0, block=32, flags=sc.SC_GRAPH_REPLAY)
    for rep in range(3):
        outs, _ = sc.sc_batch_all_edges(b, 1e-2, None, o2)
        for i in range(len(graphs)):
            np.testing.assert_array_equal(outs[i], eager[i])
        # eager work of another configuration between replays
        other, _ = sc.sc_batch_all_edges(b, 1e-2, 5, sc.sc_default_options(precision=1, block=8))
        assert np.all(np.isfinite(other[0]))
    # device outputs, replayed on the torch stream
    dev = [torch.full((m,), -1.0, dtype=torch.float64, device="cuda") for _, m in b.sizes]
    o3 = sc.sc_default_options(method=sc.SC_TGT, precision=0, block=32, flags=sc.SC_GRAPH_REPLAY)
    for rep in range(2):
        for t in dev:
            t.fill_(-1.0)
        sc.sc_batch_all_edges(b, 1e-2, None, o3, out=dev)
        torch.cuda.synchronize()
        for i in range(len(graphs)):
            np.testing.assert_array_equal(dev[i].cpu().numpy(), eager[i])
    b.free()


def test_batch_autotune_roundtrip(sc, tmp_path):
    graphs = gg.mixed_batch(9, 200, 3000, 4)
    print("[gpu] batch autotune", flush=True)
    b = sc.sc_build_batch(graphs)
    o = sc.sc_default_options(method=sc.SC_TGT, precision=0, max_L=31)
    path = str(tmp_path / "tune.json")
    sc.sc_batch_autotune(b, 1e-2, None, o, path)
    assert os.path.getsize(path) > 0
    tuned = sc.sc_batch_blocks(b, o)
    assert set(tuned.tolist()) <= {1, 2, 4, 8, 16, 32, 64}
    b2 = sc.sc_build_batch(graphs)
    sc.sc_batch_load_tuning(b2, path)
    np.testing.assert_array_equal(sc.sc_batch_blocks(b2, o), tuned)
    outs, st = sc.sc_batch_all_edges(b2, 1e-2, None, o)
    for i, (n, u, v) in enumerate(graphs):
        _, tau = single(sc, b2, i, 1e-2, 0, 1, 64)
        ref = otgt.truncated_sc(otgt.Graph(n, u, v), np.minimum(tau, 31))
        np.testing.assert_allclose(outs[i], ref, atol=FP32_TOL, rtol=0)
    b.free()
    b2.free()


@pytest.mark.parametrize("precision", [1, 0])
def test_batch_tiny_graphs(sc, precision):
    # fewer nodes than one block, one row group, triangles and bridges
    graphs = [gg.triangle_pendant(), gg.two_triangles_bridge(), gg.complete_graph(5),
              gg.petersen_graph(), gg.cycle_graph(7)]
    print(f"[gpu] batch tiny graphs precision={precision}", flush=True)
    b = sc.sc_build_batch(graphs)
    for block in (0, 1, 64):
        o = sc.sc_default_options(method=sc.SC_TGT, precision=precision, block=block)
        outs, _ = sc.sc_batch_all_edges(b, 1e-3, [9, 9, 9, 9, 9], o)
        for i, (n, u, v) in enumerate(graphs):
            ref = ex.s_tau_eigen(n, u, v, 9)
            np.testing.assert_allclose(outs[i], ref, atol=FP64_TOL if precision else FP32_TOL,
                                       rtol=0)
    b.free()


def test_batch_errors(sc):
    graphs = small_mix()[:2]
    b = sc.sc_build_batch(graphs)
    with pytest.raises(sc.ScError) as e:
        sc.sc_batch_all_edges(b, 1e-2, None, sc.sc_default_options(method=sc.SC_TGT_PLUS))
    assert e.value.code == sc.SC_ENOTIMPL
    with pytest.raises(sc.ScError) as e:
        sc.sc_batch_all_edges(b, 1e-2, None, sc.sc_default_options(block=3))
    assert e.value.code == sc.SC_EINVAL
    with pytest.raises(sc.ScError) as e:
        sc.sc_batch_all_edges(b, 1.5, None, sc.sc_default_options())
    assert e.value.code == sc.SC_EINVAL
    with pytest.raises(sc.ScError) as e:
        sc.sc_batch_all_edges(b, 1e-2, [3, -1], sc.sc_default_options())
    assert e.value.code == sc.SC_EINVAL
    b.free()
    # a bad graph names its index
    with pytest.raises(sc.ScError) as e:
        sc.sc_build_batch([gg.king_grid(50), (4, np.array([0, 2]), np.array([1, 3]))])
    assert e.value.code == sc.SC_EDISCONNECTED and "graph 1" in str(e.value)
