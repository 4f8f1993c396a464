"""The allocation-free entry point sc_all_edges_static against the allocating
per-source run (sc_all_edges_ex with SC_PER_SOURCE) on the same inputs.

* two calls in a row, the second on a smaller graph: walk counts equal and
  estimates within 1e-12 of the allocating run (the same kernels and walks; the
  slot count and the walk-sum buffer differ, which only reorders sums), while
  any device allocation by the library would fail (a one-byte budget);
* a one-chunk walk-sum buffer (the static call then walks one half per wave);
* a graph whose buffers exceed the static array is refused with SC_EINVAL;
* lambda* must be known beforehand (computing it allocates).
"""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_16086_amd import sc as scmod
    return scmod


def test_static_entry_point_matches_allocating_run_twice(sc, monkeypatch):
    import torch
    cases = [(gg.barabasi_albert(3000, 5, 21), 0.02), (gg.tree_plus_gnp(800, 8.0, 22), 0.03)]
    for (n, u, v), eps in cases:
        print(f"[gpu] static entry n={n} m={len(u)} eps={eps}", flush=True)
        g = sc.sc_build_graph(n, u, v)
        sc.sc_lambda_star(g)   # computing lambda* allocates: before the call
        o = sc.sc_default_options(method=sc.SC_TGT_PLUS, flags=sc.SC_PER_SOURCE, seed=5)
        nr_ref = np.empty(2 * len(u), np.int64)
        ref, st_ref = sc.sc_all_edges_ex(g, eps, 0, o, nr_out=nr_ref)
        out = torch.full((len(u),), -1.0, dtype=torch.float64, device="cuda")
        nr = torch.empty(2 * len(u), dtype=torch.int64, device="cuda")
        tt = torch.empty(n, dtype=torch.int32, device="cuda")
        monkeypatch.setenv("SC_DEVICE_BYTES_LIMIT", "1")
        _, st = sc.sc_all_edges_static(g, eps, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS, seed=5),
                                       out, nr_out=nr, tilde_tau_out=tt)
        torch.cuda.synchronize()
        monkeypatch.delenv("SC_DEVICE_BYTES_LIMIT")
        np.testing.assert_array_equal(nr.cpu().numpy(), nr_ref)
        np.testing.assert_allclose(out.cpu().numpy(), ref, atol=1e-12, rtol=0)
        for k in ("walks", "walk_steps", "push_edges", "tilde_min", "tilde_max", "L_used",
                  "L_min", "L_capped"):
            assert st[k] == st_ref[k], k
        assert tt.cpu().numpy().min() == st["tilde_min"]
        g.free()


def test_static_entry_point_walk_fallback(sc, monkeypatch):
    # a walk-sum buffer of one chunk: the static call walks one half per wave
    import torch
    n, u, v = gg.tree_plus_gnp(500, 8.0, 8)
    print(f"[gpu] static entry, one-chunk walk buffer, n={n} m={len(u)}", flush=True)
    g = sc.sc_build_graph(n, u, v)
    sc.sc_lambda_star(g)
    ref, st_ref = sc.sc_all_edges_ex(
        g, 0.03, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS, flags=sc.SC_PER_SOURCE, seed=5))
    assert st_ref["walks"] > 0
    out = torch.full((len(u),), -1.0, dtype=torch.float64, device="cuda")
    monkeypatch.setenv("SC_SOURCE_PART_CAPACITY", "1")
    monkeypatch.setenv("SC_DEVICE_BYTES_LIMIT", "1")
    _, st = sc.sc_all_edges_static(g, 0.03, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS, seed=5),
                                   out)
    torch.cuda.synchronize()
    monkeypatch.delenv("SC_DEVICE_BYTES_LIMIT")
    monkeypatch.delenv("SC_SOURCE_PART_CAPACITY")
    assert st["walks"] == st_ref["walks"]
    np.testing.assert_allclose(out.cpu().numpy(), ref, atol=1e-12, rtol=0)
    g.free()


def test_static_entry_point_refuses_too_large_graph(sc):
    import torch
    n, u, v = gg.barabasi_albert(400_000, 10, 3)
    g = sc.sc_build_graph(n, u, v)
    out = torch.empty(len(u), dtype=torch.float64, device="cuda")
    with pytest.raises(sc.ScError) as e:
        sc.sc_all_edges_static(g, 1e-2, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS,
                                                                 lambda_star=0.5), out)
    assert e.value.code == sc.SC_EINVAL and "too large" in str(e.value)
    g.free()


def test_static_entry_point_needs_lambda_star(sc):
    import torch
    n, u, v = gg.barabasi_albert(500, 4, 4)
    g = sc.sc_build_graph(n, u, v)
    out = torch.empty(len(u), dtype=torch.float64, device="cuda")
    with pytest.raises(sc.ScError) as e:
        sc.sc_all_edges_static(g, 1e-2, 0, sc.sc_default_options(method=sc.SC_TGT_PLUS), out)
    assert e.value.code == sc.SC_EINVAL and "lambda*" in str(e.value)
    res, _ = sc.sc_all_edges_static(g, 1e-2, 5, sc.sc_default_options(method=sc.SC_TGT_PLUS), out)
    assert torch.isfinite(res).all()
    g.free()
