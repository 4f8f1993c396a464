"""Pins for the exact-SC oracle (oracle.exact) against facts fixed by the
paper and by graph theory, not against the oracle itself.

* spanning-tree enumeration (Definition 2.1) on tiny graphs;
* closed forms: edge-transitive graphs have s = (n-1)/m, bridges have s = 1;
* Foster's theorem, sum_e s(e) = n - 1;
* the spectral series of Lemma 3.1 / Eq. 18 summed to infinity.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import exact as ex

TINY = [
    ("K4", gg.complete_graph(4)),
    ("K5", gg.complete_graph(5)),
    ("C5", gg.cycle_graph(5)),
    ("C7", gg.cycle_graph(7)),
    ("tri_pendant", gg.triangle_pendant()),
    ("two_tri_bridge", gg.two_triangles_bridge()),
] + [(f"rand{s}", gg.random_small_connected(6, 9, seed=s)) for s in range(4)]


@pytest.mark.parametrize("name,g", TINY, ids=[t[0] for t in TINY])
def test_pinv_matches_spanning_tree_enumeration(name, g):
    n, u, v = g
    s_enum, trees = ex.sc_kirchhoff(n, u, v)
    assert trees == round(ex.reduced_laplacian_det(n, u, v))
    np.testing.assert_allclose(ex.sc_pinv(n, u, v), s_enum, atol=1e-13, rtol=0)


def test_petersen_enumeration_and_closed_form():
    n, u, v = gg.petersen_graph()
    s_enum, trees = ex.sc_kirchhoff(n, u, v)
    assert trees == 2000                       # Petersen graph has 2000 spanning trees
    np.testing.assert_allclose(s_enum, 0.6, atol=1e-15)
    np.testing.assert_allclose(ex.sc_pinv(n, u, v), 0.6, atol=1e-13)


@pytest.mark.parametrize("n", [3, 4, 7, 12, 30])
def test_complete_graph_closed_form(n):
    # edge-transitive: every edge carries (n-1)/m = 2/n
    np.testing.assert_allclose(ex.sc_pinv(*gg.complete_graph(n)), 2.0 / n, atol=1e-12)


@pytest.mark.parametrize("n", [3, 5, 9, 51])
def test_odd_cycle_closed_form(n):
    np.testing.assert_allclose(ex.sc_pinv(*gg.cycle_graph(n)), (n - 1) / n, atol=1e-12)


def test_bridges_have_sc_one():
    n, u, v = gg.triangle_pendant()
    s = ex.sc_pinv(n, u, v)
    bridge = (u == 0) & (v == 3)
    np.testing.assert_allclose(s[bridge], 1.0, atol=1e-13)
    np.testing.assert_allclose(s[~bridge], 2.0 / 3.0, atol=1e-13)
    n, u, v = gg.two_triangles_bridge()
    s = ex.sc_pinv(n, u, v)
    bridge = (u == 2) & (v == 3)
    np.testing.assert_allclose(s[bridge], 1.0, atol=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_foster_and_range_on_workload_graph(seed):
    n, u, v = gg.tree_plus_gnp(400, 10.0, seed)
    s = ex.sc_pinv(n, u, v)
    assert abs(s.sum() - (n - 1)) < 1e-9
    assert s.min() > 0 and s.max() <= 1 + 1e-12
    # tree edges that are bridges must be exactly 1: check against a bridge finder
    import scipy.sparse.csgraph as csg
    ones = np.isclose(s, 1.0, atol=1e-10)
    for e in np.flatnonzero(ones)[:20]:
        keep = np.ones(len(u), bool)
        keep[e] = False
        assert not gg.is_connected(n, u[keep], v[keep])


def test_spectral_series_matches_pinv():
    n, u, v = gg.tree_plus_gnp(300, 8.0, 5)
    np.testing.assert_allclose(ex.sc_eigen(n, u, v), ex.sc_pinv(n, u, v), atol=1e-10)


def test_sampled_pcg_matches_pinv():
    n, u, v = gg.barabasi_albert(600, 4, 3)
    s = ex.sc_pinv(n, u, v)
    ids = np.arange(0, len(u), 7)
    np.testing.assert_allclose(ex.sc_sampled_pcg(n, u, v, ids), s[ids], atol=1e-10)


def test_planted_mistake_is_caught():
    """A wrong sign in the cross term of r(i,j) must break the enumeration pin."""
    n, u, v = gg.two_triangles_bridge()
    s_enum, _ = ex.sc_kirchhoff(n, u, v)
    a = ex.adjacency_dense(n, u, v)
    lap = np.diag(a.sum(1)) - a
    minv = np.linalg.inv(lap + 1.0 / n)
    wrong = minv[u, u] + minv[v, v] + 2.0 * minv[u, v]
    assert np.abs(wrong - s_enum).max() > 1e-3


def test_batch_golden_matches_pseudoinverse_on_small_graphs():
    """The stored sampled SC of the 256-graph batch (written by
    tests/golden/make_batch_oracle.py from the oracle's block-PCG) agrees with
    the dense pseudoinverse on the smallest graph of each family."""
    import os
    import graphgen as gg
    gz = np.load(os.path.join(os.path.dirname(__file__), "golden", "batch_256_seed7_sampled_sc.npz"))
    graphs = gg.workload("batch_256", 7)
    assert len(np.unique(gz["graph"])) == 256
    for fam in range(3):
        k = min((i for i in range(256) if i % 3 == fam), key=lambda i: graphs[i][0])
        n, u, v = graphs[k]
        sel = gz["graph"] == k
        np.testing.assert_allclose(gz["sc"][sel], ex.sc_pinv(n, u, v)[gz["edge_ids"][sel]],
                                   atol=1e-9, rtol=0)


def test_sampled_pcg_torch_products_match_pseudoinverse():
    import graphgen as gg
    n, u, v = gg.barabasi_albert(400, 3, 8)
    ids = np.arange(0, len(u), 5)
    want = ex.sc_pinv(n, u, v)[ids]
    np.testing.assert_allclose(ex.sc_sampled_pcg(n, u, v, ids, block=64, spmm="torch"), want,
                               atol=1e-9, rtol=0)
