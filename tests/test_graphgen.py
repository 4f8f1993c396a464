"""Seeded generators: sizes, simplicity, connectivity, reproducibility."""
import numpy as np
import pytest

import graphgen as gg


def simple_edges(n, u, v):
    assert np.all(u < v) and np.all(u >= 0) and np.all(v < n)
    key = u.astype(np.int64) * n + v
    return len(np.unique(key)) == len(key)


@pytest.mark.parametrize("n,m", [(50, 200), (2_000, 40_000), (500, 124_000)])
def test_erdos_renyi_nm_exact_count_simple_connected(n, m):
    n2, u, v = gg.erdos_renyi_nm(n, m, 3)
    assert n2 == n and len(u) == m   # connected at these densities: no linking edges
    assert simple_edges(n, u, v)
    assert gg.is_connected(n, u, v) and not gg.is_bipartite(n, u, v)


def test_erdos_renyi_nm_is_seeded_and_uniform_in_degree():
    a = gg.erdos_renyi_nm(1_000, 20_000, 5)
    b = gg.erdos_renyi_nm(1_000, 20_000, 5)
    c = gg.erdos_renyi_nm(1_000, 20_000, 6)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert not np.array_equal(a[1], c[1])
    d = gg.degrees(*a)
    # G(n, m) degrees are close to Binomial(n-1, 2m/(n(n-1))): mean 40, sd ~ 6
    assert abs(d.mean() - 40.0) < 1e-9 and 3.0 < d.std() < 9.0


def test_erdos_renyi_nm_links_stray_components():
    # very sparse: isolated nodes are joined to the giant component
    n, u, v = gg.erdos_renyi_nm(400, 300, 1)
    assert gg.is_connected(n, u, v) and len(u) > 300
    assert simple_edges(n, u, v)


def test_erdos_renyi_nm_rejects_too_many_edges():
    with pytest.raises(ValueError):
        gg.erdos_renyi_nm(10, 46, 1)


def test_er_series_sizes():
    assert gg.ER_EDGES_SERIES == [(10_000, m) for m in (200_000, 500_000, 1_000_000, 2_000_000,
                                                        5_000_000)]
    assert gg.ER_NODES_SERIES == [(n, 1_000_000) for n in (2_000, 5_000, 10_000, 20_000, 50_000)]
