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


def test_rmat_lcc_simple_connected_seeded_heavy_tailed():
    a = gg.rmat_lcc(12, 16, seed=22)
    b = gg.rmat_lcc(12, 16, seed=22)
    c = gg.rmat_lcc(12, 16, seed=23)
    n, u, v = a
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and a[0] == b[0]
    assert not (a[0] == c[0] and np.array_equal(a[1][:100], c[1][:100]))
    assert n <= 1 << 12 and n > (1 << 12) // 2
    assert simple_edges(n, u, v)
    assert gg.is_connected(n, u, v)
    d = gg.degrees(n, u, v)
    # (a, b, c, d) = (.57, .19, .19, .05) skews the degrees: a hub far above the mean
    assert d.max() > 20 * d.mean()
    # at most 16 * 2^12 generated edges survive symmetrising and deduplication
    assert len(u) <= 16 * (1 << 12)
