"""Seeded synthetic graph generators.

This package only draws graphs: it holds none of the spanning-centrality
arithmetic, so both the CPU oracle's tests and the GPU path's tests/bench may
use it on the same inputs.  Every generator returns ``(n, u, v)`` with
``u``/``v`` int64 arrays of undirected edges (``u < v``, no duplicates, no
self-loops), sorted by ``(u, v)`` unless stated otherwise.
"""
from .graphs import (  # noqa: F401
    complete_graph,
    cycle_graph,
    petersen_graph,
    triangle_pendant,
    two_triangles_bridge,
    tree_plus_gnp,
    gnp_connected,
    barabasi_albert,
    erdos_renyi_nm,
    ER_EDGES_SERIES,
    ER_NODES_SERIES,
    king_grid,
    mixed_batch,
    rmat_lcc,
    random_small_connected,
    canonical_edges,
    is_connected,
    is_bipartite,
    degrees,
    workload,
)
