"""Host-side checks of the C-ABI library that need no GPU: the shared library
loads, exports every entry point include/sc.h declares, and the graph
validation rejects what the paper's definitions exclude (these checks run
before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "sc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    from paper_2305_16086_amd import sc
    lib = ctypes.CDLL(sc.LIB_PATH)
    names = declared_symbols()
    assert "sc_build_graph" in names and "sc_all_edges" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(sc.EXPORTED) == names


def test_version_and_error_texts():
    from paper_2305_16086_amd import sc
    assert "gfx950" in sc.sc_version()
    for code in range(0, -9, -1):
        assert sc.sc_strerror(code) and sc.sc_strerror(code) != "unknown error code"
    assert sc.sc_strerror(-99) == "unknown error code"


def _code(n, u, v, flags=0):
    from paper_2305_16086_amd import sc
    with pytest.raises(sc.ScError) as ei:
        sc.sc_build_graph(n, u, v, flags)
    return ei.value.code


def test_validation_rejects_invalid_graphs():
    from paper_2305_16086_amd import sc
    assert _code(3, [0, 1, 2], [1, 2, 2]) == sc.SC_ESELFLOOP
    assert _code(3, [0, 1, 0, 1], [1, 2, 2, 0]) == sc.SC_EDUP
    assert _code(3, [0, 1, 0], [1, 2, 3]) == sc.SC_EINVAL
    assert _code(3, [0, 1, -1], [1, 2, 2]) == sc.SC_EINVAL
    assert _code(1, [0], [0]) == sc.SC_EINVAL
    assert _code(6, [0, 1, 0, 3, 4, 3], [1, 2, 2, 4, 5, 5]) == sc.SC_EDISCONNECTED
    n, u, v = gg.cycle_graph(6)
    assert _code(n, u, v) == sc.SC_EBIPARTITE
    n, u, v = gg.king_grid(2)   # a single edge
    assert _code(n, u, v) == sc.SC_EBIPARTITE
    assert "bipartite" in sc.sc_last_error()


@pytest.mark.parametrize("order", ["degree", "bfs"])
def test_validation_with_node_order_reports_the_same_errors(order):
    """SC_DEGREE_ORDER and SC_BFS_ORDER renumber after the id checks: every invalid
    graph gets the code it gets without the flag (edge indices in the caller's
    order)."""
    from paper_2305_16086_amd import sc
    f = sc.SC_DEGREE_ORDER if order == "degree" else sc.SC_BFS_ORDER
    assert _code(3, [0, 1, 2], [1, 2, 2], f) == sc.SC_ESELFLOOP
    assert "edge 2" in sc.sc_last_error()
    assert _code(3, [0, 1, 0, 1], [1, 2, 2, 0], f) == sc.SC_EDUP
    assert "edge 3" in sc.sc_last_error()
    assert _code(3, [0, 1, 0], [1, 2, 3], f) == sc.SC_EINVAL
    assert _code(3, [0, 1, -1], [1, 2, 2], f) == sc.SC_EINVAL
    assert _code(1, [0], [0], f) == sc.SC_EINVAL
    assert _code(6, [0, 1, 0, 3, 4, 3], [1, 2, 2, 4, 5, 5], f) == sc.SC_EDISCONNECTED
    n, u, v = gg.cycle_graph(6)
    assert _code(n, u, v, f) == sc.SC_EBIPARTITE


def test_node_orders_exclude_each_other():
    from paper_2305_16086_amd import sc
    n, u, v = gg.complete_graph(4)
    assert _code(n, u, v, sc.SC_DEGREE_ORDER | sc.SC_BFS_ORDER) == sc.SC_EINVAL
    assert "exclude" in sc.sc_last_error()


@pytest.mark.parametrize("order", ["degree", "bfs"])
def test_batch_rejects_node_order(order):
    from paper_2305_16086_amd import sc
    f = sc.SC_DEGREE_ORDER if order == "degree" else sc.SC_BFS_ORDER
    with pytest.raises(sc.ScError) as ei:
        sc.sc_build_batch([gg.complete_graph(4)], f)
    assert ei.value.code == sc.SC_EINVAL
    assert "sc_build_graph only" in sc.sc_last_error()


def test_validation_of_even_cycle_plus_chord_is_not_bipartite_error():
    from paper_2305_16086_amd import sc
    # C6 plus a chord (0, 2) has a triangle; validation must not call it bipartite.
    n, u, v = gg.cycle_graph(6)
    u = np.append(u, 0)
    v = np.append(v, 2)
    try:
        sc.sc_build_graph(n, u, v)
    except sc.ScError as e:       # without a GPU the device upload fails after validation
        assert e.code in (sc.SC_EHIP, sc.SC_ENOMEM)


def test_library_has_no_unresolved_internal_symbols():
    """A shared library links with undefined symbols; every symbol of the
    library's own namespace must be defined in it."""
    import shutil
    import subprocess
    from paper_2305_16086_amd import sc
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    res = subprocess.run([nm, "-D", "--undefined-only", sc.LIB_PATH], capture_output=True,
                         text=True, check=True)
    missing = [ln.split()[-1] for ln in res.stdout.splitlines()
               if ln.split() and (ln.split()[-1].startswith("_ZN2sc") or
                                  ln.split()[-1].startswith("sc_"))]
    assert not missing, missing
