"""Host-side helpers of bench.py (no GPU): the exact-SC sampler used by the
scalability forms, and the guard that drops the HBM-traffic figure when the
measured kernel source changes."""
import hashlib
import os

import numpy as np

import bench
import graphgen as gg
from oracle import exact as ex


def test_exact_sc_sampled_matches_pseudoinverse():
    for graph in (gg.barabasi_albert(300, 3, 4), gg.king_grid(200), gg.erdos_renyi_nm(150, 900, 2)):
        n, u, v = graph
        ids = np.arange(0, len(u), 7)
        np.testing.assert_allclose(bench.exact_sc_sampled(n, u, v, ids), ex.sc_pinv(n, u, v)[ids],
                                   atol=1e-9, rtol=0)


def test_measured_traffic_tracks_the_kernel_source():
    h = hashlib.sha256()
    for rel in bench.PROP_TRAFFIC_SOURCE[0]:
        with open(os.path.join(bench.ROOT, rel), "rb") as f:
            h.update(f.read())
    digest = h.hexdigest()[:16]
    want = bench.PROP_TRAFFIC_BYTES if digest == bench.PROP_TRAFFIC_SOURCE[1] else None
    assert bench.measured_traffic() == want
    # the committed figure belongs to the committed kernel sources
    assert digest == bench.PROP_TRAFFIC_SOURCE[1]
    assert bench.PROP_TRAFFIC_BYTES > 0


def test_walk_traffic_tracks_the_kernel_source():
    h = hashlib.sha256()
    for rel in bench.WALK_TRAFFIC_SOURCE[0]:
        with open(os.path.join(bench.ROOT, rel), "rb") as f:
            h.update(f.read())
    digest = h.hexdigest()[:16]
    want = bench.WALK_TRAFFIC_BYTES_PER_STEP if digest == bench.WALK_TRAFFIC_SOURCE[1] else None
    assert bench.measured_walk_traffic_per_step() == want
    assert digest == bench.WALK_TRAFFIC_SOURCE[1]
    assert bench.WALK_TRAFFIC_BYTES_PER_STEP >= 20   # at least the algorithmic bytes


def test_bench_refuses_more_than_one_gpu(capsys, monkeypatch):
    import json
    import sys
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in json.loads(capsys.readouterr().out)["error"]
