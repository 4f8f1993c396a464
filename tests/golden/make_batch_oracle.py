"""Write the exact SC of sampled edges of every graph of the 256-graph batch.

Calls only the oracle (float64 block-PCG on the Laplacian, oracle.exact).
Sample per graph: 16 edges - 4 incident to a node of the smallest degree
(grid corners and borders, BA and G(n,p) leaves), 4 incident to a node of the
largest degree, 8 uniform - deduplicated.  Output: batch_256_seed7_sampled_sc.npz
with ``graph`` (index), ``edge_ids`` (edge number within its graph) and ``sc``.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
from oracle import exact as ex  # noqa: E402


def sample(n, u, v, rng):
    m = len(u)
    d = gg.degrees(n, u, v)
    lo = np.nonzero((d[u] == d.min()) | (d[v] == d.min()))[0]
    hi = np.nonzero((d[u] == d.max()) | (d[v] == d.max()))[0]
    pick = [rng.choice(lo, size=min(4, len(lo)), replace=False),
            rng.choice(hi, size=min(4, len(hi)), replace=False),
            rng.choice(m, size=8, replace=False)]
    return np.unique(np.concatenate(pick))


def main():
    graphs = gg.workload("batch_256", 7)
    rng = np.random.default_rng(256)
    gi, ei, sc = [], [], []
    for k, (n, u, v) in enumerate(graphs):
        ids = sample(n, u, v, rng)
        s = ex.sc_sampled_pcg(n, u, v, ids, max_iter=50000)
        gi.append(np.full(len(ids), k))
        ei.append(ids)
        sc.append(s)
        print(k, n, len(u), len(ids), float(s.min()), float(s.max()), flush=True)
    np.savez(os.path.join(HERE, "batch_256_seed7_sampled_sc.npz"), graph=np.concatenate(gi),
             edge_ids=np.concatenate(ei), sc=np.concatenate(sc))


if __name__ == "__main__":
    main()
