"""Write the exact SC of sampled edges of the BA n=100k benchmark graph.

Calls only the oracle (float64 block-PCG on the Laplacian, oracle.exact).
Sample: 2048 edges of ``graphgen.workload("ba_100k", 1)``, half uniform, half
weighted by 1/(d_i d_j) so that low-degree edges (largest SC, longest
truncation) are well represented.  Output: ba_100k_seed1_sampled_sc.npz with
``edge_ids`` and ``sc``.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
from oracle import exact as ex  # noqa: E402


def main():
    n, u, v = gg.workload("ba_100k", 1)
    m = len(u)
    d = gg.degrees(n, u, v).astype(np.float64)
    rng = np.random.default_rng(2024)
    uni = rng.choice(m, size=1024, replace=False)
    w = 1.0 / (d[u] * d[v])
    w[uni] = 0.0
    low = rng.choice(m, size=1024, replace=False, p=w / w.sum())
    ids = np.unique(np.concatenate([uni, low]))
    sc = ex.sc_sampled_pcg(n, u, v, ids)
    np.savez(os.path.join(HERE, "ba_100k_seed1_sampled_sc.npz"), edge_ids=ids, sc=sc,
             n=n, m=m)
    print(len(ids), sc.min(), sc.max())


if __name__ == "__main__":
    main()
