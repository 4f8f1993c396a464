"""Write the exact SC of sampled edges of the Orkut-shaped benchmark graph.

Calls only the oracle (float64 block-PCG on the Laplacian, oracle.exact; the
sparse products through PyTorch's CPU CSR matmul).  Graph:
``graphgen.barabasi_albert(3072441, 38, seed=1)`` (the node count of the
paper's Orkut dataset, m/n rounded).  Sample: 512 edges, half
uniform, half weighted by 1/(d_i d_j) (low-degree edges, the longest
truncations).  Relative residual 1e-10.  Output: orkut_shaped_sampled_sc.npz
with ``edge_ids``, ``sc``, ``n`` and ``m``.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
from oracle import exact as ex  # noqa: E402


def main():
    n, u, v = gg.barabasi_albert(3_072_441, 38, 1)
    m = len(u)
    d = gg.degrees(n, u, v).astype(np.float64)
    rng = np.random.default_rng(3072)
    uni = rng.choice(m, size=256, replace=False)
    w = 1.0 / (d[u] * d[v])
    w[uni] = 0.0
    low = rng.choice(m, size=256, replace=False, p=w / w.sum())
    ids = np.unique(np.concatenate([uni, low]))
    sc = ex.sc_sampled_pcg(n, u, v, ids, tol=1e-10, block=64, spmm="torch")
    np.savez(os.path.join(HERE, "orkut_shaped_sampled_sc.npz"), edge_ids=ids, sc=sc, n=n, m=m)
    print(len(ids), sc.min(), sc.max(), flush=True)


if __name__ == "__main__":
    main()
