"""CPU oracle for all-edge spanning centrality (float64, slow, plain).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the GPU library and its Python
binding never import it.  It shares no code with the GPU path.

* ``oracle.exact``  - exact SC: Laplacian pseudoinverse, spanning-tree
  enumeration, spectral closed forms, sampled block-PCG.
* ``oracle.tgt``    - the method: truncation lengths, truncated traversal,
  candidate bounds, walk counts, Philox walks, TGT+ replay.
* ``oracle.philox`` - Philox4x32-10 from its published definition.
* ``oracle.mlp``    - float64 reference of the learned tail closure network.
"""
