"""All-edge spanning centrality (TGT / TGT+) on AMD MI355X.

The computation lives in ``libsc.so`` (hand-written HIP kernels for gfx950
behind the C ABI of ``include/sc.h``); ``paper_2305_16086_amd.sc`` is its
ctypes binding.
"""
from .sc import (  # noqa: F401
    SC_DEVICE_PTRS,
    SC_LEARNED,
    SC_MERGE_DUPS,
    SC_TGT,
    SC_TGT_PLUS,
    SC_TIME_KERNELS,
    Graph,
    ScError,
    sc_all_edges,
    sc_all_edges_ex,
    sc_build_graph,
    sc_default_options,
    sc_graph_size,
    sc_lambda_star,
    sc_last_error,
    sc_strerror,
    sc_version,
    Mlp,
    sc_closure_dataset,
    sc_closure_features,
    sc_default_train_options,
    sc_mlp_create,
    sc_mlp_free,
    sc_mlp_get,
    sc_mlp_grad,
    sc_mlp_predict,
    sc_mlp_set,
    sc_mlp_train,
)
