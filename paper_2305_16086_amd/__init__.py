"""All-edge spanning centrality (TGT / TGT+) on AMD MI355X.

The computation lives in ``libsc.so`` (hand-written HIP kernels for gfx950
behind the C ABI of ``include/sc.h``); ``paper_2305_16086_amd.sc`` is its
ctypes binding.  The package re-exports the binding's names lazily, so that
``paper_2305_16086_amd.build`` can be imported (and run) before the library
exists; any use of the API loads the library and fails loudly without it.
"""
_EXPORTS = (
    "SC_DEVICE_PTRS", "SC_LEARNED", "SC_MERGE_DUPS", "SC_TGT", "SC_TGT_PLUS",
    "SC_TIME_KERNELS", "SC_GRAPH_REPLAY", "SC_TAU_SPECTRAL", "Graph", "ScError",
    "sc_all_edges", "sc_all_edges_ex", "sc_build_graph", "sc_default_options",
    "sc_graph_size", "sc_lambda_star", "sc_last_error", "sc_strerror", "sc_version",
    "Mlp", "sc_closure_dataset", "sc_closure_features", "sc_default_train_options",
    "sc_mlp_create", "sc_mlp_free", "sc_mlp_get", "sc_mlp_grad", "sc_mlp_predict",
    "sc_mlp_set", "sc_mlp_train", "sc_build_batch", "sc_batch_all_edges",
    "sc_compute_spectrum", "sc_set_spectrum", "sc_get_spectrum",
)


def __getattr__(name):
    if name in _EXPORTS:
        from . import sc as _sc
        return getattr(_sc, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")


def __dir__():
    return sorted(list(globals()) + list(_EXPORTS))
