"""ctypes binding of libsc (include/sc.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Host arrays
are numpy; device buffers are torch CUDA tensors (PyTorch is used only for
device memory and streams).  If ``libsc.so`` has not been built the import
fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsc.so")

SC_OK = 0
SC_EINVAL = -1
SC_ESELFLOOP = -2
SC_EDUP = -3
SC_EDISCONNECTED = -4
SC_EBIPARTITE = -5
SC_ENOMEM = -6
SC_EHIP = -7
SC_ENOTIMPL = -8

SC_MERGE_DUPS = 0x2
SC_DEGREE_ORDER = 0x4   # build flags (same bits as the run flags SC_TIME_KERNELS and
SC_BFS_ORDER = 0x8      # SC_GRAPH_REPLAY)
SC_DEVICE_PTRS = 0x1
SC_TIME_KERNELS = 0x4
SC_GRAPH_REPLAY = 0x8
SC_TAU_SPECTRAL = 0x10
SC_PER_SOURCE = 0x20

SC_TGT = 0
SC_TGT_PLUS = 1
SC_LEARNED = 2
MLP_PARAMS = 5313


class ScOptions(C.Structure):
    _fields_ = [
        ("method", C.c_int),
        ("precision", C.c_int),
        ("block", C.c_int),
        ("gamma", C.c_int),
        ("delta", C.c_double),
        ("seed", C.c_uint64),
        ("tilde_tau", C.c_int),
        ("max_L", C.c_int),
        ("lambda_star", C.c_double),
        ("flags", C.c_uint),
        ("stream", C.c_void_p),
        ("tau_out", C.c_void_p),
        ("tilde_tau_out", C.c_void_p),
        ("nr_out", C.c_void_p),
        ("mlp", C.c_void_p),
        ("infer_bf16", C.c_int),
        ("force_fallback", C.c_int),
        ("sources", C.c_void_p),
        ("nsources", C.c_int64),
        ("switch_rule", C.c_int),
    ]


class ScTrainOptions(C.Structure):
    _fields_ = [
        ("epochs", C.c_int),
        ("batch", C.c_int),
        ("lr", C.c_float),
        ("seed", C.c_uint64),
        ("stream", C.c_void_p),
    ]


class ScStats(C.Structure):
    _fields_ = [
        ("L_used", C.c_int),
        ("L_min", C.c_int),
        ("tilde_tau", C.c_int),
        ("block", C.c_int),
        ("lambda_star", C.c_double),
        ("walks", C.c_int64),
        ("walk_steps", C.c_int64),
        ("prop_launches", C.c_int64),
        ("prop_ms", C.c_double),
        ("prop_bytes", C.c_double),
        ("total_ms", C.c_double),
        ("fallback_edges", C.c_int64),
        ("prop_timed", C.c_int64),
        ("host_ms", C.c_double),
        ("L_capped", C.c_int64),
        ("lambda_converged", C.c_int32),
        ("tilde_min", C.c_int32),
        ("tilde_max", C.c_int32),
        ("reserved_", C.c_int32),
        ("push_edges", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ScError(RuntimeError):
    def __init__(self, code, where, text):
        super().__init__(f"{where}: {text} (code {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsc.so not built at {LIB_PATH}; run python -m paper_2305_16086_amd.build")
    lib = C.CDLL(LIB_PATH)
    lib.sc_default_options.argtypes = [C.POINTER(ScOptions)]
    lib.sc_default_options.restype = None
    lib.sc_build_graph.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_uint,
                                   C.POINTER(C.c_void_p)]
    lib.sc_build_graph.restype = C.c_int
    lib.sc_graph_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.sc_graph_size.restype = C.c_int
    lib.sc_free_graph.argtypes = [C.c_void_p]
    lib.sc_free_graph.restype = None
    lib.sc_walk_trace.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                  C.c_uint64, C.c_void_p]
    lib.sc_walk_trace.restype = C.c_int
    lib.sc_lambda_star.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
    lib.sc_lambda_star.restype = C.c_int
    lib.sc_compute_spectrum.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double,
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
    lib.sc_compute_spectrum.restype = C.c_int
    lib.sc_set_spectrum.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    lib.sc_set_spectrum.restype = C.c_int
    lib.sc_get_spectrum.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p]
    lib.sc_get_spectrum.restype = C.c_int
    lib.sc_all_edges.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_void_p]
    lib.sc_all_edges.restype = C.c_int
    lib.sc_all_edges_ex.argtypes = [C.c_void_p, C.c_double, C.c_int, C.POINTER(ScOptions),
                                    C.c_void_p, C.POINTER(ScStats)]
    lib.sc_all_edges_ex.restype = C.c_int
    lib.sc_strerror.argtypes = [C.c_int]
    lib.sc_strerror.restype = C.c_char_p
    lib.sc_last_error.argtypes = []
    lib.sc_last_error.restype = C.c_char_p
    lib.sc_version.argtypes = []
    lib.sc_version.restype = C.c_char_p
    lib.sc_default_train_options.argtypes = [C.POINTER(ScTrainOptions)]
    lib.sc_default_train_options.restype = None
    lib.sc_mlp_create.argtypes = [C.c_uint64, C.POINTER(C.c_void_p)]
    lib.sc_mlp_create.restype = C.c_int
    lib.sc_mlp_free.argtypes = [C.c_void_p]
    lib.sc_mlp_free.restype = None
    lib.sc_mlp_get.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.sc_mlp_get.restype = C.c_int
    lib.sc_mlp_set.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.sc_mlp_set.restype = C.c_int
    lib.sc_all_edges_static.argtypes = [C.c_void_p, C.c_double, C.c_int, C.POINTER(ScOptions),
                                        C.c_void_p, C.POINTER(ScStats)]
    lib.sc_all_edges_static.restype = C.c_int
    lib.sc_mlp_save.argtypes = [C.c_void_p, C.c_char_p]
    lib.sc_mlp_save.restype = C.c_int
    lib.sc_mlp_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
    lib.sc_mlp_load.restype = C.c_int
    lib.sc_closure_dataset.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
    lib.sc_closure_dataset.restype = C.c_int
    lib.sc_closure_features.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
    lib.sc_closure_features.restype = C.c_int
    lib.sc_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.POINTER(ScTrainOptions), C.c_void_p]
    lib.sc_mlp_train.restype = C.c_int
    lib.sc_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                C.c_void_p, C.c_void_p, C.c_void_p]
    lib.sc_mlp_grad.restype = C.c_int
    lib.sc_mlp_predict.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                                   C.c_void_p]
    lib.sc_mlp_predict.restype = C.c_int
    lib.sc_build_batch.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint, C.POINTER(C.c_void_p)]
    lib.sc_build_batch.restype = C.c_int
    lib.sc_batch_size.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.sc_batch_size.restype = C.c_int
    lib.sc_batch_graph.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]
    lib.sc_batch_graph.restype = C.c_int
    lib.sc_free_batch.argtypes = [C.c_void_p]
    lib.sc_free_batch.restype = None
    lib.sc_batch_all_edges.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.POINTER(ScOptions),
                                       C.c_void_p, C.POINTER(ScStats)]
    lib.sc_batch_all_edges.restype = C.c_int
    lib.sc_batch_blocks.argtypes = [C.c_void_p, C.POINTER(ScOptions), C.c_void_p]
    lib.sc_batch_blocks.restype = C.c_int
    lib.sc_batch_autotune.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.POINTER(ScOptions),
                                      C.c_char_p]
    lib.sc_batch_autotune.restype = C.c_int
    lib.sc_batch_load_tuning.argtypes = [C.c_void_p, C.c_char_p]
    lib.sc_batch_load_tuning.restype = C.c_int
    return lib


_lib = _load()

# names declared in include/sc.h, for the export check
EXPORTED = ["sc_default_options", "sc_build_graph", "sc_graph_size", "sc_free_graph",
            "sc_walk_trace",
            "sc_lambda_star", "sc_all_edges", "sc_all_edges_ex", "sc_strerror",
            "sc_last_error", "sc_version", "sc_default_train_options", "sc_mlp_create",
            "sc_mlp_free", "sc_mlp_get", "sc_mlp_set", "sc_closure_dataset",
            "sc_closure_features", "sc_mlp_train", "sc_mlp_grad", "sc_mlp_predict",
            "sc_build_batch", "sc_batch_size", "sc_batch_graph", "sc_free_batch",
            "sc_batch_all_edges", "sc_batch_blocks", "sc_batch_autotune", "sc_batch_load_tuning",
            "sc_compute_spectrum", "sc_set_spectrum", "sc_get_spectrum", "sc_mlp_save",
            "sc_mlp_load", "sc_all_edges_static"]


def _check(rc, where):
    if rc != SC_OK:
        raise ScError(rc, where, _lib.sc_last_error().decode())


def lib():
    return _lib


def sc_version() -> str:
    return _lib.sc_version().decode()


def sc_strerror(code: int) -> str:
    return _lib.sc_strerror(code).decode()


def sc_last_error() -> str:
    return _lib.sc_last_error().decode()


def sc_default_options(**kw) -> ScOptions:
    o = ScOptions()
    _lib.sc_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Graph:
    """Owning wrapper of an sc_graph handle."""

    def __init__(self, handle, n, m):
        self._h = handle
        self.n = n
        self.m = m

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph already freed")
        return self._h

    def free(self):
        if self._h is not None:
            _lib.sc_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sc_build_graph(n, u, v, flags: int = 0) -> Graph:
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    if u.shape != v.shape or u.ndim != 1:
        raise ValueError("u and v must be 1-D arrays of equal length")
    h = C.c_void_p()
    rc = _lib.sc_build_graph(int(n), len(u), u.ctypes.data, v.ctypes.data, int(flags), C.byref(h))
    _check(rc, "sc_build_graph")
    return Graph(h, int(n), len(u))


def sc_graph_size(g: Graph):
    n = C.c_int64()
    m = C.c_int64()
    _check(_lib.sc_graph_size(g.handle, C.byref(n), C.byref(m)), "sc_graph_size")
    return n.value, m.value


def sc_lambda_star(g: Graph) -> float:
    lam = C.c_double()
    _check(_lib.sc_lambda_star(g.handle, C.byref(lam)), "sc_lambda_star")
    return lam.value


def sc_compute_spectrum(g: Graph, omega: int = 128, max_iter: int = 0, tol: float = 0.0):
    """GPU Lanczos for the omega eigenpairs of D^-1/2 A D^-1/2 of largest |lambda|
    (kept in the graph for SC_TAU_SPECTRAL).  Returns (pairs kept, largest residual)."""
    kept = C.c_int()
    res = C.c_double()
    _check(_lib.sc_compute_spectrum(g.handle, int(omega), int(max_iter), float(tol),
                                    C.byref(kept), C.byref(res)), "sc_compute_spectrum")
    return kept.value, res.value


def sc_set_spectrum(g: Graph, lam, phi):
    """Load eigenpairs computed elsewhere: lam[omega], phi[n, omega] (node-major)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    omega = len(lam)
    if phi.shape != (g.n, omega):
        raise ValueError(f"phi must have shape ({g.n}, {omega})")
    _check(_lib.sc_set_spectrum(g.handle, omega, lam.ctypes.data, phi.ctypes.data),
           "sc_set_spectrum")


def sc_get_spectrum(g: Graph):
    """The graph's spectrum: (lam[omega], phi[n, omega]), or None if there is none."""
    omega = C.c_int()
    _check(_lib.sc_get_spectrum(g.handle, C.byref(omega), None, None), "sc_get_spectrum")
    if omega.value == 0:
        return None
    lam = np.empty(omega.value, np.float64)
    phi = np.empty((g.n, omega.value), np.float64)
    _check(_lib.sc_get_spectrum(g.handle, C.byref(omega), lam.ctypes.data, phi.ctypes.data),
           "sc_get_spectrum")
    return lam, phi


def sc_all_edges(g: Graph, eps: float, L: int, out=None) -> np.ndarray:
    if out is None:
        out = np.empty(g.m, dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.shape != (g.m,):
        raise ValueError("out must be a contiguous float64 array of length m")
    _check(_lib.sc_all_edges(g.handle, float(eps), int(L), out.ctypes.data), "sc_all_edges")
    return out


def _ptr(x):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()  # torch tensor


def sc_walk_trace(g: Graph, i: int, j: int, r: int, length: int, seed: int):
    """Nodes visited by walk pair r of half-edge (i -> j): returns (from_i, from_j),
    two int32 arrays of `length` nodes (include/sc.h)."""
    nodes = np.empty(2 * max(int(length), 0), dtype=np.int32)
    rc = _lib.sc_walk_trace(g.handle, int(i), int(j), int(r), int(length),
                            int(seed) & 0xFFFFFFFFFFFFFFFF, nodes.ctypes.data)
    _check(rc, "sc_walk_trace")
    return nodes[:length], nodes[length:]


def sc_all_edges_ex(g: Graph, eps: float, L: int, options: ScOptions | None = None, out=None,
                    tau_out=None, tilde_tau_out=None, nr_out=None, sources=None):
    """Run with explicit options.  ``out`` and the trace arrays are numpy arrays
    (host) or torch CUDA tensors (then SC_DEVICE_PTRS is set and the current
    torch stream is used unless options.stream is set).  ``sources`` (host
    int32 ids, SC_PER_SOURCE only) restricts the computed halves to those
    sources.  Returns (out, stats dict)."""
    o = options if options is not None else sc_default_options()
    src_arr = None
    # the source list is this call's own: the caller's options keep what they held
    # (a pointer to the temporary array must not outlive the call)
    saved_sources = (o.sources, o.nsources)
    if sources is not None:
        src_arr = np.ascontiguousarray(sources, dtype=np.int32)
        o.sources = src_arr.ctypes.data
        o.nsources = len(src_arr)
    try:
        return _all_edges_ex_call(g, eps, L, o, out, tau_out, tilde_tau_out, nr_out)
    finally:
        o.sources, o.nsources = saved_sources


def _all_edges_ex_call(g, eps, L, o, out, tau_out, tilde_tau_out, nr_out):
    device = out is not None and not isinstance(out, np.ndarray)
    if out is None:
        out = np.empty(g.m, dtype=np.float64)
    if device:
        import torch
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() != g.m:
            raise ValueError("device out must be a CUDA float64 tensor of length m")
        o.flags |= SC_DEVICE_PTRS
        if not o.stream:
            o.stream = torch.cuda.current_stream(out.device).cuda_stream
    else:
        if out.dtype != np.float64 or out.shape != (g.m,) or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous float64 array of length m")
        o.flags &= ~SC_DEVICE_PTRS
    for arr, name, n_exp, dt in ((tau_out, "tau_out", g.m, "int32"),
                                 (tilde_tau_out, "tilde_tau_out", g.n, "int32"),
                                 (nr_out, "nr_out", 2 * g.m, "int64")):
        if arr is None:
            continue
        if device == isinstance(arr, np.ndarray):
            raise ValueError(f"{name} must be on the same side (host/device) as out")
        if (arr.numel() if device else arr.size) != n_exp or str(arr.dtype).split(".")[-1] != dt:
            raise ValueError(f"{name} must hold {n_exp} {dt}")
    o.tau_out = _ptr(tau_out)
    o.tilde_tau_out = _ptr(tilde_tau_out)
    o.nr_out = _ptr(nr_out)
    st = ScStats()
    rc = _lib.sc_all_edges_ex(g.handle, float(eps), int(L), C.byref(o), _ptr(out), C.byref(st))
    _check(rc, "sc_all_edges_ex")
    return out, st.as_dict()


def sc_all_edges_static(g: Graph, eps: float, L: int, options: ScOptions, out,
                        tau_out=None, tilde_tau_out=None, nr_out=None):
    """The allocation-free per-source TGT+ call: ``out`` and the traces are CUDA
    tensors (the current torch stream unless options.stream is set).  Returns
    (out, stats dict)."""
    import torch
    o = options
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.numel() == g.m):
        raise ValueError("out must be a CUDA float64 tensor of length m")
    for arr, name, n_exp, dt in ((tau_out, "tau_out", g.m, torch.int32),
                                 (tilde_tau_out, "tilde_tau_out", g.n, torch.int32),
                                 (nr_out, "nr_out", 2 * g.m, torch.int64)):
        if arr is not None and not (isinstance(arr, torch.Tensor) and arr.is_cuda
                                    and arr.dtype == dt and arr.numel() == n_exp):
            raise ValueError(f"{name} must be a CUDA tensor of {n_exp} {dt}")
    o.flags |= SC_DEVICE_PTRS | SC_PER_SOURCE
    if not o.stream:
        o.stream = torch.cuda.current_stream(out.device).cuda_stream
    o.tau_out = _ptr(tau_out)
    o.tilde_tau_out = _ptr(tilde_tau_out)
    o.nr_out = _ptr(nr_out)
    st = ScStats()
    rc = _lib.sc_all_edges_static(g.handle, float(eps), int(L), C.byref(o), _ptr(out), C.byref(st))
    _check(rc, "sc_all_edges_static")
    return out, st.as_dict()


# ---------------------------------------------------------------- learned closure

class Mlp:
    """Owning wrapper of an sc_mlp handle."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("network already freed")
        return self._h

    def free(self):
        if self._h is not None:
            _lib.sc_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _stream_of(t):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _dev(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.numel() != numel \
            or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor with {numel} elements")
    return t.data_ptr()


def sc_default_train_options(**kw) -> ScTrainOptions:
    t = ScTrainOptions()
    _lib.sc_default_train_options(C.byref(t))
    for k, v in kw.items():
        if not hasattr(t, k):
            raise KeyError(k)
        setattr(t, k, v)
    return t


def sc_mlp_create(seed: int = 1) -> Mlp:
    h = C.c_void_p()
    _check(_lib.sc_mlp_create(int(seed), C.byref(h)), "sc_mlp_create")
    return Mlp(h)


def sc_mlp_free(net: Mlp):
    net.free()


def sc_mlp_get(net: Mlp):
    p = np.empty(MLP_PARAMS, np.float32)
    nrm = np.empty(32, np.float32)
    rng = np.empty(32, np.float32)
    _check(_lib.sc_mlp_get(net.handle, p.ctypes.data, nrm.ctypes.data, rng.ctypes.data), "sc_mlp_get")
    return p, nrm, rng


def sc_mlp_set(net: Mlp, params=None, norm=None, range_=None):
    def arr(x, k):
        if x is None:
            return None, None
        a = np.ascontiguousarray(x, dtype=np.float32)
        if a.size != k:
            raise ValueError(f"expected {k} floats")
        return a, a.ctypes.data
    pa, pp = arr(params, MLP_PARAMS)
    na, npp = arr(norm, 32)
    ra, rp = arr(range_, 32)
    _check(_lib.sc_mlp_set(net.handle, pp, npp, rp), "sc_mlp_set")


def sc_mlp_save(net: Mlp, path: str):
    _check(_lib.sc_mlp_save(net.handle, os.fsencode(path)), "sc_mlp_save")


def sc_mlp_load(path: str) -> Mlp:
    h = C.c_void_p()
    _check(_lib.sc_mlp_load(os.fsencode(path), C.byref(h)), "sc_mlp_load")
    return Mlp(h)


def sc_closure_dataset(g: Graph, L_ref: int, precision: int, X, z, w):
    """X: CUDA float32 [m,16]; z, w: CUDA float32 [m]."""
    import torch
    _check(_lib.sc_closure_dataset(g.handle, int(L_ref), int(precision),
                                   _dev(X, torch.float32, 16 * g.m, "X"),
                                   _dev(z, torch.float32, g.m, "z"),
                                   _dev(w, torch.float32, g.m, "w"), _stream_of(X)),
           "sc_closure_dataset")


def sc_closure_features(g: Graph, precision: int, X, s0=None, uK=None, lo=None, hi=None):
    import torch
    ptr = lambda t, nm: None if t is None else _dev(t, torch.float64, g.m, nm)  # noqa: E731
    _check(_lib.sc_closure_features(g.handle, int(precision), _dev(X, torch.float32, 16 * g.m, "X"),
                                    ptr(s0, "s0"), ptr(uK, "uK"), ptr(lo, "lo"), ptr(hi, "hi"),
                                    _stream_of(X)), "sc_closure_features")


def sc_mlp_train(net: Mlp, X, z, w, options: ScTrainOptions | None = None):
    import torch
    N = z.numel()
    t = options if options is not None else sc_default_train_options()
    if not t.stream:
        t.stream = _stream_of(X)
    losses = np.zeros(max(t.epochs, 1), np.float32)
    _check(_lib.sc_mlp_train(net.handle, _dev(X, torch.float32, 16 * N, "X"),
                             _dev(z, torch.float32, N, "z"),
                             None if w is None else _dev(w, torch.float32, N, "w"), N,
                             C.byref(t), losses.ctypes.data), "sc_mlp_train")
    return losses[: t.epochs]


def sc_mlp_grad(net: Mlp, X, z, w=None):
    import torch
    N = z.numel()
    g = np.empty(MLP_PARAMS, np.float32)
    loss = np.empty(1, np.float32)
    _check(_lib.sc_mlp_grad(net.handle, _dev(X, torch.float32, 16 * N, "X"),
                            _dev(z, torch.float32, N, "z"),
                            None if w is None else _dev(w, torch.float32, N, "w"), N,
                            g.ctypes.data, loss.ctypes.data, _stream_of(X)), "sc_mlp_grad")
    return g, float(loss[0])


def sc_mlp_predict(net: Mlp, X, bf16: int = 1, y=None):
    import torch
    N = X.numel() // 16
    if y is None:
        y = torch.empty(N, dtype=torch.float32, device=X.device)
    _check(_lib.sc_mlp_predict(net.handle, _dev(X, torch.float32, 16 * N, "X"), N, int(bf16),
                               _dev(y, torch.float32, N, "y"), _stream_of(X)), "sc_mlp_predict")
    return y


# ---------------------------------------------------------------- batches

class Batch:
    """Owning wrapper of an sc_batch handle; ``graphs[i]`` are borrowed handles."""

    def __init__(self, handle, sizes):
        self._h = handle
        self.sizes = sizes          # [(n, m)] per graph
        self.graphs = []
        for i, (n, m) in enumerate(sizes):
            gh = C.c_void_p()
            _check(_lib.sc_batch_graph(handle, i, C.byref(gh)), "sc_batch_graph")
            g = Graph(gh, n, m)
            g.free = lambda: None       # owned by the batch
            g._h = gh
            self.graphs.append(g)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch already freed")
        return self._h

    def free(self):
        if self._h is not None:
            for g in self.graphs:
                g._h = None
            _lib.sc_free_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sc_build_batch(graphs, flags: int = 0) -> Batch:
    """graphs: list of (n, u, v)."""
    G = len(graphs)
    ns = np.array([int(g[0]) for g in graphs], dtype=np.int64)
    us = [np.ascontiguousarray(g[1], dtype=np.int64) for g in graphs]
    vs = [np.ascontiguousarray(g[2], dtype=np.int64) for g in graphs]
    ms = np.array([len(u) for u in us], dtype=np.int64)
    up = (C.c_void_p * G)(*[u.ctypes.data for u in us])
    vp = (C.c_void_p * G)(*[v.ctypes.data for v in vs])
    h = C.c_void_p()
    rc = _lib.sc_build_batch(G, ns.ctypes.data, ms.ctypes.data, up, vp, int(flags), C.byref(h))
    _check(rc, "sc_build_batch")
    return Batch(h, [(int(ns[i]), int(ms[i])) for i in range(G)])


def _L_array(b: Batch, L):
    if L is None:
        return None
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.int32), (len(b.sizes),)))
    return L


def sc_batch_all_edges(b: Batch, eps: float, L=None, options: ScOptions | None = None,
                       out=None):
    """out: None (host arrays are allocated), a list of numpy arrays, or a list
    of CUDA float64 tensors (then SC_DEVICE_PTRS and the current torch stream).
    Returns (list of outputs, stats dict)."""
    o = options if options is not None else sc_default_options()
    G = len(b.sizes)
    if out is None:
        out = [np.empty(m, dtype=np.float64) for _, m in b.sizes]
    if len(out) != G:
        raise ValueError("need one output per graph")
    device = not isinstance(out[0], np.ndarray)
    for x, (_, m) in zip(out, b.sizes):
        if device:
            import torch
            if isinstance(x, np.ndarray) or x.dtype != torch.float64 or not x.is_cuda or x.numel() != m:
                raise ValueError("device outputs must be CUDA float64 tensors of length m")
        elif not isinstance(x, np.ndarray) or x.dtype != np.float64 or x.shape != (m,) \
                or not x.flags.c_contiguous:
            raise ValueError("host outputs must be contiguous float64 arrays of length m")
    if device:
        import torch
        o.flags |= SC_DEVICE_PTRS
        if not o.stream:
            o.stream = torch.cuda.current_stream(out[0].device).cuda_stream
    else:
        o.flags &= ~SC_DEVICE_PTRS
    ptrs = (C.c_void_p * G)(*[_ptr(x) for x in out])
    La = _L_array(b, L)
    st = ScStats()
    rc = _lib.sc_batch_all_edges(b.handle, float(eps), None if La is None else La.ctypes.data,
                                 C.byref(o), ptrs, C.byref(st))
    _check(rc, "sc_batch_all_edges")
    return out, st.as_dict()


def sc_batch_blocks(b: Batch, options: ScOptions | None = None) -> np.ndarray:
    o = options if options is not None else sc_default_options()
    blocks = np.empty(len(b.sizes), dtype=np.int32)
    _check(_lib.sc_batch_blocks(b.handle, C.byref(o), blocks.ctypes.data), "sc_batch_blocks")
    return blocks


def sc_batch_autotune(b: Batch, eps: float, L=None, options: ScOptions | None = None,
                      json_path: str | None = None):
    o = options if options is not None else sc_default_options()
    La = _L_array(b, L)
    rc = _lib.sc_batch_autotune(b.handle, float(eps), None if La is None else La.ctypes.data,
                                C.byref(o), json_path.encode() if json_path else None)
    _check(rc, "sc_batch_autotune")


def sc_batch_load_tuning(b: Batch, json_path: str):
    _check(_lib.sc_batch_load_tuning(b.handle, json_path.encode()), "sc_batch_load_tuning")
