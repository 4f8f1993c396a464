#!/usr/bin/env python3
"""All-edge spanning centrality throughput on one MI355X.

Workload: Barabasi-Albert graph, n = 100,000 nodes, 10 edges per new node
(999,945 edges), seed 1; TGT+ with FP32 propagation and FP64 per-edge sums,
eps = 1e-3, truncation from the lambda* bound (L = 0), source block 64.

One step = one call of sc_all_edges_ex over the whole graph (truncation
policy, switch-point cost model, traversal, candidate bounds, walk counts,
walks and edge combine), with the graph already resident on the GPU and the
output written to device memory.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-edge SC edges/sec at max abs err ≤1e-2 vs FP64 oracle; learned vs plain"
EPS = 1e-3
SEED = 1
BLOCK = 64
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "ba_100k_seed1_sampled_sc.npz")
# HBM bytes per k_propagate launch on this workload (the generator's node order) from the
# FETCH_SIZE / WRITE_SIZE counters, scaled by kernels of known traffic
# (profiles/hbm_ba100k_k_propagate.md); valid only for the
# kernel sources they were taken on (first 16 hex digits of the SHA-256 of the files in order)
PROP_TRAFFIC_BYTES = 419604636
PROP_TRAFFIC_SOURCE = (("paper_2305_16086_amd/csrc/kernels_tgt.hip",
                        "paper_2305_16086_amd/csrc/accumulate.hpp"), "a7a719226577e17d")


# Fabric bytes per single-walk step of the per-source walk kernel on R-MAT scale 22 with the
# nodes in degree order (the timed 4,096-source call), from the same counters and scale
# factors (profiles/hbm_rmat22_k_src_walks.md); valid only for the sources they were taken on
WALK_TRAFFIC_BYTES_PER_STEP = 252.0
WALK_TRAFFIC_SOURCE = (("paper_2305_16086_amd/csrc/kernels_sparse.hip",
                        "paper_2305_16086_amd/csrc/philox.hpp"), "250d6397ae5e35f7")


def node_order_flag(sc, order):
    """Build flag and JSON description of a --node-order value."""
    if order == "degree":
        return sc.SC_DEGREE_ORDER, "degree (SC_DEGREE_ORDER: stored by descending degree)"
    if order == "bfs":
        return sc.SC_BFS_ORDER, "bfs (SC_BFS_ORDER: stored in breadth-first order from the top hub)"
    return 0, "the generator's"


def traffic_source_digest(files=PROP_TRAFFIC_SOURCE[0]):
    import hashlib
    h = hashlib.sha256()
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    return PROP_TRAFFIC_BYTES if traffic_source_digest() == PROP_TRAFFIC_SOURCE[1] else None


def measured_walk_traffic_per_step():
    ok = traffic_source_digest(WALK_TRAFFIC_SOURCE[0]) == WALK_TRAFFIC_SOURCE[1]
    return WALK_TRAFFIC_BYTES_PER_STEP if ok else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sources", type=int, default=1500,
                   help="sources in the CPU-baseline sample (about 10-15 s of CPU work)")
    p.add_argument("--form", choices=["plain", "batch", "learned", "er", "eps", "caltau",
                                      "params", "rmat", "orkut"],
                   default="plain",
                   help="plain: the BA-100k TGT+ line; batch: 256 mixed graphs in one "
                        "persistent launch against one graph at a time; learned: the "
                        "learned tail closure against plain TGT+ on BA-100k")
    p.add_argument("--train-graphs", type=int, default=16, help="learned: training graphs")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="plain: one untimed device-to-device copy of this many MB (a kernel "
                        "of known traffic, to scale HBM counters)")
    p.add_argument("--er-eps", type=float, default=0.05, help="er: error bound eps")
    p.add_argument("--check-edges", type=int, default=16,
                   help="er/eps: sampled edges checked against exact SC (conjugate gradients)")
    p.add_argument("--replay", action="store_true", help="batch: replay a captured hipGraph")
    p.add_argument("--rmat-scale", type=int, default=22, help="rmat: R-MAT scale")
    p.add_argument("--orkut-eps", type=float, default=1e-3,
                   help="orkut: error bound eps (at 1e-2 lambda* = 0.23 keeps tau at 1)")
    p.add_argument("--switch-rule", type=int, default=0, choices=[0, 1],
                   help="rmat, orkut: Eq. 14 as printed (0) or weighing walks by their steps (1)")
    p.add_argument("--full-call-limit", type=float, default=150.0,
                   help="rmat, orkut: time the whole call when the sample extrapolates below this (s)")
    p.add_argument("--node-order", default=None, choices=["generator", "degree", "bfs"],
                   help="how the library stores the nodes (build flags SC_DEGREE_ORDER, "
                        "SC_BFS_ORDER; the input and the ids at the interface are unchanged); "
                        "default: the generator's for plain, degree for rmat and orkut")
    p.add_argument("--rmat-sources", type=int, default=4096,
                   help="rmat: uniform random sources timed (the full call is extrapolated)")
    p.add_argument("--no-extras", action="store_true",
                   help="plain: skip the comparison forms carried in the line (learned closure, "
                        "TGT+ at eps=1e-5, per-source TGT+, the 256-graph batch)")
    p.add_argument("--tune-json", default=None, help="batch: tuning table (written if absent)")
    return p.parse_args()


def cpu_baseline(graph, tau, tilde, nr, nsrc):
    """The oracle's TGT+ (replay with the GPU's switch step and walk counts)
    from a random sample of sources, scaled to the whole graph."""
    from oracle import tgt as otgt
    n, u, v = graph
    m = len(u)
    rng = np.random.default_rng(7)
    srcs = rng.choice(n, size=nsrc, replace=False)
    G = otgt.Graph(n, u, v)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):   # one core, as reported
        t0 = time.perf_counter()
        otgt.tgt_plus_replay(G, tau, tilde, nr[:m], nr[m:], seed=0x5C5C, sources=srcs)
        dt = time.perf_counter() - t0
    full = dt * n / nsrc
    return {"value": m / full, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"TGT+ replay (float64, scipy sparse, single thread) from {nsrc} random "
                      f"sources with all their half-edges, {dt:.1f} s, scaled by n/{nsrc} to all "
                      f"{m} edges", "host_cpus": os.cpu_count()}


BATCH_EPS = 1e-2
TUNING = os.path.join(ROOT, "paper_2305_16086_amd", "tuning", "batch_fp32_mi355x.json")
BATCH_MAX_L = 31
LDS_PEAK_GBS = 128 * 256 * 2.4   # 128 B per clock per CU, 256 CUs, 2.4 GHz


def batch_form(a):
    """256 graphs (n uniform in [200, 20000]; G(n,p) deg 8, BA m=5, king grid)
    by TGT at eps = 1e-2 with the automatic truncation capped at 31: one
    persistent launch per step against the same graphs one at a time (TGT and
    TGT+ through sc_all_edges_ex)."""
    import tempfile
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg
    from oracle import exact as ex

    graphs = gg.workload("batch_256", 7)
    M = sum(len(g[1]) for g in graphs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    b = sc.sc_build_batch(graphs)
    outs = [torch.empty(len(g[1]), dtype=torch.float64, device=dev) for g in graphs]

    def opts(**kw):
        return sc.sc_default_options(method=sc.SC_TGT, precision=0, max_L=BATCH_MAX_L,
                                     stream=stream.cuda_stream, **kw)

    path = a.tune_json or (TUNING if os.path.exists(TUNING)
                           else os.path.join(tempfile.gettempdir(), "sc_batch_tuning.json"))
    print(f"[batch] built {len(graphs)} graphs", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(), out=outs)   # lambda* of every graph
    torch.cuda.synchronize()
    pre_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    if os.path.exists(path):
        sc.sc_batch_load_tuning(b, path)
    else:
        sc.sc_batch_autotune(b, BATCH_EPS, None, opts(), path)
    tune_s = time.perf_counter() - t0
    print(f"[batch] tuning {path} ({tune_s:.1f} s)", file=sys.stderr, flush=True)
    blocks = sc.sc_batch_blocks(b, opts())
    flags = sc.SC_GRAPH_REPLAY if a.replay else 0
    for _ in range(a.warmup):
        sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(flags=flags), out=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(flags=flags), out=outs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    _, kst = sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(flags=sc.SC_TIME_KERNELS), out=outs)
    res = [o.cpu().numpy() for o in outs]
    print(f"[batch] timed {1e3 * dt:.1f} ms per step", file=sys.stderr, flush=True)
    if a.no_cpu_baseline and a.steps <= 1:
        # short profiling runs stop after the batched launches
        print(json.dumps({"batch_ms_per_step": 1e3 * dt, "kernel_ms": kst["prop_ms"]}), flush=True)
        return

    # certified configuration: CalTau (Algorithm 1) for the king grids from their
    # device spectra (omega = 128), the lambda*-bound uncapped (255) elsewhere
    t0 = time.perf_counter()
    spec = []
    for i in range(len(graphs)):
        if i % 3 == 2:
            kept, res_ = sc.sc_compute_spectrum(b.graphs[i], 128, 2048, 1e-8)
            spec.append((i, kept, res_))
            print(f"[batch] spectrum {len(spec)}: grid n={graphs[i][0]}, {kept} pairs "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    spec_s = time.perf_counter() - t0
    print(f"[batch] spectra of {len(spec)} grids: {spec_s:.1f} s", file=sys.stderr, flush=True)

    def copts(**kw):
        return sc.sc_default_options(method=sc.SC_TGT, precision=0, stream=stream.cuda_stream,
                                     flags=sc.SC_TAU_SPECTRAL, **kw)

    sc.sc_batch_all_edges(b, BATCH_EPS, None, copts(), out=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, cst = sc.sc_batch_all_edges(b, BATCH_EPS, None, copts(), out=outs)
    torch.cuda.synchronize()
    cdt = (time.perf_counter() - t0) / a.steps
    cres = [o.cpu().numpy() for o in outs]
    golden = None
    if os.path.exists(BATCH_GOLDEN):
        gz = np.load(BATCH_GOLDEN)
        golden = list(zip(gz["graph"], gz["edge_ids"], gz["sc"]))
    certified = {"ms": 1e3 * cdt, "edges_per_s": M / cdt, "L_capped": cst["L_capped"],
                 "L_used": cst["L_used"], "spectra_s": spec_s,
                 "omega_kept_min": int(min(k for _, k, _ in spec)) if spec else None,
                 "max_abs_err_sampled_all_graphs":
                     max(float(abs(cres[k][e] - v)) for k, e, v in golden) if golden else None}
    print(f"[batch] certified: {1e3 * cdt:.1f} ms per step, L_capped {cst['L_capped']}",
          file=sys.stderr, flush=True)

    # one graph at a time, same accuracy target
    single = {}
    taus = []
    for name, method in (("tgt", sc.SC_TGT), ("tgt_plus", sc.SC_TGT_PLUS)):
        vals = [torch.empty_like(o) for o in outs]
        tau = [torch.empty(len(g[1]), dtype=torch.int32, device=dev) for g in graphs]
        for i, g in enumerate(b.graphs):   # warm: per-graph buffers and plans
            o = sc.sc_default_options(method=method, precision=0, max_L=BATCH_MAX_L,
                                      stream=stream.cuda_stream)
            sc.sc_all_edges_ex(g, BATCH_EPS, 0, o, out=vals[i], tau_out=tau[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, g in enumerate(b.graphs):
            o = sc.sc_default_options(method=method, precision=0, max_L=BATCH_MAX_L,
                                      stream=stream.cuda_stream)
            sc.sc_all_edges_ex(g, BATCH_EPS, 0, o, out=vals[i])
        torch.cuda.synchronize()
        s = time.perf_counter() - t0
        single[name] = {"value": M / s, "ms": 1e3 * s,
                        "vals": [x.cpu().numpy() for x in vals]}
        if method == sc.SC_TGT:
            taus = [t.cpu().numpy() for t in tau]
    agree = max(float(np.abs(r - t).max()) for r, t in zip(res, single["tgt"]["vals"]))

    errs_all = None
    if golden:
        errs_all = {"batch": max(float(abs(res[k][e] - v)) for k, e, v in golden)}
        for k_ in ("tgt", "tgt_plus"):
            errs_all[k_] = max(float(abs(single[k_]["vals"][k][e] - v)) for k, e, v in golden)
    # exact SC on the smallest graphs of each family
    errs = {"batch": 0.0, "tgt": 0.0, "tgt_plus": 0.0}
    checked = []
    for fam in range(3):
        idx = sorted([i for i in range(len(graphs)) if i % 3 == fam],
                     key=lambda i: graphs[i][0])[:3]
        for i in idx:
            n, u, v = graphs[i]
            exact = ex.sc_pinv(n, u, v)
            errs["batch"] = max(errs["batch"], float(np.abs(res[i] - exact).max()))
            for k in ("tgt", "tgt_plus"):
                errs[k] = max(errs[k], float(np.abs(single[k]["vals"][i] - exact).max()))
            checked.append(int(n))

    # algorithmic bytes of the persistent launches: per item and step l = 2..tmax,
    # neighbour values read (2m B) and rows written (n B), FP32
    alg = 0.0
    for i, (n, u, v) in enumerate(graphs):
        tr = np.zeros(n, np.int64)
        np.maximum.at(tr, u, taus[i])
        np.maximum.at(tr, v, taus[i])
        B = int(blocks[i])
        nblk = (n + B - 1) // B
        tb = np.zeros(nblk * B, np.int64)
        tb[:n] = tr
        tmax = tb.reshape(nblk, B).max(axis=1)
        steps = np.maximum(tmax - 1, 0).sum()
        alg += steps * (2 * len(u) + n) * B * 4.0
    kms = kst["prop_ms"]
    achieved = alg / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    hist = {int(k): int(c) for k, c in zip(*np.unique(blocks, return_counts=True))}
    line = {
        "metric": METRIC,
        "value": M / dt,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batch_256: 256 graphs, n uniform in [200, 20000], G(n,p) deg 8 / "
                        f"BA m=5 / king grid (seed 7), sum n={sum(g[0] for g in graphs)}, "
                        f"sum m={M}; TGT, eps=1e-2, lambda* truncation capped at "
                        f"{BATCH_MAX_L}, FP32 propagation, FP64 sums",
            "replay": bool(a.replay),
            "blocks": hist,
            "one_at_a_time_tgt_edges_per_s": single["tgt"]["value"],
            "one_at_a_time_tgt_plus_edges_per_s": single["tgt_plus"]["value"],
            "max_abs_diff_vs_one_at_a_time_tgt": agree,
            "max_abs_err_exact": errs,
            "exact_checked_n": checked,
            "max_abs_err_sampled_all_graphs": errs_all,
            "err_sample": "16 edges of each of the 256 graphs, exact SC by float64 block-PCG",
            "L_capped": kst["L_capped"],
            "certified_caltau": certified,
            "L_used": kst["L_used"], "L_min": kst["L_min"],
            "preprocess_s": pre_s, "tune_s": tune_s,
        },
        "roofline": {
            "bound": "lds",
            "kernel": "k_batch (persistent, block states in LDS)",
            "achieved": achieved,
            "peak": LDS_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / LDS_PEAK_GBS,
            "traffic": None,
            "kernel_ms": kms,
            "alg_bytes": alg,
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def learned_form(a):
    """Learned tail closure (MLP 16-64-64-1, FP32 training on the GPU, BF16
    inference) against plain TGT+ on the BA-100k graph at eps = 1e-3.
    Training data: BA (m in {5, 10}) and G(n,p) (average degree 8, 10) graphs
    with n log-uniform in [1e4, 1e5], seeds 100.., targets from TGT at L = 201
    (untimed).  Both methods are timed on the same resident graph; accuracy on
    the 2048 sampled edges whose exact SC the oracle stored."""
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    rng = np.random.default_rng(100)
    t0 = time.perf_counter()
    Xs, zs, ws = [], [], []
    train_sizes = []
    for k in range(a.train_graphs):
        n = int(round(10 ** rng.uniform(4.0, 5.0)))
        seed = 100 + k
        if k % 2 == 0:
            graph = gg.barabasi_albert(n, 5 if k % 4 == 0 else 10, seed)
        else:
            graph = gg.gnp_connected(n, 8.0 if k % 4 == 1 else 10.0, seed)
        n, u, v = graph
        g = sc.sc_build_graph(n, u, v)
        m = len(u)
        X = torch.empty(m * 16, dtype=torch.float32, device=dev)
        z = torch.empty(m, dtype=torch.float32, device=dev)
        w = torch.empty(m, dtype=torch.float32, device=dev)
        sc.sc_closure_dataset(g, 201, 0, X, z, w)
        torch.cuda.synchronize()
        g.free()
        Xs.append(X)
        zs.append(z)
        ws.append(w)
        train_sizes.append((n, m))
        print(f"[learned] dataset {k}: n={n} m={m} {time.perf_counter() - t0:.1f}s",
              file=sys.stderr, flush=True)
    data_s = time.perf_counter() - t0
    X = torch.cat(Xs)
    z = torch.cat(zs)
    w = torch.cat(ws)
    del Xs, zs, ws
    net = sc.sc_mlp_create(7)
    t0 = time.perf_counter()
    losses = sc.sc_mlp_train(net, X, z, w, sc.sc_default_train_options(epochs=30, batch=4096))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, z, w

    graph = gg.workload("ba_100k", SEED)
    n, u, v = graph
    m = len(u)
    g = sc.sc_build_graph(n, u, v)
    out = torch.empty(m, dtype=torch.float64, device=dev)
    gz = np.load(GOLDEN) if os.path.exists(GOLDEN) else None

    def run(method, **kw):
        o = sc.sc_default_options(method=method, precision=0, block=BLOCK,
                                  stream=stream.cuda_stream, **kw)
        return sc.sc_all_edges_ex(g, EPS, 0, o, out=out)[1]

    def run_eps(method, eps, **kw):
        o = sc.sc_default_options(method=method, precision=0, block=BLOCK,
                                  stream=stream.cuda_stream, **kw)
        return sc.sc_all_edges_ex(g, eps, 0, o, out=out)[1]

    res = {}
    for name, method, eps, kw in (("learned", sc.SC_LEARNED, EPS, {"mlp": net.handle.value}),
                                  ("tgt_plus", sc.SC_TGT_PLUS, EPS, {}),
                                  ("tgt", sc.SC_TGT, EPS, {}),
                                  ("tgt_eps_1e-5", sc.SC_TGT, 1e-5, {})):
        for _ in range(a.warmup):
            run_eps(method, eps, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            st = run_eps(method, eps, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        vals = out.cpu().numpy()
        err = float(np.abs(vals[gz["edge_ids"]] - gz["sc"]).max()) if gz is not None else None
        res[name] = {"edges_per_s": m / dt, "ms": 1e3 * dt, "max_abs_err_sampled": err,
                     "fallback_edges": st["fallback_edges"], "L_used": st["L_used"]}
    line = {
        "metric": METRIC,
        "value": res["learned"]["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["learned"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"ba_100k: Barabasi-Albert n=100000, 10 edges per new node, seed 1 "
                        f"(m={m}); learned tail closure (L0=8, MLP 16-64-64-1, BF16 inference, "
                        f"certified fallback to TGT), eps=1e-3, FP32 propagation",
            "learned": res["learned"], "plain_tgt_plus": res["tgt_plus"], "plain_tgt": res["tgt"],
            "plain_tgt_eps_1e-5": res["tgt_eps_1e-5"],
            "train": {"graphs": train_sizes, "samples": int(sum(mm for _, mm in train_sizes)),
                      "dataset_s": data_s, "train_s": train_s,
                      "loss_first": float(losses[0]), "loss_last": float(losses[-1])},
        },
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def exact_sc_sampled(n, u, v, ids):
    """Exact SC of the edges ids: (e_i - e_j)^T L^+ (e_i - e_j) by Jacobi-preconditioned
    conjugate gradients on the Laplacian in float64 (the right-hand sides sum to
    zero, so the singular system is consistent)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    uu = np.concatenate([u, v])
    vv = np.concatenate([v, u])
    A = sp.csr_matrix((np.ones(len(uu)), (uu, vv)), shape=(n, n))
    d = np.asarray(A.sum(axis=1)).ravel()
    Lap = sp.diags(d) - A
    M = sp.diags(1.0 / d)
    out = np.empty(len(ids))
    for t, e in enumerate(ids):
        b = np.zeros(n)
        b[u[e]] = 1.0
        b[v[e]] = -1.0
        x, info = sla.cg(Lap, b, rtol=1e-12, atol=0.0, maxiter=10 * n, M=M)
        if info != 0:
            raise RuntimeError(f"conjugate gradients did not converge on edge {e}")
        out[t] = x[u[e]] - x[v[e]]
    return out


def timed_calls(sc, g, eps, o, out, steps, warmup):
    import torch
    for _ in range(warmup):
        sc.sc_all_edges_ex(g, eps, 0, o, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = sc.sc_all_edges_ex(g, eps, 0, o, out=out)[1]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, st


def er_form(a):
    """Scalability on Erdos-Renyi graphs G(n, m) (seed 1): n = 10^4 with m = 0.2, 0.5,
    1, 2, 5 x 10^6, and m = 10^6 with n = 2, 5, 10, 20, 50 x 10^3 (the sizes of the
    paper's scalability tables); TGT+, FP32 propagation, block 64, eps = --er-eps.
    Graph build and lambda* are preprocessing (not timed).  Accuracy on
    --check-edges sampled edges against exact SC by conjugate gradients."""
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    rng = np.random.default_rng(7)
    rows = []
    for series, sizes in (("edges", gg.ER_EDGES_SERIES), ("nodes", gg.ER_NODES_SERIES)):
        for n, m_target in sizes:
            n, u, v = gg.erdos_renyi_nm(n, m_target, SEED)
            m = len(u)
            g = sc.sc_build_graph(n, u, v)
            out = torch.empty(m, dtype=torch.float64, device=dev)
            o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, block=BLOCK,
                                      stream=stream.cuda_stream)
            dt, st = timed_calls(sc, g, a.er_eps, o, out, a.steps, a.warmup)
            ids = rng.choice(m, size=min(a.check_edges, m), replace=False)
            err = float(np.abs(out.cpu().numpy()[ids] - exact_sc_sampled(n, u, v, ids)).max())
            g.free()
            row = {"series": series, "n": n, "m": m, "ms": 1e3 * dt, "edges_per_s": m / dt,
                   "max_abs_err_sampled": err, "L_used": st["L_used"],
                   "tilde_tau": st["tilde_tau"], "lambda_star": st["lambda_star"],
                   "walks": st["walks"],
                   # tau = 1 everywhere: the call is the closed-form l = 0, 1 terms only
                   "closed_form_only": st["L_used"] <= 1}
            rows.append(row)
            print(f"[er] {series} n={n} m={m}: {1e3 * dt:.1f} ms, err {err:.2e}, "
                  f"L={st['L_used']} tilde={st['tilde_tau']}", file=sys.stderr, flush=True)
    head = rows[[r["series"] == "nodes" and r["n"] == 10_000 for r in rows].index(True)]
    line = {
        "metric": "all-edge SC edges/sec (TGT+) on Erdos-Renyi graphs",
        "value": head["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Erdos-Renyi G(n, m) scalability series, seed {SEED}; "
                               f"value = the n=10^4, m=10^6 graph; TGT+, eps={a.er_eps}, "
                               f"FP32 propagation, block 64", "eps": a.er_eps, "rows": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def eps_form(a):
    """Error-bound sweep eps in {0.05, 0.02, 0.01, 0.005}: TGT+ and TGT on ba_100k
    (max and mean error on the 2048 edges whose exact SC the oracle stored), and
    TGT+ on Barabasi-Albert stand-ins with the node and edge counts of the paper's
    datasets (attachment m/n rounded; --check-edges sampled edges against exact SC
    by conjugate gradients)."""
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    eps_list = (0.05, 0.02, 0.01, 0.005, 1e-3, 1e-4)
    rows = []
    graph = gg.workload("ba_100k", SEED)
    n, u, v = graph
    m = len(u)
    gz = np.load(GOLDEN)
    g = sc.sc_build_graph(n, u, v)
    out = torch.empty(m, dtype=torch.float64, device=dev)
    for method, mname in ((sc.SC_TGT_PLUS, "tgt_plus"), (sc.SC_TGT, "tgt")):
        for eps in eps_list:
            o = sc.sc_default_options(method=method, precision=0, block=BLOCK,
                                      stream=stream.cuda_stream)
            dt, st = timed_calls(sc, g, eps, o, out, a.steps, a.warmup)
            e = np.abs(out.cpu().numpy()[gz["edge_ids"]] - gz["sc"])
            rows.append({"graph": "ba_100k", "n": n, "m": m, "method": mname, "eps": eps,
                         "ms": 1e3 * dt, "edges_per_s": m / dt, "max_abs_err": float(e.max()),
                         "mean_abs_err": float(e.mean()), "checked_edges": len(e),
                         "L_used": st["L_used"], "tilde_tau": st["tilde_tau"],
                         "closed_form_only": st["L_used"] <= 1})
            print(f"[eps] ba_100k {mname} eps={eps}: {1e3 * dt:.1f} ms, max err {e.max():.2e}",
                  file=sys.stderr, flush=True)
    g.free()
    rng = np.random.default_rng(11)
    for name, n_ds, m_ds in (("facebook-shaped", 4_039, 88_234), ("hepph-shaped", 34_401, 420_784),
                             ("slashdot-shaped", 77_360, 469_180),
                             ("twitch-shaped", 168_114, 6_797_557)):
        k = max(1, round(m_ds / n_ds))
        n, u, v = gg.barabasi_albert(n_ds, k, SEED)
        m = len(u)
        g = sc.sc_build_graph(n, u, v)
        out = torch.empty(m, dtype=torch.float64, device=dev)
        ids = rng.choice(m, size=min(a.check_edges, m), replace=False)
        ref = exact_sc_sampled(n, u, v, ids)
        for eps in eps_list:
            o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, block=BLOCK,
                                      stream=stream.cuda_stream)
            dt, st = timed_calls(sc, g, eps, o, out, a.steps, a.warmup)
            e = np.abs(out.cpu().numpy()[ids] - ref)
            rows.append({"graph": name, "n": n, "m": m, "attach": k, "method": "tgt_plus",
                         "eps": eps, "ms": 1e3 * dt, "edges_per_s": m / dt,
                         "max_abs_err": float(e.max()), "mean_abs_err": float(e.mean()),
                         "checked_edges": len(e), "L_used": st["L_used"],
                         "tilde_tau": st["tilde_tau"], "closed_form_only": st["L_used"] <= 1})
            print(f"[eps] {name} n={n} m={m} eps={eps}: {1e3 * dt:.1f} ms, "
                  f"max err {e.max():.2e}", file=sys.stderr, flush=True)
        g.free()
    head = [r for r in rows if r["graph"] == "ba_100k" and r["method"] == "tgt_plus"
            and r["eps"] == 0.01][0]
    line = {
        "metric": "all-edge SC edges/sec across error bounds (TGT+, TGT)",
        "value": head["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "eps sweep on ba_100k (value: TGT+ at eps=0.01) and on "
                               "Barabasi-Albert stand-ins of the paper's dataset sizes",
                   "rows": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def caltau_form(a):
    """CalTau (Algorithm 1, omega = 128) against the lambda*-bound: the device
    spectrum (preprocessing, timed apart), mean and largest tau, time per call and
    error on sampled edges (exact SC by conjugate gradients).  Graphs: king grids
    of 2,500 and 10,000 nodes (slow mixing; TGT at eps = 1e-2, the lambda*-bound
    capped at max_L = 255 and so not certified) and ba_100k (TGT+ at eps = 1e-3)."""
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    rng = np.random.default_rng(5)
    rows = []
    for name, graph, method, eps in (("king_grid_2500", gg.king_grid(2500), sc.SC_TGT, 1e-2),
                                     ("king_grid_10000", gg.king_grid(10_000), sc.SC_TGT, 1e-2),
                                     ("ba_100k", gg.workload("ba_100k", SEED), sc.SC_TGT_PLUS, 1e-3)):
        n, u, v = graph
        m = len(u)
        g = sc.sc_build_graph(n, u, v)
        t0 = time.perf_counter()
        kept, res = sc.sc_compute_spectrum(g, 128, 2048, 1e-8)
        spec_s = time.perf_counter() - t0
        lam, _ = sc.sc_get_spectrum(g)
        out = torch.empty(m, dtype=torch.float64, device=dev)
        tau = torch.empty(m, dtype=torch.int32, device=dev)
        ids = rng.choice(m, size=min(a.check_edges, m), replace=False)
        ref = exact_sc_sampled(n, u, v, ids)
        for policy, flags in (("lambda_star", 0), ("caltau", sc.SC_TAU_SPECTRAL)):
            o = sc.sc_default_options(method=method, precision=0, block=BLOCK, flags=flags,
                                      stream=stream.cuda_stream)
            dt, st = timed_calls(sc, g, eps, o, out, a.steps, a.warmup)
            sc.sc_all_edges_ex(g, eps, 0, o, out=out, tau_out=tau)
            torch.cuda.synchronize()
            t = tau.cpu().numpy()
            err = float(np.abs(out.cpu().numpy()[ids] - ref).max())
            rows.append({"graph": name, "n": n, "m": m, "policy": policy,
                         "method": "tgt_plus" if method == sc.SC_TGT_PLUS else "tgt", "eps": eps,
                         "ms": 1e3 * dt, "edges_per_s": m / dt, "tau_mean": float(t.mean()),
                         "tau_max": int(t.max()), "capped": bool(t.max() >= 255),
                         "max_abs_err_sampled": err, "tilde_tau": st["tilde_tau"],
                         "omega_kept": kept, "spectrum_s": spec_s, "spectrum_residual": res,
                         "lambda_omega": float(abs(lam[-1])), "lambda_2": float(abs(lam[1]))})
            print(f"[caltau] {name} {policy}: {1e3 * dt:.1f} ms, tau mean {t.mean():.1f} max "
                  f"{t.max()}, err {err:.2e} (spectrum {spec_s:.1f} s, kept {kept})",
                  file=sys.stderr, flush=True)
        g.free()
    head = [r for r in rows if r["graph"] == "king_grid_10000" and r["policy"] == "caltau"][0]
    line = {
        "metric": "all-edge SC edges/sec with CalTau truncation",
        "value": head["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "CalTau (omega=128, device Lanczos) vs the lambda*-bound on "
                               "king grids (TGT, eps=1e-2) and ba_100k (TGT+, eps=1e-3); "
                               "value = king_grid_10000 with CalTau", "rows": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def params_form(a):
    """The parameter study of Section 5.4 (Figure 5): TGT+ time and walk count
    against omega (CalTau pairs, Algorithm 1) in {2, 8, 32, 128} with gamma = 10,
    and against gamma (Algorithm 3 candidates) in {0, 2, 5, 10, 16} with the
    lambda*-bound.  omega: the device spectrum at omega = 128, then its first
    omega pairs loaded with sc_set_spectrum.  Graphs: king grid n = 2,500 and the
    HepPh-shaped BA stand-in at eps = 0.05 (the paper's setting), and ba_100k at
    eps = 1e-3 for gamma."""
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    rows = []
    cases = (("king_grid_2500", gg.king_grid(2500), 0.05, True),
             ("hepph-shaped", gg.barabasi_albert(34_401, 12, SEED), 0.05, True),
             ("ba_100k", gg.workload("ba_100k", SEED), 1e-3, False))
    for name, graph, eps, do_omega in cases:
        n, u, v = graph
        m = len(u)
        g = sc.sc_build_graph(n, u, v)
        out = torch.empty(m, dtype=torch.float64, device=dev)

        def point(label, value, flags, gamma):
            o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, block=BLOCK,
                                      flags=flags, gamma=gamma, stream=stream.cuda_stream)
            dt, st = timed_calls(sc, g, eps, o, out, a.steps, a.warmup)
            rows.append({"graph": name, "n": n, "m": m, "eps": eps, label: value,
                         "gamma": gamma, "ms": 1e3 * dt, "walks": st["walks"],
                         "L_used": st["L_used"], "tilde_tau": st["tilde_tau"],
                         "tilde_min": st["tilde_min"], "tilde_max": st["tilde_max"]})
            print(f"[params] {name} {label}={value} gamma={gamma}: {1e3 * dt:.1f} ms, "
                  f"walks {st['walks']}, L {st['L_used']}, tilde {st['tilde_tau']}",
                  file=sys.stderr, flush=True)

        if do_omega:
            kept, _ = sc.sc_compute_spectrum(g, 128, 2048, 1e-8)
            lam, phi = sc.sc_get_spectrum(g)
            for omega in (2, 8, 32, 128):
                w = min(omega, kept)
                sc.sc_set_spectrum(g, lam[:w], phi[:, :w])
                point("omega", w, sc.SC_TAU_SPECTRAL, 10)
        for gamma in (0, 2, 5, 10, 16):
            point("gamma_sweep", gamma, 0, gamma)
        if do_omega:
            # the per-source path takes any gamma (top-gamma by radix select): Figure 5b's range
            for gamma in (0, 10, 100, 1000, 10000):
                if gamma <= n:
                    point("gamma_per_source", gamma, sc.SC_PER_SOURCE, gamma)
        g.free()
    head = [r for r in rows if r["graph"] == "ba_100k" and r.get("gamma_sweep") == 10][0]
    line = {
        "metric": "TGT+ time across omega and gamma (Section 5.4)",
        "value": m / (head["ms"] * 1e-3), "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "omega and gamma sweeps (value: ba_100k, gamma = 10)",
                   "rows": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


WEIGHTS = os.path.join(ROOT, "paper_2305_16086_amd", "weights", "closure_ba_gnp.bin")
BATCH_GOLDEN = os.path.join(ROOT, "tests", "golden", "batch_256_seed7_sampled_sc.npz")


def library_spmm_reference(graph, dev, reps=20):
    """The dense step's product D^-1 A Y by the vendor library: torch.sparse.mm on a
    CSR tensor (hipSPARSE SpMM) with a random n x 64 FP32 block, run alone on the
    GPU; mean time per product over `reps` runs by CUDA events.  A reference point
    for the dense-step kernel, which computes the same product (plus the fused
    accumulation) inside the pipeline.  None when the library call is unavailable."""
    import torch
    try:
        n, u, v = graph
        uu = np.concatenate([u, v]).astype(np.int64)
        vv = np.concatenate([v, u]).astype(np.int64)
        order = np.lexsort((vv, uu))
        uu, vv = uu[order], vv[order]
        deg = np.bincount(uu, minlength=n)
        rowptr = np.zeros(n + 1, np.int64)
        np.cumsum(deg, out=rowptr[1:])
        vals = (1.0 / deg[uu]).astype(np.float32)
        A = torch.sparse_csr_tensor(torch.from_numpy(rowptr).to(dev), torch.from_numpy(vv).to(dev),
                                    torch.from_numpy(vals).to(dev), size=(n, n))
        Y = torch.rand(n, 64, dtype=torch.float32, device=dev, generator=torch.Generator(
            device=dev).manual_seed(5))
        for _ in range(3):
            Z = torch.sparse.mm(A, Y)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            Z = torch.sparse.mm(A, Y)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        del Z, Y, A
        return {"kernel": "torch.sparse.mm (hipSPARSE SpMM) of the same D^-1 A by a random "
                          "n x 64 FP32 block, alone on the GPU",
                "us": us, "gathered_TBps": len(uu) * 64 * 4 / (us * 1e-6) / 1e12}
    except Exception as e:   # the library path is a reference only
        return {"error": f"{type(e).__name__}: {e}"}


def plain_extras(a, sc, g, graph, out, stream):
    """The comparisons the metric names, on the same resident graph and the same
    2048 sampled exact values: the learned closure (committed weights) and plain
    TGT+ at eps = 1e-3 and at eps = 1e-5 (equal measured accuracy), per-source
    TGT+ (Eq. 14 switch per source), and the 256-graph batch against one graph at
    a time.  One warm-up and two timed calls each (the batch: one timed pass one
    graph at a time)."""
    import torch
    n, u, v = graph
    m = len(u)
    gz = np.load(GOLDEN)
    res = {}

    def timed(eps, **kw):
        o = sc.sc_default_options(precision=0, block=BLOCK, stream=stream.cuda_stream, **kw)
        sc.sc_all_edges_ex(g, eps, 0, o, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            st = sc.sc_all_edges_ex(g, eps, 0, o, out=out)[1]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        e = np.abs(out.cpu().numpy()[gz["edge_ids"]] - gz["sc"])
        return {"eps": eps, "ms": 1e3 * dt, "edges_per_s": m / dt, "max_abs_err_sampled": float(e.max()),
                "mean_abs_err_sampled": float(e.mean()), "L_used": st["L_used"],
                "walks": st["walks"], "walk_steps": st["walk_steps"],
                "fallback_edges": st["fallback_edges"], "tilde_min": st["tilde_min"],
                "tilde_max": st["tilde_max"], "push_edges": st["push_edges"]}

    print("[plain] extras: TGT+ at 1e-5", file=sys.stderr, flush=True)
    res["tgt_plus_eps_1e-5"] = timed(1e-5, method=sc.SC_TGT_PLUS)
    if os.path.exists(WEIGHTS):
        print("[plain] extras: learned closure", file=sys.stderr, flush=True)
        net = sc.sc_mlp_load(WEIGHTS)
        res["learned"] = timed(EPS, method=sc.SC_LEARNED, mlp=net.handle.value)
        res["learned"]["weights"] = os.path.relpath(WEIGHTS, ROOT)
        net.free()
    print("[plain] extras: per-source TGT+", file=sys.stderr, flush=True)
    res["per_source_tgt_plus"] = timed(EPS, method=sc.SC_TGT_PLUS, flags=sc.SC_PER_SOURCE)
    print("[plain] extras: batch", file=sys.stderr, flush=True)
    res["batched"] = batch_summary(sc, stream)
    return res


def batch_summary(sc, stream):
    """The 256-graph batch (TGT, eps = 1e-2, FP32, tuned block widths, truncation
    capped at 31) in one persistent launch per (LDS class, block), against the
    same graphs one at a time through sc_all_edges_ex (TGT+); errors over 16
    sampled edges of every graph (exact SC stored by the oracle)."""
    import torch
    import graphgen as gg
    graphs = gg.workload("batch_256", 7)
    M = sum(len(x[1]) for x in graphs)
    dev = torch.device("cuda:0")
    b = sc.sc_build_batch(graphs)
    outs = [torch.empty(len(x[1]), dtype=torch.float64, device=dev) for x in graphs]

    def opts(**kw):
        return sc.sc_default_options(method=sc.SC_TGT, precision=0, max_L=BATCH_MAX_L,
                                     stream=stream.cuda_stream, **kw)

    t0 = time.perf_counter()
    sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(), out=outs)   # lambda* of every graph
    torch.cuda.synchronize()
    pre_s = time.perf_counter() - t0
    if os.path.exists(TUNING):
        sc.sc_batch_load_tuning(b, TUNING)
    sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(), out=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        _, st = sc.sc_batch_all_edges(b, BATCH_EPS, None, opts(), out=outs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 2
    res = [x.cpu().numpy() for x in outs]
    err = None
    if os.path.exists(BATCH_GOLDEN):
        gz = np.load(BATCH_GOLDEN)
        err = max(float(np.abs(res[k][e] - s)) for k, e, s in zip(gz["graph"], gz["edge_ids"], gz["sc"]))
    vals = [torch.empty_like(x) for x in outs]
    for i, gh in enumerate(b.graphs):   # warm: per-graph buffers and plans
        o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, max_L=BATCH_MAX_L,
                                  stream=stream.cuda_stream)
        sc.sc_all_edges_ex(gh, BATCH_EPS, 0, o, out=vals[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, gh in enumerate(b.graphs):
        o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, max_L=BATCH_MAX_L,
                                  stream=stream.cuda_stream)
        sc.sc_all_edges_ex(gh, BATCH_EPS, 0, o, out=vals[i])
    torch.cuda.synchronize()
    one_s = time.perf_counter() - t0
    b.free()
    return {"workload": "batch_256 (seed 7): 256 graphs, n uniform in [200, 20000], G(n,p) deg 8 / "
                        "BA m=5 / king grid; TGT, eps=1e-2, FP32, lambda* truncation capped at 31",
            "edges": M, "ms": 1e3 * dt, "edges_per_s": M / dt, "L_capped": st["L_capped"],
            "L_used": st["L_used"], "max_abs_err_sampled_all_graphs": err,
            "err_sample": "16 edges of each of the 256 graphs, exact SC by float64 block-PCG",
            "one_at_a_time_tgt_plus_edges_per_s": M / one_s, "lambda_preprocess_s": pre_s}


RMAT_GOLDEN = os.path.join(ROOT, "tests", "golden", "rmat22_seed22_sampled_sc.npz")
ORKUT_GOLDEN = os.path.join(ROOT, "tests", "golden", "orkut_shaped_sampled_sc.npz")
ORKUT_N, ORKUT_ATTACH = 3_072_441, 38   # Table 3: n = 3,072,441, m = 117,185,082 (m/n = 38.1)


def rmat_form(a):
    """R-MAT scale 22 (a, b, c, d = .57, .19, .19, .05, edge factor 16, symmetrised,
    deduplicated, largest component; seed 22) by per-source TGT+ (frontier-sparse
    traversal, switch step by Eq. 14 per source) at eps = 1e-2.  A full call is
    out of reach of the time budget here, so a uniform random sample of
    --rmat-sources sources is timed (each source's halves are independent work)
    and the call time is extrapolated by n / sample; the error is checked on the
    512 sampled edges whose exact SC the oracle stored, by a second call over
    their endpoints (both halves of every checked edge computed)."""
    import graphgen as gg
    t0 = time.perf_counter()
    n, u, v = gg.rmat_lcc(a.rmat_scale, 16, seed=22)
    gen_s = time.perf_counter() - t0
    name = f"rmat_s{a.rmat_scale}"
    workload = (f"{name}: R-MAT scale {a.rmat_scale} (a,b,c,d=.57,.19,.19,.05), edge factor 16, "
                f"symmetrised, deduplicated, largest component, seed 22")
    sampled_source_form(a, name, workload, (n, u, v), gen_s, 1e-2,
                        RMAT_GOLDEN if a.rmat_scale == 22 else None)


def orkut_form(a):
    """The Orkut-shaped stand-in (Table 3's node and edge counts): Barabasi-Albert
    with n = 3,072,441 and 38 edges per new node (m = 116.8 M), seed 1, by
    per-source TGT+ at --orkut-eps (default 1e-3: at 1e-2 its lambda* of 0.23 keeps every
    truncation at 1, the closed form), timed on sampled sources as the R-MAT form."""
    import graphgen as gg
    t0 = time.perf_counter()
    n, u, v = gg.barabasi_albert(ORKUT_N, ORKUT_ATTACH, SEED, progress=lambda k: print(
        f"[orkut] generated {k} nodes ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
        flush=True))
    gen_s = time.perf_counter() - t0
    workload = (f"orkut_shaped: Barabasi-Albert n={ORKUT_N}, {ORKUT_ATTACH} edges per new node, "
                f"seed {SEED} (the node and edge counts of the paper's Orkut dataset)")
    sampled_source_form(a, "orkut_shaped", workload, (n, u, v), gen_s, a.orkut_eps, ORKUT_GOLDEN)


def sampled_source_form(a, name, workload, graph, gen_s, eps, golden):
    import torch
    from paper_2305_16086_amd import sc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    n, u, v = graph
    m = len(u)
    print(f"[{name}] n={n} m={m} ({gen_s:.0f} s)", file=sys.stderr, flush=True)
    order = a.node_order or "degree"
    order_flag, order_desc = node_order_flag(sc, order)
    t0 = time.perf_counter()
    g = sc.sc_build_graph(n, u, v, order_flag)
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    lam = sc.sc_lambda_star(g)
    lam_s = time.perf_counter() - t0
    print(f"[{name}] built {build_s:.1f} s, lambda* {lam:.4f} ({lam_s:.1f} s)", file=sys.stderr,
          flush=True)
    out = torch.empty(m, dtype=torch.float64, device=dev)
    o = sc.sc_default_options(method=sc.SC_TGT_PLUS, flags=sc.SC_PER_SOURCE, stream=stream.cuda_stream,
                              switch_rule=a.switch_rule)
    rng = np.random.default_rng(22)
    src = rng.choice(n, size=min(a.rmat_sources, n), replace=False).astype(np.int32)
    wst = sc.sc_all_edges_ex(g, eps, 0, o, out=out, sources=src[:256])[1]   # buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ot = sc.sc_default_options(method=sc.SC_TGT_PLUS, flags=sc.SC_PER_SOURCE | sc.SC_TIME_KERNELS,
                               stream=stream.cuda_stream, switch_rule=a.switch_rule)
    _, st = sc.sc_all_edges_ex(g, eps, 0, ot, out=out, sources=src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    full_s = dt * n / len(src)
    walk_gbs = st["prop_bytes"] / (st["prop_ms"] * 1e-3) / 1e9 if st["prop_ms"] > 0 else 0.0
    print(f"[{name}] {len(src)} sources in {dt:.2f} s -> full call {full_s:.0f} s; walks {st['walks']}, "
          f"push {st['push_edges']}, tilde {st['tilde_min']}..{st['tilde_max']}", file=sys.stderr,
          flush=True)
    err = None
    checked = 0
    ck = {}
    full = None
    if full_s <= a.full_call_limit:
        # the whole call (every source) is within reach: time it instead of extrapolating
        print(f"[{name}] timing the full call", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, fst = sc.sc_all_edges_ex(g, eps, 0, ot, out=out)
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t0
        full = {"s": fdt, "walks": fst["walks"], "walk_steps": fst["walk_steps"],
                "push_edges": fst["push_edges"], "tilde_min": fst["tilde_min"],
                "tilde_max": fst["tilde_max"], "L_capped": fst["L_capped"],
                "walk_phase_ms": fst["prop_ms"]}
        walk_gbs = fst["prop_bytes"] / (fst["prop_ms"] * 1e-3) / 1e9 if fst["prop_ms"] > 0 else 0.0
        st = dict(st, prop_bytes=fst["prop_bytes"], prop_ms=fst["prop_ms"])
        print(f"[{name}] full call {fdt:.2f} s; walks {fst['walks']}", file=sys.stderr, flush=True)
        if golden and os.path.exists(golden):
            gz = np.load(golden)
            ids = gz["edge_ids"]
            e = np.abs(out.cpu().numpy()[ids] - gz["sc"])
            err = float(e.max())
            checked = int(len(ids))
            full["mean_abs_err"] = float(e.mean())
            print(f"[{name}] error on {checked} sampled edges: max {err:.2e}", file=sys.stderr,
                  flush=True)
    if full is None and golden and os.path.exists(golden):
        gz = np.load(golden)
        ids = gz["edge_ids"]
        ends = np.unique(np.concatenate([u[ids], v[ids]])).astype(np.int32)
        t0 = time.perf_counter()
        _, cst = sc.sc_all_edges_ex(g, eps, 0, o, out=out, sources=ends)
        torch.cuda.synchronize()
        ck = {"sources": int(len(ends)), "s": time.perf_counter() - t0, "walks": cst["walks"],
              "walk_steps": cst["walk_steps"], "tilde_min": cst["tilde_min"],
              "tilde_max": cst["tilde_max"]}
        e = np.abs(out.cpu().numpy()[ids] - gz["sc"])
        err = float(e.max())
        checked = int(len(ids))
        ck["mean_abs_err"] = float(e.mean())
        print(f"[{name}] error on {checked} sampled edges: max {err:.2e}", file=sys.stderr, flush=True)
    g.free()
    call_s = full["s"] if full else full_s
    # counters were taken for the R-MAT sample in degree order only
    per_step = (measured_walk_traffic_per_step()
                if name == "rmat_s22" and order == "degree" and full is None else None)
    walk_traffic = per_step * st["walk_steps"] if per_step else None
    line = {
        "metric": ("all-edge SC edges/sec (per-source TGT+, whole call)" if full else
                   "all-edge SC edges/sec (per-source TGT+, extrapolated from sampled sources)"),
        "value": m / call_s, "unit": "edges/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * call_s, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "u64 fixed point + f64", "data": "synthetic",
        "config": {
            "workload": f"{workload}: n={n}, m={m}; TGT+ per source ("
                        + ("Eq. 14 switch" if a.switch_rule == 0 else
                           "switch by Eq. 14 with walks weighed by their steps") +
                        f"), eps={eps}, lambda*-bound truncation at eps/2",
            "sample": (f"{len(src)} uniform random sources timed in one call ({dt:.2f} s) "
                       f"extrapolated by n/{len(src)} to {full_s:.1f} s" +
                       ("; the whole call then timed (value)" if full else
                        "; the value is the extrapolation")),
            "full_call": full,
            "node_order": order_desc,
            "sample_sources_per_s": len(src) / dt, "lambda_star": lam,
            "lambda_converged": st["lambda_converged"], "L_used": st["L_used"],
            "L_min": st["L_min"], "L_capped": st["L_capped"], "tilde_min": st["tilde_min"],
            "tilde_max": st["tilde_max"], "walks": st["walks"], "walk_steps": st["walk_steps"],
            "push_edges": st["push_edges"], "max_abs_err_sampled": err, "checked_edges": checked,
            "check_call": ck, "generate_s": gen_s, "build_s": build_s, "lambda_s": lam_s,
            "walk_phase_ms": st["prop_ms"], "call_ms": 1e3 * dt,
            "warmup_call": {"sources": int(min(256, len(src))), "walks": wst["walks"],
                            "walk_steps": wst["walk_steps"]},
            # tau <= 1 everywhere: only the closed-form l = 0, 1 terms, no traversal
            "closed_form_only": st["L_used"] <= 1,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "walk phase of the per-source waves (k_src_scan, k_src_walks, k_src_finish, "
                      "k_src_clear), timed by events per wave",
            "achieved": walk_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": walk_gbs / HBM_PEAK_GBS, "traffic": walk_traffic,
            "alg_bytes": st["prop_bytes"],
            "alg_bytes_note": "20 B per single-walk step (row bounds 8, neighbour id 4, column entry 8); "
                              "every access is random, so each moves at least a 64-byte line",
            "traffic_note": ("FETCH_SIZE + WRITE_SIZE counters of k_src_walks, scaled by kernels of "
                             f"known traffic: {per_step:.0f} B per single-walk step"
                             if walk_traffic else None),
            "traffic_TBps": (walk_traffic / (st["prop_ms"] * 1e-3) / 1e12
                             if walk_traffic and st["prop_ms"] > 0 else None),
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    if a.form == "batch":
        batch_form(a)
        return
    if a.form == "learned":
        learned_form(a)
        return
    if a.form == "er":
        er_form(a)
        return
    if a.form == "eps":
        eps_form(a)
        return
    if a.form == "caltau":
        caltau_form(a)
        return
    if a.form == "params":
        params_form(a)
        return
    if a.form == "rmat":
        rmat_form(a)
        return
    if a.form == "orkut":
        orkut_form(a)
        return
    import torch
    from paper_2305_16086_amd import sc
    import graphgen as gg

    graph = gg.workload("ba_100k", SEED)
    n, u, v = graph
    m = len(u)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    order_flag, order_desc = node_order_flag(sc, a.node_order or "generator")
    g = sc.sc_build_graph(n, u, v, order_flag)
    out = torch.empty(m, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(flags=0, traces=None):
        o = sc.sc_default_options(method=sc.SC_TGT_PLUS, precision=0, block=BLOCK,
                                  flags=flags, stream=stream.cuda_stream)
        kw = traces or {}
        return sc.sc_all_edges_ex(g, EPS, 0, o, out=out, **kw)[1]

    if a.copy_probe_mb > 0:
        # a fill (writes S bytes) and an elementwise product (reads S, writes S)
        src = torch.ones(a.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # the first call on the fresh graph: lambda* (two Lanczos runs), the switch-step
    # plan and buffer allocation, then the call itself
    t0 = time.perf_counter()
    cold = step()
    torch.cuda.synchronize()
    cold_ms = 1e3 * (time.perf_counter() - t0)
    for _ in range(max(a.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()

    stats = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        stats.append(step(flags=sc.SC_TIME_KERNELS))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / a.steps
    value = m / (dt / a.steps)

    launches = sum(s["prop_launches"] for s in stats)
    timed = sum(s["prop_timed"] for s in stats)
    prop_ms = sum(s["prop_ms"] for s in stats)
    prop_bytes = sum(s["prop_bytes"] for s in stats)
    avg_launch_us = 1e3 * prop_ms / max(timed, 1)
    bytes_per_launch = prop_bytes / max(launches, 1)
    achieved = bytes_per_launch / (avg_launch_us * 1e-6) / 1e9 if launches else 0.0

    # accuracy on the sampled edges whose exact SC the oracle stored
    res = out.cpu().numpy()
    err = None
    if os.path.exists(GOLDEN):
        gz = np.load(GOLDEN)
        err = float(np.abs(res[gz["edge_ids"]] - gz["sc"]).max())

    # one extra call to record the switch step and walk counts for the CPU baseline
    tau = torch.empty(m, dtype=torch.int32, device=dev)
    tt = torch.empty(n, dtype=torch.int32, device=dev)
    nr = torch.empty(2 * m, dtype=torch.int64, device=dev)
    last = step(traces={"tau_out": tau, "tilde_tau_out": tt, "nr_out": nr})
    torch.cuda.synchronize()
    extras = {}
    spmm_ref = None
    if not a.no_extras:
        extras = plain_extras(a, sc, g, graph, out, stream)
        spmm_ref = library_spmm_reference(graph, dev)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(graph, tau.cpu().numpy(), tt.cpu().numpy(), nr.cpu().numpy(),
                           a.cpu_sources)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "ba_100k: Barabasi-Albert n=100000, 10 edges per new node, seed 1 "
                        f"(m={m}); TGT+, eps=1e-3, automatic truncation, FP32 propagation, "
                        "FP64 per-edge sums, block 64",
            "max_abs_err_sampled": err,
            "err_sample": "2048 edges, exact SC by float64 block-PCG" if err is not None else None,
            "node_order": order_desc,
            "L_used": last["L_used"], "L_min": last["L_min"],
            "tilde_tau": last["tilde_tau"], "lambda_star": last["lambda_star"],
            "lambda_converged": last["lambda_converged"], "L_capped": last["L_capped"],
            "walks": last["walks"], "walk_steps": last["walk_steps"],
            "cold_call_ms": cold_ms,
            "cold_call": "first call on the built graph: lambda* (two Lanczos runs), "
                         "switch-step plan, buffers, then the call",
            **extras,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_propagate<float, 64, false> (dense block gather of every neighbour row, FP32, B=64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # the counters were taken with the nodes in the generator's order
            "traffic": measured_traffic() if (a.node_order or "generator") == "generator" else None,
            "avg_launch_us": avg_launch_us,
            "launches": launches,
            "timed_launches": timed,
            "alg_bytes_per_launch": bytes_per_launch,
            "gathered_TBps": 2 * m * 64 * 4 / (avg_launch_us * 1e-6) / 1e12 if launches else None,
            "library_spmm": spmm_ref,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
