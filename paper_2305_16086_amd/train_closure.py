"""Train the learned tail closure's network on the GPU and write its weights file.

Training set (synthetic, seeded): 16 graphs with n log-uniform in [1e4, 1e5]
(numpy seed 100); even k: Barabasi-Albert with 5 or 10 edges per new node,
odd k: G(n,p) with average degree 8 or 10; graph seeds 100 + k.  Targets: the
tail after the odd truncation 7, from TGT at the uniform truncation 201
(sc_closure_dataset).  Training: sc_mlp_train, 30 epochs of Adam, batch 4096,
network seed 7.  Everything runs in the library's kernels; this script only
marshals data.

Writes <out>.bin (sc_mlp_save) and <out>.json (this recipe, sizes, losses,
times and the file's SHA-256).

Usage: python -m paper_2305_16086_amd.train_closure [--out PATH]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(HERE, "weights", "closure_ba_gnp")
L_REF = 201
TRAIN_GRAPHS = 16
EPOCHS = 30
BATCH = 4096
NET_SEED = 7


def training_graphs(count: int = TRAIN_GRAPHS):
    import graphgen as gg
    rng = np.random.default_rng(100)
    for k in range(count):
        n = int(round(10 ** rng.uniform(4.0, 5.0)))
        seed = 100 + k
        if k % 2 == 0:
            yield k, gg.barabasi_albert(n, 5 if k % 4 == 0 else 10, seed)
        else:
            yield k, gg.gnp_connected(n, 8.0 if k % 4 == 1 else 10.0, seed)


def train(count: int = TRAIN_GRAPHS, log=sys.stderr):
    """Build the dataset and train; returns (network, record dict)."""
    import torch
    from paper_2305_16086_amd import sc
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    Xs, zs, ws, sizes = [], [], [], []
    for k, (n, u, v) in training_graphs(count):
        g = sc.sc_build_graph(n, u, v)
        m = len(u)
        X = torch.empty(m * 16, dtype=torch.float32, device=dev)
        z = torch.empty(m, dtype=torch.float32, device=dev)
        w = torch.empty(m, dtype=torch.float32, device=dev)
        sc.sc_closure_dataset(g, L_REF, 0, X, z, w)
        torch.cuda.synchronize()
        g.free()
        Xs.append(X)
        zs.append(z)
        ws.append(w)
        sizes.append((int(n), int(m)))
        print(f"[train] dataset {k}: n={n} m={m} {time.perf_counter() - t0:.1f}s", file=log,
              flush=True)
    data_s = time.perf_counter() - t0
    X = torch.cat(Xs)
    z = torch.cat(zs)
    w = torch.cat(ws)
    del Xs, zs, ws
    net = sc.sc_mlp_create(NET_SEED)
    t0 = time.perf_counter()
    losses = sc.sc_mlp_train(net, X, z, w, sc.sc_default_train_options(epochs=EPOCHS, batch=BATCH))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    rec = {"graphs": sizes, "samples": int(sum(m for _, m in sizes)), "L_ref": L_REF,
           "epochs": EPOCHS, "batch": BATCH, "net_seed": NET_SEED, "dataset_s": data_s,
           "train_s": train_s, "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
    return net, rec


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--out", default=WEIGHTS, help="path without extension")
    a = p.parse_args()
    import torch  # noqa: F401  (the device runtime comes up through torch first)
    from paper_2305_16086_amd import sc
    net, rec = train()
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    sc.sc_mlp_save(net, a.out + ".bin")
    with open(a.out + ".bin", "rb") as f:
        rec["sha256"] = hashlib.sha256(f.read()).hexdigest()
    rec["recipe"] = __doc__.split("Writes")[0].strip()
    rec["command"] = "python -m paper_2305_16086_amd.train_closure"
    with open(a.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
