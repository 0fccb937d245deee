"""Train the unit-cost model the library ships (costmodel_gfx950.fxmlp).

The model (4 -> 64 -> 64 -> 1, FP32) predicts the time of one K-block work
unit in one class launch; it only orders units inside launches (culling is
always the bound test of Eq. (8)).  Training data are unit timings the
library records itself (fx_record_task_timings) on three workloads: the
200-atom chain, the 1000-atom s+p+d cluster and the 64 s+p clusters of
50-500 atoms, each in mixed precision at tau = 1e-8.  Training runs on the
GPU with the library's own forward, backward and Adam kernels.

    python -m paper_1401_6961_amd.train_costmodel [--out PATH] [--steps N]

Needs a GPU.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "costmodel_gfx950.fxmlp")


def record(fx, torch, system, opts):
    tree = fx.build_quadtree_from(system)
    P = torch.from_numpy(system.P).cuda()
    fx.fx_exchange_ex(tree, P, system.tau, torch.zeros_like(P), opts, stats=False)   # sizes the buffers
    torch.cuda.synchronize()
    f, t, c = fx.fx_record_task_timings(tree, P, system.tau, opts).arrays()
    return f, t


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--per-workload", type=int, default=400000, help="samples kept per workload")
    ap.add_argument("--seed", type=int, default=2024)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import synthetic
    import paper_1401_6961_amd as fx

    def log(msg):
        print(msg, flush=True)

    opts = fx.make_opts(precision=fx.FX_PREC_MIXED)
    rng = np.random.default_rng(args.seed)
    feats, times = [], []
    workloads = [("200-atom chain", [synthetic.config(1)]),
                 ("1000-atom s+p+d cluster", [synthetic.config(2)]),
                 ("64 s+p clusters", synthetic.config(3))]
    for name, systems in workloads:
        t0 = time.time()
        fs, ts = [], []
        for s in systems:
            f, t = record(fx, torch, s, opts)
            fs.append(f)
            ts.append(t)
        f = np.concatenate(fs)
        t = np.concatenate(ts)
        keep = rng.permutation(len(t))[:args.per_workload]
        feats.append(f[keep])
        times.append(t[keep])
        log(f"train_costmodel: {name}: {len(t)} unit timings, kept {len(keep)} ({time.time() - t0:.1f} s)")
    f = np.concatenate(feats)
    t = np.concatenate(times)
    data = fx.TaskTimings.from_arrays(f, t)
    model, loss = fx.fx_costmodel_train(data, steps=args.steps, batch=8192, seed=args.seed)
    log(f"train_costmodel: {len(t)} samples, final loss {loss:.4f} (standardised MSE)")
    model.save(args.out)
    log(f"train_costmodel: saved {args.out}")


if __name__ == "__main__":
    main()
