#!/usr/bin/env python3
"""Benchmark of the exchange build on one MI355X.

Workload: 1000-atom s+p+d cluster (sphere at 0.1 atoms/A^3, min separation
1 A; s: 3 primitives, p: 2, Cartesian d: 1; n = 10,000 functions), density
decay length 2 A, tau = 1e-8.  One step = one fx_exchange_ex call (density
norms, hextree traversal, all class kernels, reduction) in mixed precision.
The FP64 build of the same system is timed once for the comparison fields.

Prints ONE JSON line.  value = computed shell quartets per second of the
mixed build (inputs resident in HBM).  roofline: the class kernel with the
largest summed time, algorithmic flops (generated-code count) per launch
divided by its average launch time from HIP events recorded by the library
on the launch stream.  cpu_baseline: the plain CPU oracle on a bounded
sample of K blocks of the same system.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
LNAME = "spd"


def cname(c):
    return f"({LNAME[c // 27]}{LNAME[(c // 9) % 3]}|{LNAME[(c // 3) % 3]}{LNAME[c % 3]})"


def cpu_baseline(system, budget_s=15.0, seed=0):
    """Time the oracle on seeded random K blocks (a, d) of the same system."""
    import oracle
    t0 = time.time()
    Qn = oracle.schwarz(system)
    Pn = oracle.pnorm(system, system.P)
    t_norms = time.time() - t0
    rng = np.random.default_rng(seed)
    S = system.nshell
    quartets, secs, nblocks = 0, 0.0, 0
    while secs < budget_s and nblocks < 4096:
        pairs = rng.integers(0, S, size=(8, 2)).astype(np.int32)
        t = time.time()
        _, st = oracle.exchange_blocks(system, pairs, Qn=Qn, Pn=Pn)
        secs += time.time() - t
        quartets += st["quartets"]
        nblocks += len(pairs)
    return {"value": quartets / secs, "unit": "quartets/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{nblocks} random K shell blocks (a,d) of the same system, {quartets} quartets in "
                      f"{secs:.1f} s (Schwarz/density norms {t_norms:.1f} s not included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--natom", type=int, default=1000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison build")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic
    import paper_1401_6961_amd as fx

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    log(f"bench: generating {args.natom}-atom s+p+d cluster")
    system = synthetic.cluster(args.natom)
    tau = system.tau
    dev = torch.device("cuda:0")
    t = time.time()
    tree = fx.build_quadtree_from(system)
    torch.cuda.synchronize()
    t_tree = time.time() - t
    P = torch.from_numpy(system.P).to(dev)
    K = torch.zeros_like(P)
    opts_mixed = fx.make_opts(precision=fx.FX_PREC_MIXED, profile=True)

    for i in range(args.warmup):
        log(f"bench: warmup {i}")
        fx.fx_exchange_ex(tree, P, tau, K, opts_mixed)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} mixed-precision steps")
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        _, st = fx.fx_exchange_ex(tree, P, tau, K, opts_mixed)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = stats[-1]
    ms_per_step = 1e3 * elapsed / args.steps
    quartets = st["quartets"]
    value = quartets * args.steps / elapsed

    # dominant kernel (largest summed event time over the timed steps)
    cs = sum(s["class_seconds"] for s in stats)
    cl = sum(s["class_launches"] for s in stats)
    cf = sum(s["class_flops"] for s in stats)
    c, p = np.unravel_index(int(np.argmax(cs)), cs.shape)
    per_launch_flops = cf[c, p] / max(1, cl[c, p])
    avg_launch_s = cs[c, p] / max(1, cl[c, p])
    achieved = per_launch_flops / avg_launch_s / 1e12
    peak = FP32_PEAK_TFLOPS if p else FP64_PEAK_TFLOPS
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "kernel": f"fx_k_{cname(c)[1:3]}{cname(c)[4:6]}_{'f32' if p else 'f64'}",
                "class": cname(c), "avg_launch_ms": 1e3 * avg_launch_s,
                "flops_per_launch": per_launch_flops,
                "all_class_kernels_tflops": float(cf.sum() / cs.sum() / 1e12) if cs.sum() > 0 else None}

    extra = {}
    if not args.no_fp64:
        log("bench: FP64 comparison build")
        K64 = torch.zeros_like(P)
        t = time.perf_counter()
        _, st64 = fx.fx_exchange_ex(tree, P, tau, K64, fx.make_opts(precision=fx.FX_PREC_FP64))
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        dK = (K - K64).abs()
        extra = {"fp64_kbuild_s": t64, "fp64_quartets_per_s": st64["quartets"] / t64,
                 "mixed_speedup_vs_fp64": t64 / (elapsed / args.steps),
                 "mixed_err_maxabs": float(dK.max()), "mixed_err_frob": float(torch.linalg.norm(K - K64)),
                 "mixed_err_exchange_energy": float(abs(0.25 * ((P * (K - K64)).sum()))),
                 "same_quartets": int(st64["quartets"]) == int(quartets)}
        del K64

    cpu = None
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(system, args.cpu_seconds)

    out = {"metric": "K-build s & ERI quartets/s at tau=1e-8, mixed vs FP64, 1000-atom s+p+d",
           "value": value, "unit": "quartets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": f"{args.natom}-atom s+p+d cluster, n={system.nbf}, tau=1e-8, mixed precision",
                      "natom": args.natom, "nbf": system.nbf, "tau": tau, "parallelism": "single-gpu"},
           "kbuild_s": elapsed / args.steps, "quartets": int(quartets), "quartets_fp32": int(st["quartets_fp32"]),
           "prim_quartets": st["prim_quartets"], "alg_flops": st["flops"],
           "alg_tflops": st["flops"] / (elapsed / args.steps) / 1e12, "tree_build_s": t_tree,
           "traversal_s": st["seconds_traversal"], "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
