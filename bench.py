#!/usr/bin/env python3
"""Benchmark of the exchange build on one MI355X.

Workload: 1000-atom s+p+d cluster (sphere at 0.1 atoms/A^3, min separation
1 A; s: 3 primitives, p: 2, Cartesian d: 1; n = 10,000 functions), density
decay length 2 A, tau = 1e-8.  One step = one fx_exchange_ex call (density
norms, hextree traversal, all class kernels, reduction) in mixed precision.
The FP64 build of the same system is timed once for the comparison fields.

Prints ONE JSON line.  value = shell quartets per second of the mixed
build (inputs resident in HBM), counting the ordered quartets with
beta > tau that K accounts for (the set the oracle evaluates; with a
symmetric density half of them are evaluated and stand for their mirrors,
reported as quartets_evaluated).  roofline: the class kernel with the
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
HBM_PEAK_GBPS = 8000.0
LNAME = "spd"


def cname(c):
    return f"({LNAME[c // 27]}{LNAME[(c // 9) % 3]}|{LNAME[(c // 3) % 3]}{LNAME[c % 3]})"


def kernel_sources_hash(kernel):
    """Hash of the sources a class kernel is compiled from: its generated
    class file and the shared kernel templates (None if one is missing)."""
    import hashlib
    cls = kernel[len("fx_k_"):len("fx_k_") + 4]
    h = hashlib.sha256()
    for p in (f"paper_1401_6961_amd/csrc/gen/eri_{cls}.hip", "paper_1401_6961_amd/csrc/fx_eri_common.h",
              "paper_1401_6961_amd/csrc/fx_internal.h"):
        path = os.path.join(ROOT, p)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def tuning_table_info():
    """Hash and size of the tuning table the library was generated and launched with."""
    import hashlib
    path = os.path.join(ROOT, "paper_1401_6961_amd", "tuning_gfx950.json")
    if not os.path.exists(path):
        return None
    raw = open(path, "rb").read()
    t = json.loads(raw)
    gen = t.get("generator", {})
    return {"path": os.path.relpath(path, ROOT), "sha256": hashlib.sha256(raw).hexdigest()[:16],
            "launch_entries": len(t.get("classes", {})), "generator_kernels": len(gen.get("kernels", {})),
            "generator_tuned": gen.get("tuned")}


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/hbm_traffic_*.md), provided the kernel's sources hash to
    the value recorded with the counters; (None, None) otherwise."""
    import glob
    import re
    gh = kernel_sources_hash(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("kernel") == kernel and rec.get("gen_hash") == gh:
            return rec["traffic_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, quartets_total, budget_s=10.0, seed=0):
    """The oracle on seeded random K blocks (a, d) of the same system, on one
    thread and on every host thread; the whole-K time is extrapolated from the
    all-thread rate and the oracle's quartet count of the whole build."""
    import oracle
    t0 = time.time()
    Qn = oracle.schwarz(system)
    Pn = oracle.pnorm(system, system.P)
    t_norms = time.time() - t0
    S = system.nshell
    out = {}
    all_threads = oracle.num_threads()
    for label, threads, budget in (("one_thread", 1, 0.5 * budget_s), ("all_threads", all_threads, budget_s)):
        oracle.set_threads(threads)
        rng = np.random.default_rng(seed)
        quartets, secs, nblocks = 0, 0.0, 0
        while secs < budget and nblocks < 4096:
            pairs = rng.integers(0, S, size=(8, 2)).astype(np.int32)
            t = time.time()
            _, st = oracle.exchange_blocks(system, pairs, Qn=Qn, Pn=Pn)
            secs += time.time() - t
            quartets += st["quartets"]
            nblocks += len(pairs)
        out[label] = {"threads": threads, "quartets": quartets, "seconds": secs, "blocks": nblocks,
                      "quartets_per_s": quartets / secs}
    oracle.set_threads(all_threads)
    rate = out["all_threads"]["quartets_per_s"]
    return {"value": rate, "unit": "quartets/s", "cores": all_threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "one_thread_quartets_per_s": out["one_thread"]["quartets_per_s"],
            "all_threads_quartets_per_s": rate,
            "whole_K_seconds_extrapolated": quartets_total / rate,
            "whole_K_note": "extrapolation, not measured: the oracle's exhaustive quartet count of the whole "
                            "build divided by the all-thread rate on the sample",
            "sample": f"seeded random K shell blocks (a,d) of the same system: one thread "
                      f"{out['one_thread']['blocks']} blocks, {out['one_thread']['quartets']} quartets in "
                      f"{out['one_thread']['seconds']:.1f} s; {all_threads} threads {out['all_threads']['blocks']} "
                      f"blocks, {out['all_threads']['quartets']} quartets in {out['all_threads']['seconds']:.1f} s "
                      f"(Schwarz/density norms {t_norms:.1f} s not included)"}


def shipped_costmodel(fx):
    """The cost model trained on unit timings of the chain, cluster and batch
    workloads (paper_1401_6961_amd/costmodel_gfx950.fxmlp), or None."""
    path = os.path.join(ROOT, "paper_1401_6961_amd", "costmodel_gfx950.fxmlp")
    return fx.CostModel.load(path) if os.path.exists(path) else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--natom", type=int, default=1000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison build")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed FP64 runs (median reported)")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying the captured call")
    ap.add_argument("--no-mlp", action="store_true", help="do not time the learned unit order beside the headline")
    ap.add_argument("--learned", action="store_true", help="headline build with the learned unit order")
    ap.add_argument("--workload", default="cluster",
                    choices=["cluster", "batched", "slab-mlp", "copy-probe", "scaling", "multi", "regimes", "chain"],
                    help="cluster: the headline 1000-atom s+p+d build; batched: 64 clusters in one batched "
                         "call vs 64 sequential builds; slab-mlp: 4000-atom s+p slab, learned vs bound-only "
                         "scheduling; copy-probe: one elementwise copy of 1 GiB, to scale HBM byte counters; "
                         "scaling: K-build time of s+p+d clusters of 125..2000 atoms (onset of linear scaling); "
                         "multi: two densities of the 1000-atom cluster in one call vs two single builds; "
                         "regimes: s+p+d clusters of 125..1000 atoms at the paper's two threshold pairs "
                         "(tau, tau_ovlp) = (1e-8, 1e-11) and (1e-10, 1e-13); chain: 50..3200-atom s+p chains")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the autotuned kernel table")
    ap.add_argument("--sizes", default="125,250,500,1000,2000", help="atom counts of --workload scaling")
    ap.add_argument("--no-symmetry", action="store_true", help="build every K block (no use of K = K^T)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    from paper_1401_6961_amd import autotune

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.workload == "copy-probe":
        return copy_probe()
    tuned = 0 if args.no_tuning else autotune.apply()
    log(f"bench: {tuned} autotuned class entries applied")
    if args.workload == "batched":
        return bench_batched(args, log)
    if args.workload == "slab-mlp":
        return bench_slab_mlp(args, log)
    if args.workload == "scaling":
        return bench_scaling(args, log)
    if args.workload == "multi":
        return bench_multi(args, log)
    if args.workload == "regimes":
        return bench_regimes(args, log)
    if args.workload == "chain":
        return bench_chain(args, log)

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
    sym = fx.FX_SYM_OFF if args.no_symmetry else fx.FX_SYM_AUTO
    model = shipped_costmodel(fx)
    learned = args.learned and model is not None
    sched = fx.FX_SCHED_MLP if learned else fx.FX_SCHED_BOUND
    # the build timed: mixed precision, the whole call captured once in a
    # hipGraph and replayed, units in bound-only order (the learned order is
    # timed beside it below and has measured slower: the headline takes the
    # faster schedule; --learned times the learned one instead)
    opts_head = fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=not args.no_graph, schedule=sched,
                             costmodel=model if learned else None, symmetry=sym)

    for i in range(args.warmup):
        log(f"bench: warmup {i}")
        fx.fx_exchange_ex(tree, P, tau, K, opts_head, stats=False)
        torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps (mixed, graph={not args.no_graph}, "
        f"schedule={'mlp' if learned else 'bound'})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        fx.fx_exchange_ex(tree, P, tau, K, opts_head, stats=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    # the other unit order beside it: alternating runs of both, same K bitwise
    order_cmp = None
    if model is not None and not args.no_mlp:
        other = fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=not args.no_graph,
                             schedule=fx.FX_SCHED_BOUND if learned else fx.FX_SCHED_MLP,
                             costmodel=None if learned else model, symmetry=sym)
        Ko = torch.zeros_like(P)
        fx.fx_exchange_ex(tree, P, tau, Ko, other, stats=False)
        torch.cuda.synchronize()
        ts = {"head": [], "other": []}
        for r in range(2):
            for k, o in ((("head", opts_head), ("other", other)) if r == 0 else (("other", other), ("head", opts_head))):
                t = time.perf_counter()
                fx.fx_exchange_ex(tree, P, tau, Ko if k == "other" else K, o, stats=False)
                torch.cuda.synchronize()
                ts[k].append(time.perf_counter() - t)
        log(f"bench: unit orders, headline {ts['head']} s, other {ts['other']} s")
        lo, bo = (ts["head"], ts["other"]) if learned else (ts["other"], ts["head"])
        order_cmp = {"learned_order_s": float(np.median(lo)), "bound_order_s": float(np.median(bo)),
                     "learned_runs_s": lo, "bound_runs_s": bo, "K_bitwise_equal": bool(torch.equal(Ko, K))}
        del Ko
    # counts of the same build (one more call that waits for its statistics)
    _, st = fx.fx_exchange_ex(tree, P, tau, K, opts_head)
    quartets_eval = st["quartets"]
    quartets_cov = st["quartets_covered"]
    value = quartets_eval * args.steps / elapsed

    # per-class kernel times: one eager call with HIP events around every
    # class launch (on the launch stream).  A class run in one pass for both
    # precisions (fx_k_<class>_mix) reports its time and launches on the FP64
    # entry and its FP32 work on the other; its peak is the FP64 one (packed
    # FP32 is disabled at compile time, so FP32 instructions issue at the FP64
    # rate).
    log("bench: profiled call (per-class HIP events)")
    Kp = torch.zeros_like(P)
    _, stp = fx.fx_exchange_ex(tree, P, tau, Kp, fx.make_opts(precision=fx.FX_PREC_MIXED, profile=True,
                                                                schedule=sched, costmodel=model if learned else None,
                                                                symmetry=sym))
    same_profiled = bool(torch.equal(Kp, K))
    del Kp
    cs, cl, cf, cq = stp["class_seconds"], stp["class_launches"], stp["class_flops"], stp["class_prec_quartets"]
    dual = (cl[:, 0] > 0) & (cl[:, 1] == 0) & (cf[:, 1] > 0)

    def kernel(c, p):
        tag = "mix" if dual[c] else ("f32" if p else "f64")
        flops = cf[c, 0] + cf[c, 1] if dual[c] else cf[c, p]
        quartets = cq[c, 0] + cq[c, 1] if dual[c] else cq[c, p]
        return f"fx_k_{cname(c)[1:3]}{cname(c)[4:6]}_{tag}", tag, flops, int(quartets)

    c, p = np.unravel_index(int(np.argmax(cs)), cs.shape)
    kname, tag, kflops, _ = kernel(c, p)
    per_launch_flops = kflops / max(1, cl[c, p])
    avg_launch_s = cs[c, p] / max(1, cl[c, p])
    achieved = per_launch_flops / avg_launch_s / 1e12
    peak = FP32_PEAK_TFLOPS if tag == "f32" else FP64_PEAK_TFLOPS
    traffic, traffic_src = profiled_traffic(kname)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
                "traffic_source": traffic_src,
                "traffic_GBps": traffic / avg_launch_s / 1e9 if traffic else None, "kernel": kname,
                "class": cname(c), "avg_launch_ms": 1e3 * avg_launch_s,
                "flops_per_launch": per_launch_flops,
                "limiter": "private-memory (scratch) traffic of the spilled [e0|f0] block, not the ALU: see "
                           "traffic (HBM bytes per launch from the counters) against the algorithmic bytes",
                "all_class_kernels_tflops": float(cf.sum() / cs.sum() / 1e12) if cs.sum() > 0 else None}
    order = np.argsort(-cs.reshape(-1))[:12]
    top = []
    for idx in order:
        cc, pp = divmod(int(idx), 2)
        if cs[cc, pp] <= 0:
            continue
        _, tg, fl, qq = kernel(cc, pp)
        top.append({"class": cname(cc), "prec": tg, "s": float(cs[cc, pp]), "tflops": float(fl / cs[cc, pp] / 1e12),
                    "quartets": qq})
    roofline["top_class_kernels"] = top
    if traffic:
        # the roof the counters put the kernel against: its HBM bytes (private-memory
        # traffic included) per second against 8 TB/s, next to its algorithmic ALU fraction
        hbm_frac = traffic / avg_launch_s / (HBM_PEAK_GBPS * 1e9)
        roofline["traffic_frac_of_hbm_peak"] = hbm_frac
        roofline["measured_bound"] = "hbm" if hbm_frac > roofline["frac"] else "alu"

    extra = {}
    if not args.no_fp64:
        # the plain FP64 GPU build: bound-only order, no graph; median of runs
        log(f"bench: FP64 comparison build, 1 warmup + {args.fp64_steps} timed runs")
        o64 = fx.make_opts(precision=fx.FX_PREC_FP64, symmetry=sym)
        K64 = torch.zeros_like(P)
        fx.fx_exchange_ex(tree, P, tau, K64, o64, stats=False)
        torch.cuda.synchronize()
        times64 = []
        for _ in range(args.fp64_steps):
            t = time.perf_counter()
            fx.fx_exchange_ex(tree, P, tau, K64, o64, stats=False)
            torch.cuda.synchronize()
            times64.append(time.perf_counter() - t)
        _, st64 = fx.fx_exchange_ex(tree, P, tau, K64, o64)
        t64 = float(np.median(times64))
        dK = (K - K64).abs()
        extra = {"fp64_kbuild_s": t64, "fp64_kbuild_s_runs": times64,
                 "fp64_quartets_per_s": st64["quartets"] / t64,
                 "mixed_speedup_vs_fp64": t64 / (elapsed / args.steps),
                 "mixed_err_maxabs": float(dK.max()), "mixed_err_frob": float(torch.linalg.norm(K - K64)),
                 "mixed_err_exchange_energy": float(abs(0.25 * ((P * (K - K64)).sum()))),
                 # a-priori bound of the Frobenius change: c * u32 * sum of beta over the FP32
                 # quartets (u32 = 2^-24), given here for c = 1 (c is the growth of a quartet's
                 # FP32 rounding through its recurrences)
                 "mixed_err_bound_frob_c1": 2.0 ** -24 * st["fp32_beta_sum"],
                 "fp32_beta_sum": st["fp32_beta_sum"],
                 "mixed_err_note": "mixed K minus FP64 K of this library (the FP64 path matches the oracle to "
                                   "1e-10 in the tests); FP32 instructions issue at the FP64 rate here (packed "
                                   "FP32 is off), so the speed-up comes from smaller register and private-memory "
                                   "footprints, not from a faster FP32 ALU",
                 "same_quartets": int(st64["quartets_covered"]) == int(quartets_cov)
                 and int(st64["quartets"]) == int(quartets_eval)}
        del K64

    cpu = None
    if not args.no_cpu:
        log("bench: CPU oracle baseline (one thread, all threads)")
        cpu = cpu_baseline(system, quartets_cov, args.cpu_seconds)

    out = {"metric": "K-build s & ERI quartets/s at tau=1e-8, mixed vs FP64, 1000-atom s+p+d",
           "value": value, "unit": "quartets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": f"{args.natom}-atom s+p+d cluster, n={system.nbf}, tau=1e-8, mixed precision, "
                                  f"graph-captured, {'learned' if learned else 'bound-only'} unit order",
                      "natom": args.natom, "nbf": system.nbf, "tau": tau, "parallelism": "single-gpu"},
           "value_note": "value counts the shell quartets whose integrals were evaluated (ERIs); with a "
                         "symmetric density each stands for itself and its mirror, and the K-coverage rate "
                         "counts both (the set the oracle evaluates and the CPU baseline counts)",
           "kbuild_s": elapsed / args.steps, "quartets_evaluated": int(quartets_eval),
           "quartets_covered": int(quartets_cov),
           "k_coverage_quartets_per_s": quartets_cov * args.steps / elapsed,
           "symmetric": bool(st["symmetric_systems"]), "quartets_fp32": int(st["quartets_fp32"]),
           "prim_quartets": st["prim_quartets"], "alg_flops": st["flops"],
           "alg_tflops": st["flops"] / (elapsed / args.steps) / 1e12, "tree_build_s": t_tree,
           "workspace_bytes": st["workspace_bytes"], "graph": st["graph_nodes"] == 1,
           "schedule": "mlp" if learned else "bound", "unit_orders": order_cmp,
           "profiled_K_equal": same_profiled,
           "autotuned_entries": tuned, "tuning_table": tuning_table_info(), "roofline": roofline,
           "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out))


def copy_probe():
    """One elementwise kernel that reads and writes 1 GiB each (after a
    warm-up pass): the reference for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe": True, "bytes_read": 8 * n, "bytes_written": 8 * n, "dispatches": 2}))


def bench_scaling(args, log):
    """K-build time against system size: s+p+d clusters at 0.1 atoms/A^3
    (the benchmark's recipe, seeds 2000 + natom), tau = 1e-8, mixed
    precision.  Reports time and quartets per size and the log-log slope
    between consecutive sizes (1 = linear scaling)."""
    import numpy as np
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    sizes = tuple(int(x) for x in args.sizes.split(","))
    # one stderr line per finished K row range: large sizes run many ranges
    fx.set_progress_stderr("bench: scaling")
    rows = []
    for natom in sizes:
        log(f"bench: scaling {natom} atoms: first call (sizes its buffers)")
        s = synthetic.cluster(natom, seed=2000 + natom)
        tree = fx.build_quadtree_from(s)
        P = torch.from_numpy(s.P).cuda()
        K = torch.zeros_like(P)
        opts = fx.make_opts(precision=fx.FX_PREC_MIXED)
        fx.fx_exchange_ex(tree, P, s.tau, K, opts)
        torch.cuda.synchronize()
        log(f"bench: scaling {natom} atoms: timed call")
        t = time.perf_counter()
        _, st = fx.fx_exchange_ex(tree, P, s.tau, K, opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        rows.append({"natom": natom, "nbf": s.nbf, "kbuild_s": el, "quartets": st["quartets_covered"],
                     "quartets_evaluated": st["quartets"], "workspace_bytes": st["workspace_bytes"],
                     "row_ranges": st["chunks"] + 1})
        log(f"bench: scaling {natom} atoms n={s.nbf}: {el:.3f} s, {st['quartets_covered']:.3e} quartets")
        del tree, P, K
        torch.cuda.empty_cache()
    for a, b in zip(rows, rows[1:]):
        b["slope_time"] = float(np.log(b["kbuild_s"] / a["kbuild_s"]) / np.log(b["natom"] / a["natom"]))
        b["slope_quartets"] = float(np.log(b["quartets"] / a["quartets"]) / np.log(b["natom"] / a["natom"]))
    last = rows[-1]
    print(json.dumps({"metric": f"K-build s vs size, s+p+d clusters {args.sizes} atoms, tau=1e-8, mixed",
                      "value": last["quartets"] / last["kbuild_s"], "unit": "quartets/s", "n_gpus": 1, "steps": 1,
                      "warmup": 1, "ms_per_step": 1e3 * last["kbuild_s"], "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
                      "config": {"workload": f"s+p+d clusters of {args.sizes} atoms at 0.1 atoms/A^3"},
                      "series": rows}))


def _timed_build(fx, torch, s, opts, tau, runs=3):
    """Median K-build time of a few asynchronous calls (after one that sizes
    the buffers), and the statistics of one more."""
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    K = torch.zeros_like(P)
    fx.fx_exchange_ex(tree, P, tau, K, opts, stats=False)
    torch.cuda.synchronize()
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        fx.fx_exchange_ex(tree, P, tau, K, opts, stats=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    _, st = fx.fx_exchange_ex(tree, P, tau, K, opts)
    return float(np.median(ts)), st


def _slopes(rows, xkey, keys):
    for a, b in zip(rows, rows[1:]):
        for k in keys:
            b["slope_" + k] = float(np.log(b[k] / a[k]) / np.log(b[xkey] / a[xkey]))


def bench_regimes(args, log):
    """The analogue of the paper's size series (its Fig. 1 data are not
    available): synthetic s+p+d clusters at 0.1 atoms/A^3 (seeds 2000 + N),
    mixed precision, at the paper's two threshold pairs (tau, tau_ovlp) =
    (1e-8, 1e-11) and (1e-10, 1e-13), with the metric query alone at 1e-8 for
    reference; K-build seconds, quartets and log-log slopes."""
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    sizes = (125, 250, 500, 1000)
    regimes = ((1e-8, 0.0), (1e-8, 1e-11), (1e-10, 1e-13))
    fx.set_progress_stderr("bench: regimes")
    series = {}
    for tau, tov in regimes:
        rows = []
        for natom in sizes:
            s = synthetic.cluster(natom, seed=2000 + natom, tau=tau)
            sec, st = _timed_build(fx, torch, s, fx.make_opts(precision=fx.FX_PREC_MIXED, tau_ovlp=tov), tau)
            rows.append({"natom": natom, "nbf": s.nbf, "kbuild_s": sec, "quartets": st["quartets_covered"],
                         "quartets_evaluated": st["quartets"], "leaf_entries": st["frontier"][-1]})
            log(f"bench: regimes tau={tau} tau_ovlp={tov} {natom} atoms: {sec:.3f} s, "
                f"{st['quartets_covered']:.3e} quartets")
            torch.cuda.empty_cache()
        _slopes(rows, "natom", ("kbuild_s", "quartets"))
        series[f"tau={tau:g},tau_ovlp={tov:g}"] = rows
    last = series["tau=1e-08,tau_ovlp=1e-11"][-1]
    print(json.dumps({"metric": "K-build s vs size at two threshold pairs, s+p+d clusters 125..1000 atoms, mixed",
                      "value": last["quartets_evaluated"] / last["kbuild_s"], "unit": "quartets/s", "n_gpus": 1,
                      "steps": 3, "warmup": 1, "ms_per_step": 1e3 * last["kbuild_s"], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
                      "config": {"workload": "s+p+d clusters of 125, 250, 500, 1000 atoms at 0.1 atoms/A^3"},
                      "series": series}))


def bench_chain(args, log):
    """s+p chains of 50..3200 atoms (1.5 A spacing, 0.1 A jitter, seeds
    3000 + N), tau = 1e-8, FP64 and mixed: the quartets that survive grow
    linearly with the chain, and so does the K-build time once launch
    overhead is amortised."""
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    fx.set_progress_stderr("bench: chain")
    rows = []
    for natom in (50, 100, 200, 400, 800, 1600, 3200):
        s = synthetic.chain(natom, seed=3000 + natom)
        sec, st = _timed_build(fx, torch, s, fx.make_opts(precision=fx.FX_PREC_FP64), s.tau, runs=5)
        rows.append({"natom": natom, "nbf": s.nbf, "kbuild_s": sec, "quartets": st["quartets_covered"],
                     "quartets_evaluated": st["quartets"]})
        log(f"bench: chain {natom} atoms: {sec * 1e3:.2f} ms, {st['quartets_covered']:.3e} quartets")
    _slopes(rows, "natom", ("kbuild_s", "quartets"))
    last = rows[-1]
    print(json.dumps({"metric": "K-build s vs chain length, s+p chains 50..3200 atoms, tau=1e-8, FP64",
                      "value": last["quartets_evaluated"] / last["kbuild_s"], "unit": "quartets/s", "n_gpus": 1,
                      "steps": 5, "warmup": 1, "ms_per_step": 1e3 * last["kbuild_s"], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "s+p chains of 50..3200 atoms, 1.5 A spacing"}, "series": rows}))


def bench_multi(args, log):
    """Two densities of the 1000-atom s+p+d cluster (the benchmark's P and a
    second one from the same recipe, seed 7002), mixed precision: one
    fx_exchange_multi call against two fx_exchange_ex calls."""
    import numpy as np
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    s = synthetic.cluster(args.natom)
    P2 = synthetic.make_density(np.random.default_rng(7002), s.atoms, s.func_atom(), 2.0)
    tree = fx.build_quadtree_from(s)
    Ps = [torch.from_numpy(s.P).cuda(), torch.from_numpy(P2).cuda()]
    del P2
    opts = fx.make_opts(precision=fx.FX_PREC_MIXED)
    Ks = [torch.zeros_like(P) for P in Ps]
    for _ in range(args.warmup):
        fx.fx_exchange_multi(tree, Ps, Ks, s.tau, opts)
    torch.cuda.synchronize()
    log("bench: two densities in one call")
    t = time.perf_counter()
    for _ in range(args.steps):
        _, st = fx.fx_exchange_multi(tree, Ps, Ks, s.tau, opts)
    torch.cuda.synchronize()
    tm = (time.perf_counter() - t) / args.steps
    log("bench: two single builds")
    K1 = [torch.zeros_like(P) for P in Ps]
    t = time.perf_counter()
    q = 0
    for P, K in zip(Ps, K1):
        _, s1 = fx.fx_exchange_ex(tree, P, s.tau, K, opts)
        q += s1["quartets_covered"]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    dk = max(float((a - b).abs().max()) for a, b in zip(Ks, K1))
    print(json.dumps({"metric": "K-build s, two densities, 1000-atom s+p+d, tau=1e-8, mixed",
                      "value": 2 * st["quartets_covered"] / tm, "unit": "quartet-density contractions/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * tm,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
                      "data": "synthetic",
                      "config": {"workload": f"{args.natom}-atom s+p+d cluster, two densities, one call",
                                 "nbf": s.nbf},
                      "multi_s": tm, "two_single_s": ts, "speedup": ts / tm,
                      "quartets": st["quartets_covered"], "single_quartets": q,
                      "max_abs_diff_vs_single": dk}))


def bench_batched(args, log):
    """64 clusters (50..500 atoms, s+p) in one batched call, the whole call
    captured once in a hipGraph and replayed, vs 64 sequential single builds
    enqueued one after another; K bitwise equal."""
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    systems = synthetic.batch_clusters(64)
    trees = [fx.build_quadtree_from(s) for s in systems]
    Ps = [torch.from_numpy(s.P).cuda() for s in systems]
    tau = systems[0].tau
    steps = max(3, args.steps)
    opts = fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=True)
    Kb = [torch.zeros_like(P) for P in Ps]
    for _ in range(max(1, args.warmup)):
        fx.fx_exchange_batched(trees, Ps, Kb, tau, opts, stats=False)   # sizes, then capture
    fx.fx_exchange_batched(trees, Ps, Kb, tau, opts, stats=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fx.fx_exchange_batched(trees, Ps, Kb, tau, opts, stats=False)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t) / steps
    _, st = fx.fx_exchange_batched(trees, Ps, Kb, tau, opts)
    log("bench: 64 sequential builds")
    Ks = [torch.zeros_like(P) for P in Ps]
    so = fx.make_opts(precision=fx.FX_PREC_MIXED)
    for tr, P, K in zip(trees, Ps, Ks):
        fx.fx_exchange_ex(tr, P, tau, K, so, stats=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        for tr, P, K in zip(trees, Ps, Ks):
            fx.fx_exchange_ex(tr, P, tau, K, so, stats=False)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t) / steps
    same = all(torch.equal(a, b_) for a, b_ in zip(Kb, Ks))
    print(json.dumps({"metric": "batched K-build s, 64 clusters 50-500 atoms s+p, tau=1e-8, mixed",
                      "value": st["quartets"] / tb, "unit": "quartets/s", "n_gpus": 1, "steps": steps,
                      "warmup": args.warmup, "ms_per_step": 1e3 * tb, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
                      "config": {"workload": "64 s+p clusters, log-uniform 50..500 atoms, one batched call "
                                             "captured once and replayed", "systems": 64,
                                 "nbf_total": int(sum(s.nbf for s in systems))},
                      "batched_s": tb, "sequential_s": ts, "speedup": ts / tb,
                      "quartets": st["quartets_covered"], "quartets_evaluated": st["quartets"],
                      "graph": st["graph_nodes"] == 1, "K_bitwise_equal": bool(same)}))


def bench_slab_mlp(args, log):
    """4000-atom s+p slab: learned (MLP) vs bound-only unit order, the same K
    bitwise; runs alternate between the two orders.  The model is the one
    the library ships (trained on the chain, cluster and batch workloads),
    trained here on the same workloads when it is missing."""
    import numpy as np
    import torch
    import synthetic
    import paper_1401_6961_amd as fx
    model = shipped_costmodel(fx)
    trained_here = model is None
    if model is None:
        from paper_1401_6961_amd import train_costmodel
        path = os.path.join(ROOT, "_build", "costmodel_bench.fxmlp")
        os.makedirs(os.path.dirname(path), exist_ok=True)
        train_costmodel.main(["--out", path, "--steps", "2000"])
        model = fx.CostModel.load(path)
    s = synthetic.slab(args.natom if args.natom != 1000 else 4000)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    runs = max(5, args.steps)
    opts = {"bound": fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=fx.FX_SCHED_BOUND),
            "mlp": fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=fx.FX_SCHED_MLP, costmodel=model)}
    Ks = {k: torch.zeros_like(P) for k in opts}
    for k, o in opts.items():
        fx.fx_exchange_ex(tree, P, s.tau, Ks[k], o, stats=False)
    torch.cuda.synchronize()
    times = {k: [] for k in opts}
    for r in range(runs):
        for k in (("bound", "mlp") if r % 2 == 0 else ("mlp", "bound")):
            t0 = time.perf_counter()
            fx.fx_exchange_ex(tree, P, s.tau, Ks[k], opts[k], stats=False)
            torch.cuda.synchronize()
            times[k].append(time.perf_counter() - t0)
        log(f"bench: slab run {r}: bound {times['bound'][-1]:.3f} s, mlp {times['mlp'][-1]:.3f} s")
    _, st = fx.fx_exchange_ex(tree, P, s.tau, Ks["mlp"], opts["mlp"])
    med = {k: float(np.median(v)) for k, v in times.items()}
    print(json.dumps({"metric": "K-build s, 4000-atom s+p slab, tau=1e-8, mixed, learned vs bound-only scheduling",
                      "value": st["quartets"] / med["mlp"], "unit": "quartets/s", "n_gpus": 1, "steps": runs,
                      "warmup": 1, "ms_per_step": 1e3 * med["mlp"], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
                      "config": {"workload": f"{s.nbf // 4}-atom s+p slab 40x40x25 A, n={s.nbf}", "nbf": s.nbf},
                      "mlp_s": med["mlp"], "bound_s": med["bound"], "mlp_gain": med["bound"] / med["mlp"],
                      "mlp_runs_s": times["mlp"], "bound_runs_s": times["bound"], "model_trained_here": trained_here,
                      "quartets": st["quartets_covered"],
                      "K_bitwise_equal": bool(torch.equal(Ks["bound"], Ks["mlp"]))}))


if __name__ == "__main__":
    main()
