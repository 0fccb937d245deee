"""Autotuner of the class kernels.

For every angular-momentum class it chooses between two passes (one kernel
per precision, each with its form -- one quartet per lane, or one quartet
per wave with LDS intermediates, where both are built -- and its launch
mapping, plain or XCD-aware workgroup order) and one pass for both
precisions (variant 2 on the FP64 entry), whichever runs fastest on a
representative workload.  Each candidate setting is applied to all classes
at once, the workload is built with per-launch HIP event timing, and the
fastest setting per class wins.  The launch mapping never changes K; the
form and the number of passes change only the order of the sums inside a
K block (K equal to rounding; tests check both).

    python -m paper_1401_6961_amd.autotune --natom 300 --out tuning_gfx950.json

apply(path) loads a table into the library (process-wide).

The generator's per-kernel choices (the "generator" section: routine form,
pairing, waves per SIMD, one-pass mixed precision) are compile-time, so
they are tuned on candidate libraries, each built from the current table
with one choice changed for every kernel it applies to; a class's kernels
are timed in every candidate and the candidate fastest for that class
gives the class's entries (classes are separate kernels, so their choices
do not interact):

    python -m paper_1401_6961_amd.autotune --generator build --dir DIR    # CPU
    python -m paper_1401_6961_amd.autotune --generator measure --dir DIR  # GPU
    python -m paper_1401_6961_amd.autotune --generator choose --dir DIR   # CPU, rewrites the table
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning_gfx950.json")


def apply(path: str = DEFAULT_TABLE) -> int:
    """Load a tuning table; returns the number of (class, precision) entries set."""
    from . import fx
    if not os.path.exists(path):
        return 0
    table = json.load(open(path))
    n = 0
    for key, ent in table.get("classes", {}).items():
        cls, prec = (int(x) for x in key.split(":"))
        if fx.fx_class_variants_available(cls) & (1 << ent["variant"]):
            fx.fx_set_class_variant(cls, prec, ent["variant"])
        fx.fx_set_class_launch(cls, prec, ent["flags"])
        n += 1
    return n


def tune(natom=300, with_d=True, seed=1002, repeats=2, log=print, full=False):
    """Per class: two passes (one kernel per precision, each with its form and
    launch order chosen independently) or one pass for both precisions
    (variant 2 on the FP64 entry, with its launch order), whichever took less
    time in the mixed build."""
    import numpy as np
    import torch

    import synthetic
    from . import fx

    system = synthetic.cluster(natom, seed=seed, with_d=with_d)
    tree = fx.build_quadtree_from(system)
    P = torch.from_numpy(system.P).cuda()
    K = torch.zeros_like(P)
    # the cooperative form and the XCD-aware order lose by large factors at
    # this size (1000-atom cluster: 151.6 s and 99.2 s against 15.4 s of class
    # time), so only a full sweep times them
    configs = [(v, f) for v in (0, 1, 2) for f in (0, 1)] if full else [(0, 0), (2, 0)]
    times = {}
    for v, f in configs:
        for cls in range(81):
            avail = fx.fx_class_variants_available(cls)
            for p in (0, 1):
                if v == 2:
                    # one pass: the FP64 entry runs both precisions
                    fx.fx_set_class_variant(cls, p, 2 if p == 0 else 0)
                elif avail & (1 << v):
                    fx.fx_set_class_variant(cls, p, v)
                else:
                    fx.fx_set_class_variant(cls, p, 0 if v else 1)
                fx.fx_set_class_launch(cls, p, f)
        best = None
        for r in range(repeats):
            _, st = fx.fx_exchange_ex(tree, P, system.tau, K, fx.make_opts(precision=fx.FX_PREC_MIXED, profile=True))
            cs = st["class_seconds"]
            best = cs if best is None else np.minimum(best, cs)
            log(f"autotune: variant={v} xcd={f} run {r}: {cs.sum():.3f} s")
        times[(v, f)] = best
        log(f"autotune: variant={v} xcd={f} total class time {best.sum():.3f} s")
    table = {"workload": f"{natom}-atom {'s+p+d' if with_d else 's+p'} cluster, mixed precision",
             "device": torch.cuda.get_device_name(0), "classes": {}}
    for cls in range(81):
        avail = fx.fx_class_variants_available(cls)
        two = []
        for p in (0, 1):
            cands = [(float(times[(v, f)][cls, p]), v, f) for (v, f) in configs
                     if v < 2 and avail & (1 << v) and times[(v, f)][cls, p] > 0]
            two.append(min(cands) if cands else None)
        one = [(float(times[(2, f)][cls, 0]), 2, f) for f in (0, 1)
               if (2, f) in times and avail & 4 and times[(2, f)][cls, 0] > 0]
        one = min(one) if one else None
        t_two = sum(x[0] for x in two if x) if all(two) else None
        if one and (t_two is None or one[0] < t_two):
            table["classes"][f"{cls}:0"] = {"variant": 2, "flags": one[2], "ms": 1e3 * one[0]}
            table["classes"][f"{cls}:1"] = {"variant": 0, "flags": one[2], "ms": None}
        else:
            for p in (0, 1):
                if two[p]:
                    t, v, f = two[p]
                    table["classes"][f"{cls}:{p}"] = {"variant": v, "flags": f, "ms": 1e3 * t}
    return table


# ---------------------------------------------------------------------------
# generator choices
# ---------------------------------------------------------------------------
CANDIDATES = ("current", "folded", "folded_w2", "unpaired", "waves2", "dual_all", "dual_none")


def candidate_kernels(name, kernels):
    """The generator entries of candidate `name`, derived from `kernels`."""
    k = {key: dict(e) for key, e in kernels.items()}
    routines = [key for key in k if not key.endswith(":mix")]
    classes = sorted({key.split(":")[0] for key in routines})
    if name == "register":
        for key in routines:
            k[key] = {"form": "register", "waves": 1}
    elif name.startswith("folded"):
        w = int(name[-1]) if name[-2:-1] == "w" else 1
        for key in routines:
            if "d" in key.split(":")[0]:
                k[key] = {"form": "folded", "paired": True, "waves": w}
    elif name == "unpaired":
        for key in routines:
            if k[key].get("form", "register") != "register":
                k[key]["paired"] = False
    elif name == "waves2":
        for key in k:
            k[key]["waves"] = 2
    elif name == "dual_all":
        for c in classes:
            k.setdefault(f"{c}:mix", {"waves": 1})
    elif name == "dual_none":
        k = {key: e for key, e in k.items() if not key.endswith(":mix")}
    elif name != "current":
        raise ValueError(f"unknown candidate {name}")
    return k


def generator_build(d, table_path=DEFAULT_TABLE, names=CANDIDATES, log=print):
    """Candidate libraries under d/<name>/ (objects shared with the package build)."""
    from . import build as B
    table = json.load(open(table_path))
    for name in names:
        cdir = os.path.join(d, name)
        os.makedirs(os.path.join(cdir, "gen"), exist_ok=True)
        t = dict(table)
        t["generator"] = dict(table["generator"], kernels=candidate_kernels(name, table["generator"]["kernels"]))
        tp = os.path.join(cdir, "table.json")
        with open(tp, "w") as fh:
            json.dump(t, fh, indent=1, sort_keys=True)
        log(f"autotune: building candidate {name}")
        B.build(incremental=True, table=tp, gen=os.path.join(cdir, "gen"), lib=os.path.join(cdir, "libfx.so"))


def time_classes(natom, repeats, seed=1002, log=print):
    """Per (class, precision slot) kernel seconds of the mixed build of the
    natom s+p+d cluster with the loaded library (least of `repeats`)."""
    import numpy as np
    import torch

    import synthetic
    from . import fx
    apply()
    system = synthetic.cluster(natom)
    tree = fx.build_quadtree_from(system)
    P = torch.from_numpy(system.P).cuda()
    K = torch.zeros_like(P)
    fx.fx_exchange_ex(tree, P, system.tau, K, fx.make_opts(precision=fx.FX_PREC_MIXED), stats=False)
    torch.cuda.synchronize()
    log("autotune: first call done")
    best = None
    for r in range(repeats):
        _, st = fx.fx_exchange_ex(tree, P, system.tau, K, fx.make_opts(precision=fx.FX_PREC_MIXED, profile=True))
        cs = st["class_seconds"]
        best = cs if best is None else np.minimum(best, cs)
        log(f"autotune: timed call {r}: class time {cs.sum():.3f} s")
    return best


def generator_measure(d, natom=1000, repeats=2, names=CANDIDATES, log=print):
    """Time every candidate library in a child process of its own (a library
    is loaded once per process); d/<name>/times.json."""
    import subprocess
    for name in names:
        lib = os.path.join(d, name, "libfx.so")
        if not os.path.exists(lib):
            continue
        out = os.path.join(d, name, "times.json")
        log(f"autotune: timing candidate {name}")
        r = subprocess.run([sys.executable, "-m", "paper_1401_6961_amd.autotune", "--time-lib", lib, "--natom",
                            str(natom), "--repeats", str(repeats), "--out", out],
                           cwd=os.path.dirname(HERE), timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"timing candidate {name} failed with status {r.returncode}")


def generator_choose(d, table_path=DEFAULT_TABLE, names=CANDIDATES, log=print):
    """Per class, the entries of the candidate whose kernels of that class
    took least time in the mixed build (both precision slots summed)."""
    import numpy as np
    table = json.load(open(table_path))
    cur = table["generator"]["kernels"]
    times, kern = {}, {}
    for name in names:
        tp = os.path.join(d, name, "times.json")
        if os.path.exists(tp):
            times[name] = np.asarray(json.load(open(tp))["class_seconds"])
            kern[name] = json.load(open(os.path.join(d, name, "table.json")))["generator"]["kernels"]
    if "current" not in times:
        raise RuntimeError("the current table's candidate was not timed")
    L = "spd"
    new, chosen = {}, {}
    for c in range(81):
        cls = L[c // 27] + L[(c // 9) % 3] + L[(c // 3) % 3] + L[c % 3]
        best = min(times, key=lambda nm: (float(times[nm][c].sum()) if times[nm][c].sum() > 0 else 1e30,
                                          nm != "current"))
        chosen[cls] = (best, float(times[best][c].sum()), float(times["current"][c].sum()))
        for key, e in kern[best].items():
            if key.split(":")[0] == cls:
                new[key] = e
    before = sum(v[2] for v in chosen.values())
    after = sum(v[1] for v in chosen.values())
    changed = {c: v[0] for c, v in chosen.items() if v[0] != "current"}
    log(f"autotune: class time {before:.3f} s with the current table, {after:.3f} s with the choices; "
        f"{len(changed)} classes changed: {changed}")
    table["generator"] = dict(table["generator"], kernels=new,
                              tuned={"candidates": sorted(times), "class_seconds_before": before,
                                     "class_seconds_after": after})
    with open(table_path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--natom", type=int, default=300)
    ap.add_argument("--sp", action="store_true", help="s+p shells only")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--base", default=DEFAULT_TABLE, help="table whose generator section the result keeps")
    ap.add_argument("--generator", choices=["build", "measure", "choose"], help="tune the generator's choices")
    ap.add_argument("--dir", default=os.path.join(os.path.dirname(HERE), "_autotune"))
    ap.add_argument("--candidates", default=",".join(CANDIDATES))
    ap.add_argument("--full", action="store_true", help="also time the cooperative form and the XCD-aware order")
    ap.add_argument("--time-lib", help=argparse.SUPPRESS)
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    names = tuple(args.candidates.split(","))
    if args.time_lib:
        from . import fx
        fx.LIB_PATH = args.time_lib
        cs = time_classes(args.natom, args.repeats, log=log)
        with open(args.out, "w") as fh:
            json.dump({"lib": args.time_lib, "natom": args.natom, "class_seconds": cs.tolist()}, fh)
        log(f"autotune: {args.time_lib}: class time {cs.sum():.3f} s")
        return
    if args.generator == "build":
        return generator_build(args.dir, names=names, log=log)
    if args.generator == "measure":
        return generator_measure(args.dir, args.natom, args.repeats, names=names, log=log)
    if args.generator == "choose":
        return generator_choose(args.dir, names=names, log=log)
    table = tune(args.natom, with_d=not args.sp, log=lambda m: print(m, flush=True), full=args.full)
    if os.path.exists(args.base):
        # keep the generator's choices
        table = dict(json.load(open(args.base)), **table)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print(f"autotune: wrote {len(table['classes'])} entries to {args.out}", flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
