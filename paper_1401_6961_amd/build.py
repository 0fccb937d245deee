"""Build libfx.so for gfx950: generate the class kernels, compile every HIP
and C++ source with hipcc (in parallel), link the shared library in-tree.

build(incremental=False) recompiles everything; with incremental=True (or
FX_BUILD_INCREMENTAL=1) objects whose source, headers and flags are
unchanged are reused from _build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(CSRC, "gen")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _flags(gen=GEN):
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", CSRC, "-I", gen, "-I", os.path.join(ROOT, "include"),
            "-Wno-unused-variable", "-Wno-unused-lambda-capture"]


HIP_FLAGS = _flags()


def _sources(gen=GEN):
    srcs = [os.path.join(CSRC, f) for f in ("fx_kernels.hip", "fx_host.cpp", "fx_exec.cpp", "fx_noalloc.cpp", "fx_costmodel.hip")
            if os.path.exists(os.path.join(CSRC, f))]
    srcs += sorted(os.path.join(gen, f) for f in os.listdir(gen) if f.endswith(".hip"))
    return srcs


# Headers a generated class-kernel source can include (directly or through
# fx_eri_common.h); every other source may include any header.
CLASS_HEADERS = ("fx_eri_common.h", "fx_internal.h")


def _headers_digest(only=None, gen=GEN):
    h = hashlib.sha256()
    for d in (CSRC, gen, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h") and (only is None or f in only):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def _digest_for(src, full, classes):
    """Class-kernel sources depend on the kernel-template headers only."""
    return classes if os.path.basename(src).startswith("eri_") else full


def _compile(src, hdr_digest, incremental, flags=HIP_FLAGS):
    h = hashlib.sha256()
    h.update(open(src, "rb").read())
    h.update(hdr_digest.encode())
    # the flags without the generation directory: its headers are in hdr_digest
    h.update(" ".join(HIP_FLAGS).encode())
    obj = os.path.join(BUILD, os.path.basename(src) + "." + h.hexdigest()[:16] + ".o")
    if incremental and os.path.exists(obj):
        return obj
    tmp = obj + ".tmp"
    cmd = [HIPCC] + flags + ["-x", "hip", "-c", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stderr[-4000:]}")
    os.replace(tmp, obj)
    return obj


def build(incremental: bool | None = None, jobs: int | None = None, table: str | None = None,
          gen: str = GEN, lib: str = LIB) -> str:
    """Generate the class kernels from the tuning table's generator choices
    (`table`, default the package's), compile and link `lib`.  Another
    table is built into its own `gen` directory and `lib` (the autotuner's
    candidate libraries)."""
    if incremental is None:
        incremental = os.environ.get("FX_BUILD_INCREMENTAL", "0") == "1"
    os.makedirs(BUILD, exist_ok=True)
    sys.path.insert(0, CSRC)
    import gen_eri  # noqa: E402
    gen_eri.load_choices(table or gen_eri.TABLE)
    try:
        gen_eri.main(gen)
    finally:
        gen_eri.load_choices()
    full, classes = _headers_digest(gen=gen), _headers_digest(CLASS_HEADERS, gen=gen)
    flags = _flags(gen)
    srcs = _sources(gen)
    # biggest sources first so the long compiles start early
    srcs.sort(key=lambda s: -os.path.getsize(s))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, _digest_for(s, full, classes), incremental, flags), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    inc = "--incremental" in sys.argv
    print(build(incremental=inc))
