"""Python binding of libfx (ctypes): argument marshalling only.

Every step of the exchange build runs in the library's HIP kernels; PyTorch
is used only for device memory (float64 CUDA tensors) and streams.  The
function names mirror the C ABI in include/fx.h.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfx.so")
_lib = None

FX_PREC_FP64, FX_PREC_MIXED = 0, 1
FX_SCHED_BOUND, FX_SCHED_MLP, FX_SCHED_NONE = 0, 1, 2
FX_SYM_AUTO, FX_SYM_OFF = 0, 1
FX_LEAF_SHELL, FX_LEAF_BLOCK = 0, 1


class FxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


class fx_shells(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int32), ("l", ctypes.POINTER(ctypes.c_int32)),
                ("nprim", ctypes.POINTER(ctypes.c_int32)), ("center", ctypes.POINTER(ctypes.c_double)),
                ("exps", ctypes.POINTER(ctypes.c_double)), ("coefs", ctypes.POINTER(ctypes.c_double))]


class fx_tree_opts(ctypes.Structure):
    _fields_ = [("leaf_max_functions", ctypes.c_int32), ("ordering", ctypes.c_int32)]


class fx_exchange_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("fp32_threshold", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("costmodel", ctypes.c_void_p),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("max_frontier_entries", ctypes.c_int64), ("profile", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("symmetry", ctypes.c_int32), ("leaf_screen", ctypes.c_int32),
                ("tau_ovlp", ctypes.c_double), ("max_workspace_bytes", ctypes.c_int64)]


class fx_train_opts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class fx_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("frontier", ctypes.c_int64 * 32),
                ("leaf_items", ctypes.c_int64), ("units", ctypes.c_int64),
                ("quartets", ctypes.c_int64), ("quartets_fp32", ctypes.c_int64),
                ("class_quartets", ctypes.c_int64 * 81), ("prim_quartets", ctypes.c_double),
                ("flops", ctypes.c_double), ("chunks", ctypes.c_int32), ("graph_nodes", ctypes.c_int32),
                ("class_seconds", ctypes.c_double * 162), ("class_launches", ctypes.c_int32 * 162),
                ("class_flops", ctypes.c_double * 162), ("class_prec_quartets", ctypes.c_int64 * 162),
                ("seconds_traversal", ctypes.c_double), ("seconds_eri", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("quartets_covered", ctypes.c_int64),
                ("symmetric_systems", ctypes.c_int32), ("partition", ctypes.c_int64 * 3),
                ("overflow", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("fp32_beta_sum", ctypes.c_double)]

    def as_dict(self):
        return {"levels": self.levels, "frontier": list(self.frontier)[: self.levels],
                "leaf_items": self.leaf_items, "units": self.units, "quartets": self.quartets,
                "quartets_fp32": self.quartets_fp32,
                "class_quartets": np.array(self.class_quartets, dtype=np.int64).reshape(3, 3, 3, 3),
                "prim_quartets": self.prim_quartets, "flops": self.flops, "chunks": self.chunks,
                "graph_nodes": self.graph_nodes,
                "seconds_traversal": self.seconds_traversal, "seconds_eri": self.seconds_eri,
                "seconds_total": self.seconds_total, "quartets_covered": self.quartets_covered,
                "symmetric_systems": self.symmetric_systems,
                "partition": [int(x) for x in self.partition],
                "overflow": int(self.overflow), "workspace_bytes": int(self.workspace_bytes),
                "fp32_beta_sum": float(self.fp32_beta_sum),
                "class_seconds": np.array(self.class_seconds).reshape(81, 2),
                "class_launches": np.array(self.class_launches).reshape(81, 2),
                "class_flops": np.array(self.class_flops).reshape(81, 2),
                "class_prec_quartets": np.array(self.class_prec_quartets, dtype=np.int64).reshape(81, 2)}


EXPORTED = ["fx_build_quadtree", "fx_exchange", "fx_exchange_ex", "fx_exchange_opts_init", "fx_exchange_noalloc",
            "fx_noalloc_scratch_bytes", "fx_exchange_batched", "fx_exchange_multi", "fx_nbf",
            "fx_nshell",
            "fx_tree_perm", "fx_tree_levels", "fx_tree_schwarz", "fx_tree_overlap", "fx_tree_free", "fx_set_allocator",
            "fx_status_string", "fx_last_error_message", "fx_plan_tree", "fx_hilbert_key3",
            "fx_set_class_variant", "fx_get_class_variant", "fx_class_variants_available",
            "fx_set_class_launch", "fx_get_class_launch", "fx_xcd_block",
            "fx_record_task_timings", "fx_task_timings_create", "fx_task_timings_count", "fx_task_timings_get",
            "fx_task_timings_free", "fx_costmodel_train", "fx_costmodel_nparams", "fx_costmodel_create",
            "fx_costmodel_params", "fx_costmodel_predict", "fx_costmodel_loss_grad", "fx_costmodel_free",
            "fx_costmodel_save", "fx_costmodel_load", "fx_set_progress", "fx_progress_stderr",
            "fx_set_group_screen", "fx_get_group_screen", "fx_plan_row_cuts"]


def lib():
    """Load libfx.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfx.so not found at {LIB_PATH}: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fx_build_quadtree.argtypes = [ctypes.POINTER(fx_shells), ctypes.POINTER(fx_tree_opts), vp,
                                    ctypes.POINTER(vp)]
    L.fx_exchange.argtypes = [vp, vp, dbl, vp, vp]
    L.fx_exchange_ex.argtypes = [vp, vp, dbl, vp, ctypes.POINTER(fx_exchange_opts), ctypes.POINTER(fx_stats), vp]
    L.fx_exchange_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, dbl,
                                      ctypes.POINTER(fx_exchange_opts), ctypes.POINTER(fx_stats), vp]
    L.fx_exchange_multi.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, dbl,
                                    ctypes.POINTER(fx_exchange_opts), ctypes.POINTER(fx_stats), vp]
    L.fx_exchange_noalloc.argtypes = [vp, vp, dbl, vp, ctypes.POINTER(fx_exchange_opts), ctypes.POINTER(fx_stats), vp]
    L.fx_exchange_noalloc.restype = ctypes.c_int
    L.fx_noalloc_scratch_bytes.argtypes = []
    L.fx_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.fx_exchange_opts_init.argtypes = [ctypes.POINTER(fx_exchange_opts)]
    L.fx_exchange_opts_init.restype = None
    L.fx_set_progress.argtypes = [vp, vp]
    L.fx_set_progress.restype = ctypes.c_int
    L.fx_plan_row_cuts.argtypes = [vp, i32, i32, ctypes.POINTER(i32)]
    L.fx_plan_row_cuts.restype = ctypes.c_int
    L.fx_set_group_screen.argtypes = [i32]
    L.fx_set_group_screen.restype = ctypes.c_int
    L.fx_get_group_screen.argtypes = []
    L.fx_get_group_screen.restype = i32
    for f in ("fx_build_quadtree", "fx_exchange", "fx_exchange_ex", "fx_exchange_batched", "fx_exchange_multi", "fx_tree_perm",
              "fx_tree_schwarz", "fx_set_allocator", "fx_plan_tree"):
        getattr(L, f).restype = ctypes.c_int
    L.fx_nbf.argtypes = [vp]
    L.fx_nbf.restype = i32
    L.fx_nshell.argtypes = [vp]
    L.fx_nshell.restype = i32
    L.fx_tree_perm.argtypes = [vp, ctypes.POINTER(i32)]
    L.fx_tree_levels.argtypes = [vp, ctypes.POINTER(i64)]
    L.fx_tree_levels.restype = i32
    L.fx_tree_schwarz.argtypes = [vp, ctypes.POINTER(dbl)]
    L.fx_tree_overlap.argtypes = [vp, ctypes.POINTER(dbl)]
    L.fx_tree_overlap.restype = ctypes.c_int
    L.fx_tree_free.argtypes = [vp]
    L.fx_tree_free.restype = None
    L.fx_status_string.argtypes = [ctypes.c_int]
    L.fx_status_string.restype = ctypes.c_char_p
    L.fx_last_error_message.restype = ctypes.c_char_p
    L.fx_plan_tree.argtypes = [ctypes.POINTER(fx_shells), ctypes.POINTER(fx_tree_opts), ctypes.POINTER(i32),
                               ctypes.POINTER(i32), ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    L.fx_hilbert_key3.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, i32]
    L.fx_hilbert_key3.restype = ctypes.c_uint64
    L.fx_set_class_variant.argtypes = [i32, i32, i32]
    L.fx_set_class_variant.restype = ctypes.c_int
    L.fx_get_class_variant.argtypes = [i32, i32]
    L.fx_get_class_variant.restype = i32
    L.fx_class_variants_available.argtypes = [i32]
    L.fx_class_variants_available.restype = i32
    L.fx_set_class_launch.argtypes = [i32, i32, i32]
    L.fx_set_class_launch.restype = ctypes.c_int
    L.fx_get_class_launch.argtypes = [i32, i32]
    L.fx_get_class_launch.restype = i32
    L.fx_xcd_block.argtypes = [i64, i64]
    L.fx_xcd_block.restype = i64
    fp = ctypes.POINTER(ctypes.c_float)
    L.fx_record_task_timings.argtypes = [vp, vp, dbl, ctypes.POINTER(fx_exchange_opts), ctypes.POINTER(vp), vp]
    L.fx_task_timings_create.argtypes = [fp, fp, ctypes.POINTER(i32), i64, ctypes.POINTER(vp)]
    L.fx_task_timings_count.argtypes = [vp]
    L.fx_task_timings_count.restype = i64
    L.fx_task_timings_get.argtypes = [vp, fp, fp, ctypes.POINTER(i32)]
    L.fx_task_timings_free.argtypes = [vp]
    L.fx_task_timings_free.restype = None
    L.fx_costmodel_train.argtypes = [vp, ctypes.POINTER(fx_train_opts), ctypes.POINTER(vp), fp, vp]
    L.fx_costmodel_nparams.restype = i32
    L.fx_costmodel_create.argtypes = [fp, fp, ctypes.POINTER(vp)]
    L.fx_costmodel_params.argtypes = [vp, fp, fp]
    L.fx_costmodel_predict.argtypes = [vp, fp, i64, fp, vp]
    L.fx_costmodel_loss_grad.argtypes = [vp, fp, fp, i64, fp, fp, vp]
    L.fx_costmodel_free.argtypes = [vp]
    L.fx_costmodel_free.restype = None
    L.fx_costmodel_save.argtypes = [vp, ctypes.c_char_p]
    L.fx_costmodel_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    for f in ("fx_record_task_timings", "fx_task_timings_create", "fx_task_timings_get", "fx_costmodel_train",
              "fx_costmodel_create", "fx_costmodel_params", "fx_costmodel_predict", "fx_costmodel_loss_grad",
              "fx_costmodel_save", "fx_costmodel_load"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def status_string(st):
    return lib().fx_status_string(st).decode()


def _check(st):
    if st != 0:
        raise FxError(st, lib().fx_last_error_message().decode())


class _ShellArrays:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, l, nprim, center, exps, coefs):
        self.l = np.ascontiguousarray(l, np.int32)
        self.nprim = np.ascontiguousarray(nprim, np.int32)
        self.center = np.ascontiguousarray(center, np.float64).reshape(-1)
        self.exps = np.ascontiguousarray(exps, np.float64)
        self.coefs = np.ascontiguousarray(coefs, np.float64)
        P = ctypes.POINTER
        self.s = fx_shells(len(self.l), self.l.ctypes.data_as(P(ctypes.c_int32)),
                           self.nprim.ctypes.data_as(P(ctypes.c_int32)),
                           self.center.ctypes.data_as(P(ctypes.c_double)),
                           self.exps.ctypes.data_as(P(ctypes.c_double)),
                           self.coefs.ctypes.data_as(P(ctypes.c_double)))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_matrix(x, n, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if tuple(x.shape) != (n, n) or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({n}, {n}) tensor")


class Tree:
    """Owning handle of an fx_tree (see fx_build_quadtree)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    @property
    def nbf(self):
        return lib().fx_nbf(self._h)

    @property
    def nshell(self):
        return lib().fx_nshell(self._h)

    def perm(self):
        out = np.zeros(self.nshell, np.int32)
        _check(lib().fx_tree_perm(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def levels(self):
        out = np.zeros(32, np.int64)
        n = lib().fx_tree_levels(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return out[:n]

    def overlap(self):
        S = self.nshell
        out = np.zeros(S * S)
        _check(lib().fx_tree_overlap(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(S, S)

    def schwarz(self):
        S = self.nshell
        out = np.zeros(S * S)
        _check(lib().fx_tree_schwarz(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(S, S)

    def free(self):
        if self._h:
            lib().fx_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fx_build_quadtree(l, nprim, center, exps, coefs, leaf_max_functions=0, ordering=0, stream=None) -> Tree:
    sh = _ShellArrays(l, nprim, center, exps, coefs)
    opts = fx_tree_opts(int(leaf_max_functions), int(ordering))
    h = ctypes.c_void_p()
    _check(lib().fx_build_quadtree(ctypes.byref(sh.s), ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
    return Tree(h.value)


def build_quadtree_from(system, **kw) -> Tree:
    """Convenience: a synthetic.System-like object with l, nprim, center, exps, coefs."""
    return fx_build_quadtree(system.l, system.nprim, system.center, system.exps, system.coefs, **kw)


def plan_row_cuts(leaf_entries, nchunks: int, nleaf: int | None = None) -> np.ndarray:
    """Host-only: the leaf cuts of nchunks K row ranges (fx_plan_row_cuts);
    leaf_entries None gives ranges of about equal leaf counts."""
    if leaf_entries is None:
        if nleaf is None:
            raise ValueError("give leaf_entries or nleaf")
        ptr = None
    else:
        le = np.ascontiguousarray(leaf_entries, dtype=np.int64)
        nleaf = le.shape[0]
        ptr = le.ctypes.data
    cuts = np.zeros(int(nchunks) + 1, dtype=np.int32)
    _check(lib().fx_plan_row_cuts(ptr, int(nleaf), int(nchunks),
                                  cuts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return cuts


def set_group_screen(enabled: bool) -> None:
    """Process-wide: one shared screen per (l_a, l_d) group, or a screen in
    every class kernel (default); K is bitwise the same."""
    _check(lib().fx_set_group_screen(int(bool(enabled))))


def get_group_screen() -> bool:
    return bool(lib().fx_get_group_screen())


_progress_prefix = None


def set_progress_stderr(prefix: str | None = "fx"):
    """Print one line to stderr as each K row range of an eager one-system
    call finishes on the device (the library's own C callback, so no Python
    runs on the runtime thread); None turns it off."""
    global _progress_prefix
    L = lib()
    if prefix is None:
        _check(L.fx_set_progress(None, None))
        _progress_prefix = None
        return
    _progress_prefix = ctypes.create_string_buffer(prefix.encode())
    fn = ctypes.cast(L.fx_progress_stderr, ctypes.c_void_p)
    _check(L.fx_set_progress(fn, ctypes.cast(_progress_prefix, ctypes.c_void_p)))


def opts_init():
    """The library's defaults (fx_exchange_opts_init)."""
    o = fx_exchange_opts()
    lib().fx_exchange_opts_init(ctypes.byref(o))
    return o


def make_opts(precision=FX_PREC_FP64, fp32_threshold=1e-5, schedule=FX_SCHED_BOUND, costmodel=None, alpha=1.0,
              beta=0.0, max_frontier_entries=0, profile=False, use_graph=False, symmetry=FX_SYM_AUTO,
              leaf_screen=FX_LEAF_SHELL, tau_ovlp=0.0, max_workspace_bytes=0):
    return fx_exchange_opts(int(precision), float(fp32_threshold), int(schedule),
                            ctypes.c_void_p(costmodel.handle if costmodel is not None else None),
                            float(alpha), float(beta), int(max_frontier_entries), int(bool(profile)),
                            int(bool(use_graph)), int(symmetry), int(leaf_screen), float(tau_ovlp),
                            int(max_workspace_bytes))


def fx_exchange(tree: Tree, P, tau, K, stream=None):
    n = tree.nbf
    _check_matrix(P, n, "P")
    _check_matrix(K, n, "K")
    _check(lib().fx_exchange(tree.handle, ctypes.c_void_p(P.data_ptr()), float(tau),
                             ctypes.c_void_p(K.data_ptr()), _stream_ptr(stream)))
    return K


def fx_exchange_ex(tree: Tree, P, tau, K, opts=None, stream=None, stats=True):
    """With stats=True the call waits and returns (K, stats); with
    stats=False it only enqueues the work and returns (K, None)."""
    n = tree.nbf
    _check_matrix(P, n, "P")
    _check_matrix(K, n, "K")
    st = fx_stats() if stats else None
    o = opts if opts is not None else make_opts()
    _check(lib().fx_exchange_ex(tree.handle, ctypes.c_void_p(P.data_ptr()), float(tau),
                                ctypes.c_void_p(K.data_ptr()), ctypes.byref(o),
                                ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
    return K, (st.as_dict() if st is not None else None)


def fx_exchange_noalloc(tree: Tree, P, tau, K, opts=None, stream=None, stats=True):
    """fx_exchange_ex working in the library's scratch array (allocates nothing)."""
    n = tree.nbf
    _check_matrix(P, n, "P")
    _check_matrix(K, n, "K")
    st = fx_stats() if stats else None
    o = opts if opts is not None else make_opts()
    _check(lib().fx_exchange_noalloc(tree.handle, ctypes.c_void_p(P.data_ptr()), float(tau),
                                     ctypes.c_void_p(K.data_ptr()), ctypes.byref(o),
                                     ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
    return K, (st.as_dict() if st is not None else None)


def fx_exchange_batched(trees, Ps, Ks, tau, opts=None, stream=None, stats=True):
    count = len(trees)
    for t, P, K in zip(trees, Ps, Ks):
        _check_matrix(P, t.nbf, "P")
        _check_matrix(K, t.nbf, "K")
    VP = ctypes.c_void_p * count
    th = VP(*[t.handle for t in trees])
    ph = VP(*[P.data_ptr() for P in Ps])
    kh = VP(*[K.data_ptr() for K in Ks])
    st = fx_stats() if stats else None
    o = opts if opts is not None else make_opts()
    _check(lib().fx_exchange_batched(th, ph, kh, count, float(tau), ctypes.byref(o),
                                     ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
    return Ks, (st.as_dict() if st is not None else None)


def fx_exchange_multi(tree: Tree, Ps, Ks, tau, opts=None, stream=None):
    """Several densities of one system, contracted with the same integrals."""
    nd = len(Ps)
    if len(Ks) != nd:
        raise ValueError("one K per density")
    for P, K in zip(Ps, Ks):
        _check_matrix(P, tree.nbf, "P")
        _check_matrix(K, tree.nbf, "K")
    VP = ctypes.c_void_p * nd
    ph = VP(*[P.data_ptr() for P in Ps])
    kh = VP(*[K.data_ptr() for K in Ks])
    st = fx_stats()
    o = opts if opts is not None else make_opts()
    _check(lib().fx_exchange_multi(tree.handle, ph, kh, nd, float(tau), ctypes.byref(o), ctypes.byref(st),
                                   _stream_ptr(stream)))
    return Ks, st.as_dict()


def fx_plan_tree(l, nprim, center, exps, coefs, leaf_max_functions=0, ordering=0):
    """Host-only planning: (perm, nodes[level, first shell, end shell, children])."""
    sh = _ShellArrays(l, nprim, center, exps, coefs)
    opts = fx_tree_opts(int(leaf_max_functions), int(ordering))
    S = len(sh.l)
    perm = np.zeros(S, np.int32)
    nlev = ctypes.c_int32()
    nn = ctypes.c_int64()
    _check(lib().fx_plan_tree(ctypes.byref(sh.s), ctypes.byref(opts),
                              perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nlev), None, 0,
                              ctypes.byref(nn)))
    nodes = np.zeros((nn.value, 4), np.int32)
    _check(lib().fx_plan_tree(ctypes.byref(sh.s), ctypes.byref(opts),
                              perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nlev),
                              nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nn.value, ctypes.byref(nn)))
    return perm, nodes


def hilbert_key3(x, y, z, bits):
    return int(lib().fx_hilbert_key3(x, y, z, bits))


def fx_set_class_variant(cls, prec32, variant):
    _check(lib().fx_set_class_variant(int(cls), int(prec32), int(variant)))


def fx_get_class_variant(cls, prec32):
    return int(lib().fx_get_class_variant(int(cls), int(prec32)))


def fx_class_variants_available(cls):
    return int(lib().fx_class_variants_available(int(cls)))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class TaskTimings:
    """(features, log2 ns) samples of K-block work units."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return int(lib().fx_task_timings_count(self._h))

    def arrays(self):
        n = len(self)
        f = np.zeros((n, 4), np.float32)
        t = np.zeros(n, np.float32)
        c = np.zeros(n, np.int32)
        _check(lib().fx_task_timings_get(self._h, _fptr(f), _fptr(t), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return f, t, c

    @staticmethod
    def from_arrays(feats, log2_ns, cls=None):
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, 4)
        t = np.ascontiguousarray(log2_ns, np.float32)
        c = None if cls is None else np.ascontiguousarray(cls, np.int32)
        h = ctypes.c_void_p()
        _check(lib().fx_task_timings_create(_fptr(f), _fptr(t),
                                            None if c is None else c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            len(t), ctypes.byref(h)))
        return TaskTimings(h.value)

    def __del__(self):
        try:
            if self._h:
                lib().fx_task_timings_free(self._h)
                self._h = None
        except Exception:
            pass


class CostModel:
    """Handle of a trained MLP cost model."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def params(self):
        n = int(lib().fx_costmodel_nparams())
        w = np.zeros(n, np.float32)
        norm = np.zeros(10, np.float32)
        _check(lib().fx_costmodel_params(self._h, _fptr(w), _fptr(norm)))
        return w, norm

    @staticmethod
    def create(params, norm):
        w = np.ascontiguousarray(params, np.float32)
        nm = np.ascontiguousarray(norm, np.float32)
        h = ctypes.c_void_p()
        _check(lib().fx_costmodel_create(_fptr(w), _fptr(nm), ctypes.byref(h)))
        return CostModel(h.value)

    def save(self, path):
        _check(lib().fx_costmodel_save(self._h, os.fsencode(path)))

    @staticmethod
    def load(path):
        h = ctypes.c_void_p()
        _check(lib().fx_costmodel_load(os.fsencode(path), ctypes.byref(h)))
        return CostModel(h.value)

    def predict(self, feats, stream=None):
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, 4)
        out = np.zeros(len(f), np.float32)
        _check(lib().fx_costmodel_predict(self._h, _fptr(f), len(f), _fptr(out), _stream_ptr(stream)))
        return out

    def loss_grad(self, feats, log2_ns, stream=None):
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, 4)
        t = np.ascontiguousarray(log2_ns, np.float32)
        g = np.zeros(int(lib().fx_costmodel_nparams()), np.float32)
        loss = np.zeros(1, np.float32)
        _check(lib().fx_costmodel_loss_grad(self._h, _fptr(f), _fptr(t), len(t), _fptr(loss), _fptr(g),
                                            _stream_ptr(stream)))
        return float(loss[0]), g

    def __del__(self):
        try:
            if self._h:
                lib().fx_costmodel_free(self._h)
                self._h = None
        except Exception:
            pass


def fx_record_task_timings(tree, P, tau, opts=None, stream=None) -> TaskTimings:
    _check_matrix(P, tree.nbf, "P")
    o = opts if opts is not None else make_opts()
    h = ctypes.c_void_p()
    _check(lib().fx_record_task_timings(tree.handle, ctypes.c_void_p(P.data_ptr()), float(tau), ctypes.byref(o),
                                        ctypes.byref(h), _stream_ptr(stream)))
    return TaskTimings(h.value)


def fx_costmodel_train(timings, steps=2000, batch=8192, lr=3e-3, seed=12345, stream=None):
    o = fx_train_opts(int(steps), int(batch), float(lr), int(seed))
    h = ctypes.c_void_p()
    loss = ctypes.c_float()
    _check(lib().fx_costmodel_train(timings.handle, ctypes.byref(o), ctypes.byref(h), ctypes.byref(loss),
                                    _stream_ptr(stream)))
    return CostModel(h.value), float(loss.value)


def fx_set_class_launch(cls, prec32, flags):
    _check(lib().fx_set_class_launch(int(cls), int(prec32), int(flags)))


def fx_get_class_launch(cls, prec32):
    return int(lib().fx_get_class_launch(int(cls), int(prec32)))
