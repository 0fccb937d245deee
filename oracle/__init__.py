"""Plain FP64 CPU oracle for the N-body exchange build (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It shares no code with the GPU library: the arithmetic lives
in ``fxo.c`` (McMurchie-Davidson integrals, Boys function by series / erf,
shell-level metric query of Eq. (8)); this module only marshals numpy
arrays through ctypes.  See ``fxo.c`` for the definitions and citations.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        shells = [ctypes.c_int, i32p, i32p, f64p, f64p, f64p]
        L.fxo_boys.argtypes = [ctypes.c_int, ctypes.c_double, f64p]
        L.fxo_norm_coefs.argtypes = shells + [f64p]
        L.fxo_eri_quartet.argtypes = shells + [ctypes.c_int] * 4 + [f64p]
        L.fxo_eri_tensor.argtypes = shells + [f64p]
        L.fxo_schwarz.argtypes = shells + [f64p]
        L.fxo_pnorm.argtypes = [ctypes.c_int, i32p, f64p, f64p]
        L.fxo_exchange.argtypes = shells + [f64p, ctypes.c_double, f64p, f64p]
        L.fxo_exchange_blocks.argtypes = shells + [f64p, ctypes.c_double, f64p, f64p, ctypes.c_int,
                                                   i32p, f64p, f64p]
        L.fxo_bound_matrix.argtypes = [ctypes.c_int, i32p, f64p, f64p, ctypes.c_double, f64p]
        L.fxo_exchange_leafblock.argtypes = shells + [f64p, ctypes.c_double, ctypes.c_int, f64p, f64p]
        L.fxo_overlap.argtypes = shells + [f64p, ctypes.c_void_p]
        L.fxo_exchange_ovlp.argtypes = shells + [f64p, ctypes.c_double, ctypes.c_double, f64p, f64p]
        L.fxo_exchange_sym8.argtypes = shells + [f64p, ctypes.c_double, f64p, f64p]
        L.fxo_count.argtypes = [ctypes.c_int, i32p, i32p, f64p, f64p, ctypes.c_double, f64p,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        for f in ("fxo_norm_coefs", "fxo_eri_quartet", "fxo_eri_tensor", "fxo_schwarz", "fxo_pnorm",
                  "fxo_exchange", "fxo_exchange_blocks", "fxo_bound_matrix", "fxo_count", "fxo_exchange_leafblock",
                  "fxo_overlap", "fxo_exchange_ovlp", "fxo_exchange_sym8"):
            getattr(L, f).restype = ctypes.c_int
        L.fxo_num_threads.restype = ctypes.c_int
        L.fxo_set_threads.argtypes = [ctypes.c_int]
        L.fxo_set_threads.restype = None
        _lib = L
    return _lib


NCART = (1, 3, 6)


def _sh(s):
    return (int(s.l.shape[0]), np.ascontiguousarray(s.l, np.int32), np.ascontiguousarray(s.nprim, np.int32),
            np.ascontiguousarray(s.center, np.float64), np.ascontiguousarray(s.exps, np.float64),
            np.ascontiguousarray(s.coefs, np.float64))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid shells (l must be 0..2, 1..8 primitives)")


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().fxo_boys(mmax, float(T), out)
    return out


def norm_coefs(s) -> np.ndarray:
    """[nshell, 6, 8] normalised contraction weights per Cartesian component."""
    out = np.zeros(s.l.shape[0] * 48)
    _check(lib().fxo_norm_coefs(*_sh(s), out), "norm_coefs")
    return out.reshape(-1, 6, 8)


def eri_quartet(s, a, b, c, d) -> np.ndarray:
    dims = [NCART[s.l[x]] for x in (a, b, c, d)]
    out = np.zeros(int(np.prod(dims)))
    _check(lib().fxo_eri_quartet(*_sh(s), a, b, c, d, out), "eri_quartet")
    return out.reshape(dims)


def eri_tensor(s) -> np.ndarray:
    n = s.nbf
    out = np.zeros(n ** 4)
    _check(lib().fxo_eri_tensor(*_sh(s), out), "eri_tensor")
    return out.reshape(n, n, n, n)


def schwarz(s) -> np.ndarray:
    S = s.l.shape[0]
    out = np.zeros(S * S)
    _check(lib().fxo_schwarz(*_sh(s), out), "schwarz")
    return out.reshape(S, S)


def pnorm(s, P) -> np.ndarray:
    S = s.l.shape[0]
    out = np.zeros(S * S)
    lib().fxo_pnorm(S, np.ascontiguousarray(s.l, np.int32), np.ascontiguousarray(P, np.float64), out)
    return out.reshape(S, S)


def exchange(s, P=None, tau=None):
    """Screened exchange K (factor 1) and stats (computed quartets,
    threshold-sensitive quartets, primitive quartets).  tau < 0: brute force."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    n = s.nbf
    K = np.zeros(n * n)
    st = np.zeros(3)
    _check(lib().fxo_exchange(*_sh(s), np.ascontiguousarray(P, np.float64), float(tau), K, st), "exchange")
    return K.reshape(n, n), {"quartets": int(st[0]), "near_threshold": int(st[1]), "prim_quartets": int(st[2])}


def exchange_leafblock(s, leaf_max=10, P=None, tau=None):
    """K under the paper's leaf rule: shells in the given order bisected into
    leaves of at most leaf_max functions, every quartet of a kept leaf task
    computed.  Returns K and stats (quartets, near-threshold leaf tasks, kept
    leaf tasks, leaves)."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    n = s.nbf
    K = np.zeros(n * n)
    st = np.zeros(4)
    _check(lib().fxo_exchange_leafblock(*_sh(s), np.ascontiguousarray(P, np.float64), float(tau), int(leaf_max), K,
                                        st), "exchange_leafblock")
    return K.reshape(n, n), {"quartets": int(st[0]), "near_threshold": int(st[1]), "leaf_tasks": int(st[2]),
                             "leaves": int(st[3])}


def overlap(s, full=False):
    """Shell-pair largest overlaps Smax [S, S] (and the full overlap matrix)."""
    S = s.l.shape[0]
    sm = np.zeros(S * S)
    Sfull = np.zeros(s.nbf * s.nbf) if full else None
    _check(lib().fxo_overlap(*_sh(s), sm, Sfull.ctypes.data if full else None), "overlap")
    return (sm.reshape(S, S), Sfull.reshape(s.nbf, s.nbf)) if full else sm.reshape(S, S)


def exchange_ovlp(s, tau_ovlp, P=None, tau=None):
    """Exchange with the overlap criterion of Eqs. (3)-(4) as well (exhaustive
    loop: small systems).  stats: quartets, near-threshold tests, quartets
    beta alone keeps."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    n = s.nbf
    K = np.zeros(n * n)
    st = np.zeros(4)
    _check(lib().fxo_exchange_ovlp(*_sh(s), np.ascontiguousarray(P, np.float64), float(tau), float(tau_ovlp), K,
                                   st), "exchange_ovlp")
    return K.reshape(n, n), {"quartets": int(st[0]), "near_threshold": int(st[1]), "beta_quartets": int(st[3])}


def exchange_sym8(s, P=None, tau=None):
    """K through the permutational symmetry of Section IV: each unique shell
    quartet evaluated once and contracted into every ordered quartet it
    stands for that its own bound keeps.  stats: unique quartets evaluated,
    ordered quartets contracted, primitive quartets evaluated, and the
    evaluated quartets by symmetry block: full (eight distinct images, all
    kept), diagonal (coinciding indices, all kept), sparse (an image culled)."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    n = s.nbf
    K = np.zeros(n * n)
    st = np.zeros(6)
    _check(lib().fxo_exchange_sym8(*_sh(s), np.ascontiguousarray(P, np.float64), float(tau), K, st),
           "exchange_sym8")
    return K.reshape(n, n), {"integrals": int(st[0]), "quartets": int(st[1]), "prim_quartets": int(st[2]),
                             "full": int(st[3]), "diagonal": int(st[4]), "sparse": int(st[5])}


def exchange_blocks(s, pairs, P=None, tau=None, Qn=None, Pn=None):
    """K blocks for the requested shell pairs (a, d); returns a list of arrays."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    Qn = schwarz(s) if Qn is None else Qn
    Pn = pnorm(s, P) if Pn is None else Pn
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    sizes = [NCART[s.l[a]] * NCART[s.l[d]] for a, d in pairs]
    out = np.zeros(max(1, sum(sizes)))
    st = np.zeros(2)
    _check(lib().fxo_exchange_blocks(*_sh(s), np.ascontiguousarray(P, np.float64), float(tau),
                                     np.ascontiguousarray(Qn), np.ascontiguousarray(Pn),
                                     len(pairs), pairs, out, st), "exchange_blocks")
    res, o = [], 0
    for (a, d), z in zip(pairs, sizes):
        res.append(out[o:o + z].reshape(NCART[s.l[a]], NCART[s.l[d]]))
        o += z
    return res, {"quartets": int(st[0]), "near_threshold": int(st[1])}


def bound_matrix(s, tau, Qn=None, Pn=None, P=None) -> np.ndarray:
    P = s.P if P is None else P
    Qn = schwarz(s) if Qn is None else Qn
    Pn = pnorm(s, P) if Pn is None else Pn
    n = s.nbf
    E = np.zeros(n * n)
    lib().fxo_bound_matrix(int(s.l.shape[0]), np.ascontiguousarray(s.l, np.int32), np.ascontiguousarray(Qn),
                           np.ascontiguousarray(Pn), float(tau), E)
    return E.reshape(n, n)


def count(s, tau=None, Qn=None, Pn=None, P=None):
    """Exact surviving ordered shell quartets, per class (3x3x3x3 array)."""
    P = s.P if P is None else P
    tau = s.tau if tau is None else tau
    Qn = schwarz(s) if Qn is None else Qn
    Pn = pnorm(s, P) if Pn is None else Pn
    cnt = np.zeros(81)
    pt, nn = ctypes.c_double(0), ctypes.c_double(0)
    lib().fxo_count(int(s.l.shape[0]), np.ascontiguousarray(s.l, np.int32),
                    np.ascontiguousarray(s.nprim, np.int32), np.ascontiguousarray(Qn),
                    np.ascontiguousarray(Pn), float(tau), cnt, ctypes.byref(pt), ctypes.byref(nn))
    return cnt.reshape(3, 3, 3, 3).astype(np.int64), int(pt.value), int(nn.value)


def num_threads() -> int:
    return int(lib().fxo_num_threads())


def set_threads(n: int) -> None:
    lib().fxo_set_threads(int(n))
