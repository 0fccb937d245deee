#!/usr/bin/env python3
"""Code generator for the shell-quartet ERI + exchange-contraction routines.

For every ordered angular-momentum class (la lb|lc ld), la..ld in {s,p,d},
this emits a device routine that evaluates one contracted shell quartet by
the Head-Gordon-Pople scheme the paper's implementation uses (Section V):

  1. per primitive quartet: Boys function F_m(T) (FP64), then the
     Obara-Saika vertical recursion (VRR) building [e0|f0]^(0) from
     [00|00]^(m), first on the bra centre (OS), then transferring angular
     momentum to the ket centre;
  2. the primitive sum of [e0|f0];
  3. the horizontal recursion (HRR) on the contracted quantities,
     (a, b+1_i| = (a+1_i, b| + AB_i (a b|, first on the bra, then the ket;
  4. the exchange contraction of Eq. (6) for this quartet,
     K_{mu sig} += sum_{nu lam} (mu nu|lam sig) P_{nu lam}, accumulated in
     FP64 registers.

Each class is oriented internally so that the VRR/HRR run on the centre of
higher angular momentum of each pair, and with the bra/ket order that gives
fewer floating-point operations; the external (a,b,c,d) roles of the
exchange contraction are mapped back when the contraction is emitted.

The routine is emitted in FP64 and in FP32 (VRR/HRR/primitive sum in FP32,
Boys, pair geometry and all K accumulation in FP64).  The generator also
counts the floating-point operations it emits, per primitive quartet and
per contracted quartet, which the library reports as algorithmic flops.
"""
from __future__ import annotations

import itertools
import math
import re
import os
import sys

LNAME = "spd"


def cart(l):
    """Cartesian exponent triples of shell l, lexicographic (x^l first)."""
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def comp_factor_sq(t):
    """sqrt((2l-1)!! / ((2i-1)!!(2j-1)!!(2k-1)!!)) squared -> ratio as float."""
    def df(n):
        r = 1
        while n > 1:
            r *= n
            n -= 2
        return r
    l = sum(t)
    return df(2 * l - 1) / (df(2 * t[0] - 1) * df(2 * t[1] - 1) * df(2 * t[2] - 1))


def comp_factor(t):
    return comp_factor_sq(t) ** 0.5


def sub(t, i, k=1):
    return tuple(t[j] - (k if j == i else 0) for j in range(3))


def add(t, i, k=1):
    return tuple(t[j] + (k if j == i else 0) for j in range(3))


def argmax_dir(t):
    best = 0
    for i in range(3):
        if t[i] > t[best]:
            best = i
    return best


XYZ = "xyz"


class Emitter:
    """Emits straight-line code for one class; counts flops."""

    def __init__(self, real):
        self.real = real
        self.lines = []
        self.names = {}
        self.flops = 0
        self.counter = 0

    def new(self, prefix):
        self.counter += 1
        return f"{prefix}{self.counter}"

    def emit(self, s):
        self.lines.append(s)


class VRR:
    """Memoised OS/HGP vertical recursion for [e0|f0]^(m)."""

    def __init__(self, em):
        self.em = em
        self.memo = {}

    def get(self, e, f, m):
        if min(e) < 0 or min(f) < 0:
            return None
        key = (e, f, m)
        if key in self.memo:
            return self.memo[key]
        em = self.em
        if sum(e) == 0 and sum(f) == 0:
            name = f"s{m}"        # base, defined by the caller: pref * F_m
            self.memo[key] = name
            return name
        terms = []
        if sum(f) == 0:
            # [e+1_i|0]^(m) = PA_i [e]^(m) + WP_i [e]^(m+1) + e_i/(2p) ([e-1_i]^(m) - rho/p [e-1_i]^(m+1))
            i = argmax_dir(e)
            e1 = sub(e, i)
            k = e1[i]
            a0 = self.get(e1, f, m)
            a1 = self.get(e1, f, m + 1)
            expr = f"PA{XYZ[i]} * {a0} + WP{XYZ[i]} * {a1}"
            fl = 3
            if k > 0:
                b0 = self.get(sub(e1, i), f, m)
                b1 = self.get(sub(e1, i), f, m + 1)
                expr += f" + {k}.0f * (oo2p * {b0} - oo2p_rp * {b1})" if em.real == "float" else \
                    f" + {k}.0 * (oo2p * {b0} - oo2p_rp * {b1})"
                fl += 5
        else:
            # [e|f+1_i]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
            #   + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1)) + e_i/(2(p+q)) [e-1_i|f]^(m+1)
            i = argmax_dir(f)
            f1 = sub(f, i)
            k = f1[i]
            a0 = self.get(e, f1, m)
            a1 = self.get(e, f1, m + 1)
            expr = f"QC{XYZ[i]} * {a0} + WQ{XYZ[i]} * {a1}"
            fl = 3
            suf = ".0f" if em.real == "float" else ".0"
            if k > 0:
                b0 = self.get(e, sub(f1, i), m)
                b1 = self.get(e, sub(f1, i), m + 1)
                expr += f" + {k}{suf} * (oo2q * {b0} - oo2q_rq * {b1})"
                fl += 5
            if e[i] > 0:
                c1 = self.get(sub(e, i), f1, m + 1)
                expr += f" + {e[i]}{suf} * oo2pq * {c1}" if e[i] > 1 else f" + oo2pq * {c1}"
                fl += 2 if e[i] == 1 else 3
        name = em.new("v")
        em.emit(f"const {em.real} {name} = {expr};")
        em.flops += fl
        self.memo[key] = name
        return name


class HRR:
    """Memoised horizontal recursion on contracted [e0|f0] = C[e][f]."""

    def __init__(self, em, cname):
        self.em = em
        self.cname = cname    # function (e, f) -> accumulator expression
        self.memo = {}

    def bra(self, a, b, f):
        key = ("b", a, b, f)
        if key in self.memo:
            return self.memo[key]
        if sum(b) == 0:
            name = self.cname(a, f)
            self.memo[key] = name
            return name
        i = argmax_dir(b)
        b1 = sub(b, i)
        x = self.bra(add(a, i), b1, f)
        y = self.bra(a, b1, f)
        name = self.em.new("h")
        self.em.emit(f"const {self.em.real} {name} = {x} + AB{XYZ[i]}_ * {y};")
        self.em.flops += 2
        self.memo[key] = name
        return name

    def full(self, a, b, c, d):
        key = ("k", a, b, c, d)
        if key in self.memo:
            return self.memo[key]
        if sum(d) == 0:
            name = self.bra(a, b, c)
            self.memo[key] = name
            return name
        i = argmax_dir(d)
        d1 = sub(d, i)
        x = self.full(a, b, add(c, i), d1)
        y = self.full(a, b, c, d1)
        name = self.em.new("k")
        self.em.emit(f"const {self.em.real} {name} = {x} + CD{XYZ[i]}_ * {y};")
        self.em.flops += 2
        self.memo[key] = name
        return name


def orientation(la, lb, lc, ld):
    """Internal order of the four external roles (0=a,1=b,2=c,3=d):
    (x1 x2|x3 x4) with l(x1) >= l(x2), l(x3) >= l(x4).  The bra/ket order is
    chosen by trying both and keeping the one with fewer emitted flops
    (VRR per primitive quartet plus HRR per contracted quartet)."""
    ls = (la, lb, lc, ld)
    bra = (0, 1) if la >= lb else (1, 0)
    ket = (2, 3) if lc >= ld else (3, 2)
    best = None
    for o in (bra + ket, ket + bra):
        L = [ls[x] for x in o]
        body = build_body("double", L)
        hrr = body["hrr"]
        comps = [cart(l) for l in L]
        for t in itertools.product(*comps):
            hrr.full(*t)
        cost = body["vem"].flops + body["hem"].flops
        if best is None or cost < best[0]:
            best = (cost, o)
    return best[1]


def build_body(real, L):
    """VRR (emitted inside the primitive loop) and HRR (after it) for the
    internal angular momenta L = (l1,l2,l3,l4)."""
    l1, l2, l3, l4 = L
    vem = Emitter(real)
    vrr = VRR(vem)
    targets = []
    for le in range(l1, l1 + l2 + 1):
        for e in cart(le):
            for lf in range(l3, l3 + l4 + 1):
                for f in cart(lf):
                    targets.append((e, f))
    tnames = [vrr.get(e, f, 0) for (e, f) in targets]
    idx = {t: k for k, t in enumerate(targets)}
    hem = Emitter(real)
    hrr = HRR(hem, lambda e, f: f"C[{idx[(e, f)]}]")
    return dict(vem=vem, targets=targets, tnames=tnames, hem=hem, hrr=hrr)


def gen_class(la, lb, lc, ld, real, diag=False):
    """Return (code, flops_per_prim, flops_per_contracted) for one class.

    diag=True emits the Schwarz routine for (ab|ab) (la==lc, lb==ld):
    the sum over mu, nu of max(0, (mu nu|mu nu))."""
    ls = (la, lb, lc, ld)
    o = orientation(la, lb, lc, ld) if not diag else ((0, 1, 2, 3) if la >= lb else (1, 0, 3, 2))
    L = [ls[x] for x in o]
    body = build_body(real, L)
    vem, targets, tnames, hem, hrr = body["vem"], body["targets"], body["tnames"], body["hem"], body["hrr"]
    Lsum = sum(L)
    suffix = "f" if real == "float" else ""
    # external component lists
    comps = [cart(l) for l in ls]
    # integral over (mu nu|lam sig) external -> internal component tuple
    def integral(mu, nu, lam, sig):
        ext = (mu, nu, lam, sig)
        t = [None] * 4
        for pos, role in enumerate(o):
            t[pos] = ext[role]
        return hrr.full(t[0], t[1], t[2], t[3])

    out = []
    w = out.append
    cls = f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"
    prec = "f32" if real == "float" else "f64"
    fname = f"eri_{'diag_' if diag else ''}{cls}_{prec}"
    # centres: external a,b,c,d -> X[role]
    w(f"// class ({LNAME[la]}{LNAME[lb]}|{LNAME[lc]}{LNAME[ld]}) {prec}; internal order "
      f"({'abcd'[o[0]]}{'abcd'[o[1]]}|{'abcd'[o[2]]}{'abcd'[o[3]]})")
    if diag:
        w(f"__device__ __forceinline__ double {fname}(const FxShellRef& s0, const FxShellRef& s1,")
        w(f"    const FxDevBasis& B, const double* __restrict__ boys_tab) {{")
        w("  const FxShellRef& ra = s0; const FxShellRef& rb = s1; const FxShellRef& rc = s0; const FxShellRef& rd = s1;")
    else:
        w("template <int NDENS>")
        w(f"__device__ __forceinline__ void {fname}(const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc,")
        w(f"    const FxShellRef& rd, const FxDevBasis& B,")
        w(f"    const double* __restrict__ boys_tab, const double* const* __restrict__ Pq, long ldp, double* __restrict__ kacc) {{")
    roles = ["ra", "rb", "rc", "rd"]
    x = [roles[r] for r in o]
    w(f"  const FxShellRef& x1 = {x[0]}; const FxShellRef& x2 = {x[1]}; const FxShellRef& x3 = {x[2]}; const FxShellRef& x4 = {x[3]};")
    nacc = len(targets)
    w(f"  {real} C[{nacc}];")
    w(f"  #pragma unroll")
    w(f"  for (int k = 0; k < {nacc}; ++k) C[k] = 0;")
    w("  const double ABx = x1.x - x2.x, ABy = x1.y - x2.y, ABz = x1.z - x2.z;")
    w("  const double CDx = x3.x - x4.x, CDy = x3.y - x4.y, CDz = x3.z - x4.z;")
    w("  const long Nt = B.ntprim;")
    w("  const FxPrimPair* __restrict__ pab = B.pp + (long)x1.pofs * Nt + x2.pofs;")
    w("  const FxPrimPair* __restrict__ pcd = B.pp + (long)x3.pofs * Nt + x4.pofs;")
    w("  for (int i1 = 0; i1 < x1.nprim; ++i1) {")
    w("    for (int i2 = 0; i2 < x2.nprim; ++i2) {")
    w("      const FxPrimPair bra = pab[i1 * Nt + i2];")
    w("      const double p = bra.p, op = bra.op, Px = bra.Px, Py = bra.Py, Pz = bra.Pz;")
    w("      for (int i3 = 0; i3 < x3.nprim; ++i3) {")
    w("        for (int i4 = 0; i4 < x4.nprim; ++i4) {")
    w("          const FxPrimPair ket = pcd[i3 * Nt + i4];")
    w("          const double q = ket.p, oq = ket.op, Qx = ket.Px, Qy = ket.Py, Qz = ket.Pz;")
    w("          const double ppq = p + q, oppq = 1.0 / ppq, rho = p * q * oppq;")
    w("          const double PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;")
    w("          const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);")
    w("          const double pref = FX_TWO_PI_POW_2_5 * op * oq * sqrt(oppq) * bra.K * ket.K;")
    w(f"          double F[{Lsum + 1}];")
    w(f"          fx_boys<{Lsum}>(T, boys_tab, F);")
    for m in range(Lsum + 1):
        w(f"          const {real} s{m} = ({real})(pref * F[{m}]);")
    if Lsum > 0:
        w("          const double Wx = (p * Px + q * Qx) * oppq, Wy = (p * Py + q * Qy) * oppq, Wz = (p * Pz + q * Qz) * oppq;")
        for c in "xyz":
            w(f"          const {real} PA{c} = ({real})(P{c} - x1.{c}), WP{c} = ({real})(W{c} - P{c});")
            w(f"          const {real} QC{c} = ({real})(Q{c} - x3.{c}), WQ{c} = ({real})(W{c} - Q{c});")
        w(f"          const {real} oo2p = ({real})(0.5 * op), oo2q = ({real})(0.5 * oq), oo2pq = ({real})(0.5 * oppq);")
        w(f"          const {real} oo2p_rp = ({real})(0.5 * op * rho * op), oo2q_rq = ({real})(0.5 * oq * rho * oq);")
        w("          (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz;")
        w("          (void)QCx; (void)QCy; (void)QCz; (void)WQx; (void)WQy; (void)WQz;")
        w("          (void)oo2p; (void)oo2q; (void)oo2pq; (void)oo2p_rp; (void)oo2q_rq;")
    for line in vem.lines:
        w("          " + line)
    for k, nm in enumerate(tnames):
        w(f"          C[{k}] += {nm};")
    w("        }")
    w("      }")
    w("    }")
    w("  }")
    # HRR + contraction
    w(f"  const {real} ABx_ = ({real})ABx, ABy_ = ({real})ABy, ABz_ = ({real})ABz;")
    w(f"  const {real} CDx_ = ({real})CDx, CDy_ = ({real})CDy, CDz_ = ({real})CDz;")
    w("  (void)ABx_; (void)ABy_; (void)ABz_; (void)CDx_; (void)CDy_; (void)CDz_;")
    if diag:
        # sum_{mu nu} max(0, (mu nu|mu nu)); internal (x1 x2|x1 x2) is the same quartet
        terms = []
        for mu in comps[0]:
            for nu in comps[1]:
                terms.append(integral(mu, nu, mu, nu))
        for line in hem.lines:
            w("  " + line)
        w("  double s2 = 0.0;")
        # the same component-normalisation factors apply: (mu nu|mu nu) scales by (f_mu f_nu)^2
        for (mu, nu), tn in zip(itertools.product(comps[0], comps[1]), terms):
            fac = comp_factor_sq(mu) * comp_factor_sq(nu)
            w(f"  {{ const double v = (double){tn} * {fac!r}; s2 += v > 0.0 ? v : 0.0; }}")
        w("  return s2;")
        w("}")
        return "\n".join(out), vem.flops, hem.flops
    # contraction: kacc[mu*nd + sig] += sum_{nu,lam} I * (f_nu f_lam P_{nu lam})
    nb, nc, nd = len(comps[1]), len(comps[2]), len(comps[3])
    ints = {}
    for im, mu in enumerate(comps[0]):
        for jn, nu in enumerate(comps[1]):
            for kl, lam in enumerate(comps[2]):
                for ls_, sig in enumerate(comps[3]):
                    ints[(im, jn, kl, ls_)] = integral(mu, nu, lam, sig)
    for line in hem.lines:
        w("  " + line)
    cflops = 0
    for jn, nu in enumerate(comps[1]):
        for kl, lam in enumerate(comps[2]):
            fac = comp_factor(nu) * comp_factor(lam)
            pv = f"pv{jn}_{kl}"
            scale = "" if abs(fac - 1.0) < 1e-15 else f" * {fac!r}"
            w(f"  double {pv}[NDENS];")
            w(f"  FX_FOR_DENS {pv}[_d] = Pq[_d][{jn} * ldp + {kl}]{scale};")
            cflops += 1 if scale else 0
            nkb = len(comps[0]) * nd
            for im in range(len(comps[0])):
                for ls_ in range(nd):
                    w(f"  {{ const double _v = (double){ints[(im, jn, kl, ls_)]}; "
                      f"FX_FOR_DENS kacc[_d * {nkb} + {im * nd + ls_}] += _v * {pv}[_d]; }}")
                    cflops += 2
    w("}")
    return "\n".join(out), vem.flops, hem.flops + cflops


def _emit_prim_setup(w, real, Lsum, j, ind, wexpr=None):
    """Set-up of primitive quartet j (names suffixed _j: pair data, Boys
    F_m scaled by the prefactor, VRR geometry); `wexpr` scales its prefactor
    (0 for a padding quartet).  Expects i1_j..i4_j, pab, pcd, Nt, x1, x3."""
    sfx = f"_{j}"
    w(f"{ind}const FxPrimPair bra{sfx} = pab[i1{sfx} * Nt + i2{sfx}];")
    w(f"{ind}const double p{sfx} = bra{sfx}.p, op{sfx} = bra{sfx}.op, Px{sfx} = bra{sfx}.Px, Py{sfx} = bra{sfx}.Py, "
      f"Pz{sfx} = bra{sfx}.Pz;")
    w(f"{ind}const FxPrimPair ket{sfx} = pcd[i3{sfx} * Nt + i4{sfx}];")
    w(f"{ind}const double q{sfx} = ket{sfx}.p, oq{sfx} = ket{sfx}.op, Qx{sfx} = ket{sfx}.Px, Qy{sfx} = ket{sfx}.Py, "
      f"Qz{sfx} = ket{sfx}.Pz;")
    w(f"{ind}const double ppq{sfx} = p{sfx} + q{sfx}, oppq{sfx} = 1.0 / ppq{sfx}, rho{sfx} = p{sfx} * q{sfx} * oppq{sfx};")
    w(f"{ind}const double PQx{sfx} = Px{sfx} - Qx{sfx}, PQy{sfx} = Py{sfx} - Qy{sfx}, PQz{sfx} = Pz{sfx} - Qz{sfx};")
    w(f"{ind}const double T{sfx} = rho{sfx} * (PQx{sfx} * PQx{sfx} + PQy{sfx} * PQy{sfx} + PQz{sfx} * PQz{sfx});")
    scale = f" * {wexpr}" if wexpr else ""
    w(f"{ind}const double pref{sfx} = FX_TWO_PI_POW_2_5 * op{sfx} * oq{sfx} * sqrt(oppq{sfx}) * bra{sfx}.K * "
      f"ket{sfx}.K{scale};")
    w(f"{ind}double F{sfx}[{Lsum + 1}];")
    w(f"{ind}fx_boys<{Lsum}>(T{sfx}, boys_tab, F{sfx});")
    for m in range(Lsum + 1):
        w(f"{ind}const {real} s{m}{sfx} = ({real})(pref{sfx} * F{sfx}[{m}]);")
    if Lsum == 0:
        return
    w(f"{ind}const double Wx{sfx} = (p{sfx} * Px{sfx} + q{sfx} * Qx{sfx}) * oppq{sfx}, "
      f"Wy{sfx} = (p{sfx} * Py{sfx} + q{sfx} * Qy{sfx}) * oppq{sfx}, Wz{sfx} = (p{sfx} * Pz{sfx} + q{sfx} * Qz{sfx}) * oppq{sfx};")
    for c in "xyz":
        w(f"{ind}const {real} PA{c}{sfx} = ({real})(P{c}{sfx} - x1.{c}), WP{c}{sfx} = ({real})(W{c}{sfx} - P{c}{sfx});")
        w(f"{ind}const {real} QC{c}{sfx} = ({real})(Q{c}{sfx} - x3.{c}), WQ{c}{sfx} = ({real})(W{c}{sfx} - Q{c}{sfx});")
    w(f"{ind}const {real} oo2p{sfx} = ({real})(0.5 * op{sfx}), oo2q{sfx} = ({real})(0.5 * oq{sfx}), "
      f"oo2pq{sfx} = ({real})(0.5 * oppq{sfx});")
    w(f"{ind}const {real} oo2p_rp{sfx} = ({real})(0.5 * op{sfx} * rho{sfx} * op{sfx}), "
      f"oo2q_rq{sfx} = ({real})(0.5 * oq{sfx} * rho{sfx} * oq{sfx});")
    for nm in ("PAx", "PAy", "PAz", "WPx", "WPy", "WPz", "QCx", "QCy", "QCz", "WQx", "WQy", "WQz", "oo2p", "oo2q",
               "oo2pq", "oo2p_rp", "oo2q_rq"):
        w(f"{ind}(void){nm}{sfx};")


_VRR_TOKEN = re.compile(r"\b(v\d+|s\d+|PA[xyz]|WP[xyz]|QC[xyz]|WQ[xyz]|oo2p|oo2q|oo2pq|oo2p_rp|oo2q_rq)\b")


def _emit_vrr(w, vem, tpos0, nj, ind, put_fmt):
    """The VRR of nj primitive quartets, interleaved node by node; each
    target is handed to put_fmt(k, "v_0 + v_1 ...") as soon as all nj
    copies of it are formed."""
    tpos = dict(tpos0)

    def put(nm):
        k = tpos.pop(nm)
        w(ind + put_fmt(k, " + ".join(f"{nm}_{j}" for j in range(nj))))
    for line in vem.lines:
        for j in range(nj):
            w(ind + _VRR_TOKEN.sub(lambda m: m.group(1) + f"_{j}", line))
        nm = line.split(" = ", 1)[0].split()[-1]
        if nm in tpos:
            put(nm)
    for nm in list(tpos):          # targets that are base values s_m
        put(nm)


def _emit_fold(w, real, o, comps, icomp, fcols, idx, preamble=True, ucount=None):
    """Steps 2+3 of the folded staged routine: per ket column f, the bra HRR
    of X[., f] into registers, then every (x3 x4) component whose closed-form
    ket HRR uses column f adds (x1 x2|f) * coef * P into kacc."""
    fl = 0
    nd = len(comps[3])
    index = [{t: k for k, t in enumerate(comps[r])} for r in range(4)]
    nkb = len(comps[0]) * nd
    for jn, nu in (enumerate(comps[1]) if preamble else []):
        for kl, lam in enumerate(comps[2]):
            fac = comp_factor(nu) * comp_factor(lam)
            scale = "" if abs(fac - 1.0) < 1e-15 else f" * {fac!r}"
            w(f"  double pv{jn}_{kl}[NDENS];")
            w(f"  FX_FOR_DENS pv{jn}_{kl}[_d] = Pq[_d][{jn} * ldp + {kl}]{scale};")
            fl += 1 if scale else 0
    if preamble:
        w("  const double CDx2 = CDx * CDx, CDy2 = CDy * CDy, CDz2 = CDz * CDz;")
        w("  (void)CDx2; (void)CDy2; (void)CDz2;")
    powname = {1: "CD{}", 2: "CD{}2"}
    for f in fcols:
        hem = Emitter(real)
        loads = {}

        def xval(e, f_, hem=hem, loads=loads):
            k = idx[(e, f_)]
            if k not in loads:
                nm = hem.new("x")
                hem.emit(f"const {real} {nm} = X[{k}];")
                loads[k] = nm
            return loads[k]
        hrr = HRR(hem, xval)
        yf = {}
        for t1 in icomp[0]:
            for t2 in icomp[1]:
                yf[(t1, t2)] = hrr.bra(t1, t2, f)
        w("  {")
        for line in hem.lines:
            w("    " + line)
        fl += hem.flops
        nu_ = ucount[0] if ucount else 0
        for t3 in icomp[2]:
            for t4 in icomp[3]:
                k = tuple(f[i] - t3[i] for i in range(3))
                if any(k[i] < 0 or k[i] > t4[i] for i in range(3)):
                    continue
                fac = 1
                parts = []
                for i in range(3):
                    fac *= math.comb(t4[i], k[i])
                    pw = t4[i] - k[i]
                    if pw:
                        parts.append(powname[pw].format(XYZ[i]))
                coef = " * ".join(([f"{fac}.0"] if fac != 1 else []) + parts)
                # one FP64 factor coef * P per distinct density element
                us = {}
                for t1 in icomp[0]:
                    for t2 in icomp[1]:
                        ext = [None] * 4
                        for pos, role in enumerate(o):
                            ext[role] = (t1, t2, t3, t4)[pos]
                        im, jn, kl, ls_ = (index[r][ext[r]] for r in range(4))
                        key = (jn, kl)
                        if key not in us:
                            if coef:
                                nu_ += 1
                                us[key] = f"u{nu_}"
                                w(f"    double u{nu_}[NDENS];")
                                w(f"    FX_FOR_DENS u{nu_}[_d] = {coef} * pv{jn}_{kl}[_d];")
                                fl += 1 + len(parts) + (fac != 1)
                            else:
                                us[key] = f"pv{jn}_{kl}"
                        w(f"    {{ const double _v = (double){yf[(t1, t2)]}; "
                          f"FX_FOR_DENS kacc[_d * {nkb} + {im * nd + ls_}] += _v * {us[key]}[_d]; }}")
                        fl += 2
        w("  }")
        if ucount:
            ucount[0] = nu_
    return fl


def gen_class_staged(la, lb, lc, ld, real, paired=False, fold=False):
    """Staged form of the same routine, for classes whose [e0|f0] block does
    not fit in registers.  Same arithmetic, different data movement: the
    accumulated [e0|f0] block X and the bra-transferred block Y = (x1 x2|f)
    live in per-lane private memory (lane-interleaved, so each access of a
    wave is one coalesced transaction), each written once per primitive
    quartet and read once:

      1. per primitive quartet: Boys, VRR; every target [e0|f0] is added
         into X as soon as it is formed (with `paired`, two primitive
         quartets are evaluated side by side and X is updated once per
         pair);
      2. bra HRR one ket column f at a time: read X[., f], write Y[., f];
      3. ket HRR one bra row at a time: read Y[row, .], form the row's
         integrals and contract each into kacc at once.

    With `fold`, steps 2 and 3 become one pass over the ket columns and Y is
    not formed: the ket HRR has the closed form
      (x3, x4| = sum_{k <= x4} prod_i C(x4_i, k_i) CD_i^(x4_i - k_i) (x3 + k, 0|,
    so column f = x3 + k of the bra-transferred block contributes
    (x1 x2|f) * coef * P to the K block directly, in FP64.

    Returns (code, flops_per_prim, flops_per_contracted) like gen_class."""
    ls = (la, lb, lc, ld)
    o = orientation(la, lb, lc, ld)
    L = [ls[x] for x in o]
    body = build_body(real, L)
    vem, targets, tnames = body["vem"], body["targets"], body["tnames"]
    Lsum = sum(L)
    comps = [cart(l) for l in ls]
    icomp = [cart(l) for l in L]
    fcols = [f for lf in range(L[2], L[2] + L[3] + 1) for f in cart(lf)]
    fidx = {f: k for k, f in enumerate(fcols)}
    nrow = len(icomp[0]) * len(icomp[1])
    NX, NY = len(targets), nrow * len(fcols)
    out = []
    w = out.append
    cls = f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"
    prec = "f32" if real == "float" else "f64"
    w(f"// class ({LNAME[la]}{LNAME[lb]}|{LNAME[lc]}{LNAME[ld]}) {prec}, staged; internal order "
      f"({'abcd'[o[0]]}{'abcd'[o[1]]}|{'abcd'[o[2]]}{'abcd'[o[3]]}); X {NX}, Y {NY} private slots")
    w("template <int NDENS>")
    w(f"__device__ __forceinline__ void eri_{cls}_{prec}(const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc,")
    w(f"    const FxShellRef& rd, const FxDevBasis& B,")
    w(f"    const double* __restrict__ boys_tab, const double* const* __restrict__ Pq, long ldp, double* __restrict__ kacc) {{")
    roles = ["ra", "rb", "rc", "rd"]
    x = [roles[r] for r in o]
    w(f"  const FxShellRef& x1 = {x[0]}; const FxShellRef& x2 = {x[1]}; const FxShellRef& x3 = {x[2]}; const FxShellRef& x4 = {x[3]};")
    # The asm statement hides the arrays' addresses from the optimiser, so
    # they stay in private memory instead of being promoted to registers.
    if fold:
        w(f"  {real} Xs[{NX}];")
        w(f"  __attribute__((address_space(5))) {real}* X = (__attribute__((address_space(5))) {real}*)Xs;")
        w("  asm volatile(\"\" : \"+v\"(X));")
    else:
        w(f"  {real} Xs[{NX}], Ys[{NY}];")
        w(f"  __attribute__((address_space(5))) {real}* X = (__attribute__((address_space(5))) {real}*)Xs;")
        w(f"  __attribute__((address_space(5))) {real}* Y = (__attribute__((address_space(5))) {real}*)Ys;")
        w("  asm volatile(\"\" : \"+v\"(X), \"+v\"(Y));")
    w("  const double ABx = x1.x - x2.x, ABy = x1.y - x2.y, ABz = x1.z - x2.z;")
    w("  const double CDx = x3.x - x4.x, CDy = x3.y - x4.y, CDz = x3.z - x4.z;")
    w("  const long Nt = B.ntprim;")
    w("  const FxPrimPair* __restrict__ pab = B.pp + (long)x1.pofs * Nt + x2.pofs;")
    w("  const FxPrimPair* __restrict__ pcd = B.pp + (long)x3.pofs * Nt + x4.pofs;")
    tpos0 = {nm: k for k, nm in enumerate(tnames)}

    def setup(j, ind, wexpr=None):
        _emit_prim_setup(w, real, Lsum, j, ind, wexpr)

    def vrr_lines(nj, ind):
        _emit_vrr(w, vem, tpos0, nj, ind,
                  lambda k, sm: f"if constexpr (ACC) X[{k}] += {sm}; else X[{k}] = {sm};")

    if paired:
        # two primitive quartets per pass (the second of an odd count is a
        # zero-weight copy of the last): one X update per target and pass
        w("  const int n4 = x4.nprim, n34 = x3.nprim * n4, n234 = x2.nprim * n34;")
        w("  const int nq = x1.nprim * n234;")
        w("  auto prim2 = [&](int qa, int qb, double wb, auto acc) {")
        w("    constexpr bool ACC = decltype(acc)::value;")
        for j, qv in ((0, "qa"), (1, "qb")):
            w(f"    const int i1_{j} = {qv} / n234, i2_{j} = ({qv} / n34) % x2.nprim, i3_{j} = ({qv} / n4) % x3.nprim, "
              f"i4_{j} = {qv} % n4;")
        setup(0, "    ")
        setup(1, "    ", "wb")
        vrr_lines(2, "    ")
        w("  };")
        w("  prim2(0, nq > 1 ? 1 : 0, nq > 1 ? 1.0 : 0.0, FxAcc<false>{});")
        w("  for (int q = 2; q < nq; q += 2)")
        w("    prim2(q, q + 1 < nq ? q + 1 : q, q + 1 < nq ? 1.0 : 0.0, FxAcc<true>{});")
    else:
        # the primitive-quartet body, instantiated twice: the first primitive
        # quartet stores into X, the others add to it
        w("  auto prim = [&](int i1_0, int i2_0, int i3_0, int i4_0, auto acc) {")
        w("    constexpr bool ACC = decltype(acc)::value;")
        setup(0, "    ")
        vrr_lines(1, "    ")
        w("  };")
        w("  prim(0, 0, 0, 0, FxAcc<false>{});")
        w("  for (int i1 = 0; i1 < x1.nprim; ++i1)")
        w("    for (int i2 = 0; i2 < x2.nprim; ++i2)")
        w("      for (int i3 = 0; i3 < x3.nprim; ++i3)")
        w("        for (int i4 = 0; i4 < x4.nprim; ++i4)")
        w("          if (i1 | i2 | i3 | i4) prim(i1, i2, i3, i4, FxAcc<true>{});")
    w(f"  const {real} ABx_ = ({real})ABx, ABy_ = ({real})ABy, ABz_ = ({real})ABz;")
    w(f"  const {real} CDx_ = ({real})CDx, CDy_ = ({real})CDy, CDz_ = ({real})CDz;")
    w("  (void)ABx_; (void)ABy_; (void)ABz_; (void)CDx_; (void)CDy_; (void)CDz_;")
    idx = {t: k for k, t in enumerate(targets)}
    hflops = 0
    if fold:
        hflops += _emit_fold(w, real, o, comps, icomp, fcols, idx)
        w("}")
        return "\n".join(out), vem.flops, hflops
    # 2. bra HRR per ket column
    for f in fcols:
        hem = Emitter(real)
        loads = {}

        def xval(e, f_, hem=hem, loads=loads):
            k = idx[(e, f_)]
            if k not in loads:
                nm = hem.new("x")
                hem.emit(f"const {real} {nm} = X[{k}];")
                loads[k] = nm
            return loads[k]
        hrr = HRR(hem, xval)
        res = []
        for ia, a in enumerate(icomp[0]):
            for ib, b in enumerate(icomp[1]):
                res.append(((ia * len(icomp[1]) + ib) * len(fcols) + fidx[f], hrr.bra(a, b, f)))
        w("  {")
        for line in hem.lines:
            w("    " + line)
        for k, nm in res:
            w(f"    Y[{k}] = {nm};")
        w("  }")
        hflops += hem.flops
    # 3. ket HRR per bra row, contraction
    nd = len(comps[3])
    index = [{t: k for k, t in enumerate(comps[r])} for r in range(4)]
    pvs = {}
    for jn, nu in enumerate(comps[1]):
        for kl, lam in enumerate(comps[2]):
            fac = comp_factor(nu) * comp_factor(lam)
            pv = f"pv{jn}_{kl}"
            pvs[(jn, kl)] = pv
            scale = "" if abs(fac - 1.0) < 1e-15 else f" * {fac!r}"
            w(f"  double {pv}[NDENS];")
            w(f"  FX_FOR_DENS {pv}[_d] = Pq[_d][{jn} * ldp + {kl}]{scale};")
            hflops += 1 if scale else 0
    for ia, a in enumerate(icomp[0]):
        for ib, b in enumerate(icomp[1]):
            hem = Emitter(real)
            row = (ia * len(icomp[1]) + ib) * len(fcols)
            loads = {}

            def yval(a_, f_, hem=hem, loads=loads, row=row):
                k = row + fidx[f_]
                if k not in loads:
                    nm = hem.new("y")
                    hem.emit(f"const {real} {nm} = Y[{k}];")
                    loads[k] = nm
                return loads[k]
            hrr = HRR(hem, None)
            # bra(a, b, f) of this row is the staged Y value
            for f in fcols:
                hrr.memo[("b", a, b, f)] = None
            hrr.bra = lambda a_, b_, f_, yv=yval: yv(a_, f_)
            w("  {")
            contr = []
            for c in icomp[2]:
                for d in icomp[3]:
                    nm = hrr.full(a, b, c, d)
                    ext = [None] * 4
                    for pos, role in enumerate(o):
                        ext[role] = (a, b, c, d)[pos]
                    im, jn, kl, ls_ = (index[r][ext[r]] for r in range(4))
                    contr.append((im * nd + ls_, nm, pvs[(jn, kl)]))
            for line in hem.lines:
                w("    " + line)
            nkb = len(comps[0]) * nd
            for slot, nm, pv in contr:
                w(f"    {{ const double _v = (double){nm}; FX_FOR_DENS kacc[_d * {nkb} + {slot}] += _v * {pv}[_d]; }}")
                hflops += 2
            w("  }")
            hflops += hem.flops
    w("}")
    return "\n".join(out), vem.flops, hflops


def gen_class_chunked(la, lb, lc, ld, real, nchunks, paired=True, xreg=False):
    """Folded staged routine with the ket columns in nchunks chunks: for each
    chunk the primitive loop rebuilds only that chunk's [e0|f0] columns (the
    VRR of the other columns' ancestors is recomputed), then folds them into
    kacc.  The live [e0|f0] slice is 1/nchunks of the block."""
    ls = (la, lb, lc, ld)
    o = orientation(la, lb, lc, ld)
    L = [ls[x] for x in o]
    l1, l2, l3, l4 = L
    Lsum = sum(L)
    comps = [cart(l) for l in ls]
    icomp = [cart(l) for l in L]
    fcols = [f for lf in range(L[2], L[2] + L[3] + 1) for f in cart(lf)]
    erows = [e for le in range(l1, l1 + l2 + 1) for e in cart(le)]
    chunks = [fcols[c * len(fcols) // nchunks:(c + 1) * len(fcols) // nchunks] for c in range(nchunks)]
    NX = max(len(erows) * len(ch) for ch in chunks)
    out = []
    w = out.append
    cls = f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"
    prec = "f32" if real == "float" else "f64"
    w(f"// class ({cls}) {prec}, staged in {nchunks} ket-column chunks; X {NX}")
    w("template <int NDENS>")
    w(f"__device__ __forceinline__ void eri_{cls}_{prec}(const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc,")
    w(f"    const FxShellRef& rd, const FxDevBasis& B,")
    w(f"    const double* __restrict__ boys_tab, const double* const* __restrict__ Pq, long ldp, double* __restrict__ kacc) {{")
    roles = ["ra", "rb", "rc", "rd"]
    x = [roles[r] for r in o]
    w(f"  const FxShellRef& x1 = {x[0]}; const FxShellRef& x2 = {x[1]}; const FxShellRef& x3 = {x[2]}; const FxShellRef& x4 = {x[3]};")
    if xreg:
        w(f"  {real} X[{NX}];")
    else:
        w(f"  {real} Xs[{NX}];")
        w(f"  __attribute__((address_space(5))) {real}* X = (__attribute__((address_space(5))) {real}*)Xs;")
        w("  asm volatile(\"\" : \"+v\"(X));")
    w("  const double ABx = x1.x - x2.x, ABy = x1.y - x2.y, ABz = x1.z - x2.z;")
    w("  const double CDx = x3.x - x4.x, CDy = x3.y - x4.y, CDz = x3.z - x4.z;")
    w("  const long Nt = B.ntprim;")
    w("  const FxPrimPair* __restrict__ pab = B.pp + (long)x1.pofs * Nt + x2.pofs;")
    w("  const FxPrimPair* __restrict__ pcd = B.pp + (long)x3.pofs * Nt + x4.pofs;")
    w(f"  const {real} ABx_ = ({real})ABx, ABy_ = ({real})ABy, ABz_ = ({real})ABz;")
    w(f"  const {real} CDx_ = ({real})CDx, CDy_ = ({real})CDy, CDz_ = ({real})CDz;")
    w("  (void)ABx_; (void)ABy_; (void)ABz_; (void)CDx_; (void)CDy_; (void)CDz_;")
    # P factors and CD powers once
    for jn, nu in enumerate(comps[1]):
        for kl, lam in enumerate(comps[2]):
            fac = comp_factor(nu) * comp_factor(lam)
            scale = "" if abs(fac - 1.0) < 1e-15 else f" * {fac!r}"
            w(f"  double pv{jn}_{kl}[NDENS];")
            w(f"  FX_FOR_DENS pv{jn}_{kl}[_d] = Pq[_d][{jn} * ldp + {kl}]{scale};")
    w("  const double CDx2 = CDx * CDx, CDy2 = CDy * CDy, CDz2 = CDz * CDz;")
    w("  (void)CDx2; (void)CDy2; (void)CDz2;")
    ucount = [0]
    vfl = 0
    for ci, ch in enumerate(chunks):
        vem = Emitter(real)
        vrr = VRR(vem)
        targets = [(e, f) for e in erows for f in ch]
        tnames = [vrr.get(e, f, 0) for (e, f) in targets]
        vfl += vem.flops
        tpos0 = {nm: k for k, nm in enumerate(tnames)}
        idx = {t: k for k, t in enumerate(targets)}
        w(f"  {{  // ket columns {ci}")

        def setup(j, ind, wexpr=None):
            _emit_prim_setup(w, real, Lsum, j, ind, wexpr)

        def vrr_lines(nj, ind, vem=vem, tpos0=tpos0):
            _emit_vrr(w, vem, tpos0, nj, ind,
                      lambda k, sm: f"if constexpr (ACC) X[{k}] += {sm}; else X[{k}] = {sm};")
        if paired:
            w("  const int n4 = x4.nprim, n34 = x3.nprim * n4, n234 = x2.nprim * n34;")
            w("  const int nq = x1.nprim * n234;")
            w("  auto prim2 = [&](int qa, int qb, double wb, auto acc) {")
            w("    constexpr bool ACC = decltype(acc)::value;")
            for j, qv in ((0, "qa"), (1, "qb")):
                w(f"    const int i1_{j} = {qv} / n234, i2_{j} = ({qv} / n34) % x2.nprim, i3_{j} = ({qv} / n4) % x3.nprim, "
                  f"i4_{j} = {qv} % n4;")
            setup(0, "    ")
            setup(1, "    ", "wb")
            vrr_lines(2, "    ")
            w("  };")
            w("  prim2(0, nq > 1 ? 1 : 0, nq > 1 ? 1.0 : 0.0, FxAcc<false>{});")
            w("  for (int q = 2; q < nq; q += 2)")
            w("    prim2(q, q + 1 < nq ? q + 1 : q, q + 1 < nq ? 1.0 : 0.0, FxAcc<true>{});")
        else:
            w("  auto prim = [&](int i1_0, int i2_0, int i3_0, int i4_0, auto acc) {")
            w("    constexpr bool ACC = decltype(acc)::value;")
            setup(0, "    ")
            vrr_lines(1, "    ")
            w("  };")
            w("  prim(0, 0, 0, 0, FxAcc<false>{});")
            w("  for (int i1 = 0; i1 < x1.nprim; ++i1)")
            w("    for (int i2 = 0; i2 < x2.nprim; ++i2)")
            w("      for (int i3 = 0; i3 < x3.nprim; ++i3)")
            w("        for (int i4 = 0; i4 < x4.nprim; ++i4)")
            w("          if (i1 | i2 | i3 | i4) prim(i1, i2, i3, i4, FxAcc<true>{});")
        _emit_fold(w, real, o, comps, icomp, ch, idx, preamble=False, ucount=ucount)
        w("  }")
    w("}")
    return "\n".join(out), vfl


def classes():
    return list(itertools.product(range(3), repeat=4))


def pair_size(l1, l2):
    """Number of accumulated [e0| components of a pair (higher l first)."""
    hi, lo = max(l1, l2), min(l1, l2)
    return sum(len(cart(x)) for x in range(hi, hi + lo + 1))


# Variants generated per class, by the size of the accumulated [e0|f0] block:
# one thread per quartet while it fits in registers, the cooperative
# one-quartet-per-wave form beyond; in between both exist and the autotuner
# (or the default table) chooses.
COOP_MIN, THREAD_MAX = 100, 1 << 30


# Per-kernel generator choices, read from the "generator" section of the
# tuning table (tuning_gfx950.json, written by the autotuner from per-kernel
# timings): for each (class, precision) the form of the one-quartet-per-lane
# routine -- "register" (gen_class), "staged" or "folded" (gen_class_staged
# without / with the folded ket HRR), "chunked" (gen_class_chunked, with
# "chunks" and "xreg") --, whether staged forms evaluate two primitive
# quartets per pass ("paired"), the waves per SIMD that the register
# allocation must allow ("waves"), and the entry groups per fill step of the
# candidate scan ("groups", default 3); a "<class>:mix" entry builds the class's
# mixed-precision kernel that screens each candidate once and runs both
# precisions in one pass, with its own "waves".  Without a table every
# kernel is the register form at one wave, in two passes.
TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tuning_gfx950.json")

STAGED, FOLD, UNPAIRED, DUAL = set(), set(), set(), set()
MIN_WAVES, CHUNKS, GROUPS = {}, {}, {}
XREG = set()


def load_choices(path=TABLE):
    """Fill the choice sets from a tuning table (empty sets without one)."""
    global STAGED, FOLD, UNPAIRED, DUAL, MIN_WAVES, CHUNKS, XREG, GROUPS
    STAGED, FOLD, UNPAIRED, DUAL = set(), set(), set(), set()
    MIN_WAVES, CHUNKS, XREG, GROUPS = {}, {}, set(), {}
    if not os.path.exists(path):
        return
    import json
    kernels = json.load(open(path)).get("generator", {}).get("kernels", {})
    for key, e in kernels.items():
        cls, prec = key.split(":")
        if e.get("waves", 1) > 1:
            MIN_WAVES[(cls, prec)] = int(e["waves"])
        if e.get("groups", 3) != 3:
            GROUPS[(cls, prec)] = int(e["groups"])
        if prec == "mix":
            DUAL.add(cls)
            continue
        form = e.get("form", "register")
        if form in ("staged", "folded"):
            STAGED.add((cls, prec))
            if form == "folded":
                FOLD.add((cls, prec))
        elif form == "chunked":
            CHUNKS[(cls, prec)] = int(e["chunks"])
            if e.get("xreg"):
                XREG.add((cls, prec))
        if form != "register" and not e.get("paired", True):
            UNPAIRED.add((cls, prec))


load_choices()


def variants(la, lb, lc, ld):
    nacc = pair_size(la, lb) * pair_size(lc, ld)
    return (nacc < THREAD_MAX, nacc >= COOP_MIN)


def main(outdir):
    import gen_coop
    os.makedirs(outdir, exist_ok=True)
    stats = []
    for (la, lb, lc, ld) in classes():
        cls = f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"
        th, co = variants(la, lb, lc, ld)
        parts = []
        for real in ("double", "float"):
            code, fp, fc = gen_class(la, lb, lc, ld, real)
            prec = "f32" if real == "float" else "f64"
            if (cls, prec) in CHUNKS:
                code = gen_class_chunked(la, lb, lc, ld, real, CHUNKS[(cls, prec)], paired=(cls, prec) not in UNPAIRED,
                                         xreg=(cls, prec) in XREG)[0]
            elif (cls, prec) in STAGED:
                code = gen_class_staged(la, lb, lc, ld, real, paired=(cls, prec) not in UNPAIRED,
                                        fold=(cls, prec) in FOLD)[0]
            if th:
                parts.append(code)
            if real == "double":
                stats.append((cls, fp, fc))
            if co:
                parts.append(gen_coop.gen_coop(la, lb, lc, ld, real)[0])
        src = ["// Generated by gen_eri.py -- do not edit.", '#include "fx_eri_common.h"', ""]
        src += parts
        kind = "BOTH" if (th and co) else ("THREAD" if th else "COOP")
        for prec in ("f64", "f32", "mix"):
            mw = MIN_WAVES.get((cls, prec), 1)
            if mw > 1:
                src.append(f"#undef FX_THREAD_MIN_WAVES_{prec}")
                src.append(f"#define FX_THREAD_MIN_WAVES_{prec} {mw}")
            g = GROUPS.get((cls, prec), 3)
            if g != 3:
                src.append(f"#undef FX_FILL_GROUPS_{prec}")
                src.append(f"#define FX_FILL_GROUPS_{prec} {g}")
        src.append(f'FX_DEFINE_CLASS_KERNELS_{kind}({la}, {lb}, {lc}, {ld}, {cls})')
        path = os.path.join(outdir, f"eri_{cls}.hip")
        new = "\n".join(src) + "\n"
        if not os.path.exists(path) or open(path).read() != new:
            open(path, "w").write(new)
    # Schwarz (diagonal) routines: (ab|ab) for the 9 ordered pair types
    src = ["// Generated by gen_eri.py -- do not edit.", '#include "fx_eri_common.h"', ""]
    for la in range(3):
        for lb in range(3):
            code, _, _ = gen_class(la, lb, la, lb, "double", diag=True)
            src.append(code)
    src.append("FX_DEFINE_SCHWARZ_KERNEL()")
    path = os.path.join(outdir, "eri_schwarz.hip")
    new = "\n".join(src) + "\n"
    if not os.path.exists(path) or open(path).read() != new:
        open(path, "w").write(new)
    # dispatch table
    names = [f"{LNAME[a]}{LNAME[b]}{LNAME[c]}{LNAME[d]}" for (a, b, c, d) in classes()]
    lines = ["// Generated by gen_eri.py -- do not edit.", "#pragma once", '#include "fx_internal.h"']
    lines += [f"FX_DECLARE_LAUNCH({n})" for n in names]
    lines.append("// indexed by ((la*3+lb)*3+lc)*3+ld")
    lines.append("static const fx_class_launcher fx_class_table[81] = {" + ", ".join(f"fx_launch_{n}" for n in names) + "};")
    # available variants (bit 0 thread, bit 1 cooperative) and the default choice
    av = []
    for (a, b, c, d) in classes():
        th, co = variants(a, b, c, d)
        av.append(str((1 if th else 0) | (2 if co else 0) | (4 if th else 0)))
    lines.append("// bit 0: one quartet per lane, bit 1: one quartet per wave, bit 2: both precisions in one pass")
    lines.append("static const int fx_class_variants[81] = {" + ", ".join(av) + "};")
    dv = ["1" if "".join(LNAME[x] for x in t) in DUAL else "0" for t in classes()]
    lines.append("// default: mixed precision in one pass (variant 2 for the FP64 half)")
    lines.append("static const int fx_class_dual_default[81] = {" + ", ".join(dv) + "};")
    path = os.path.join(outdir, "eri_table.h")
    new = "\n".join(lines) + "\n"
    if not os.path.exists(path) or open(path).read() != new:
        open(path, "w").write(new)
    # flop table (FP64 emission; FP32 emits the same operations)
    lines = ["// Generated by gen_eri.py -- do not edit.",
             "// Flops emitted per primitive quartet (VRR) and per contracted quartet (HRR + contraction),",
             "// indexed by ((la*3+lb)*3+lc)*3+ld.  Boys, pair set-up and exp are counted separately.",
             "#pragma once",
             "static const int fx_class_vrr_flops[81] = {" + ", ".join(str(s[1]) for s in stats) + "};",
             "static const int fx_class_hrr_flops[81] = {" + ", ".join(str(s[2]) for s in stats) + "};"]
    path = os.path.join(outdir, "eri_flops.h")
    new = "\n".join(lines) + "\n"
    if not os.path.exists(path) or open(path).read() != new:
        open(path, "w").write(new)
    return stats


if __name__ == "__main__":
    st = main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen"))
    for s in st:
        print(*s)
