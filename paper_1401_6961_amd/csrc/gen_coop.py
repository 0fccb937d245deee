"""Cooperative (one quartet per wave) variant of the HGP class routines.

For angular-momentum classes whose contracted intermediates do not fit in
one lane's registers (e.g. (dd|dd): 961 accumulated [e0|f0] values and a
few thousand VRR intermediates), the wave evaluates one shell quartet at a
time: every intermediate of the Obara-Saika VRR, the primitive sum and the
HRR lives in an LDS slot, and the elements of each recursion level are
spread over the 64 lanes.  The generator

  * builds the same recursion DAGs as gen_eri.py (same direction choices),
  * orders the elements by dependency level and groups each level by
    formula shape (bra OS / ket transfer, direction, which terms exist), so
    that every group is one loop with compile-time coefficients,
  * allocates LDS slots with liveness (VRR slots are reused per primitive
    quartet, HRR reuses the VRR space; the accumulated [e0|f0] persist),
  * emits packed 16-bit slot descriptors per element and the slot table of
    the final contraction, in which lane t owns K element t of the block.
"""
from __future__ import annotations

import itertools

from gen_eri import LNAME, XYZ, add, argmax_dir, cart, comp_factor, orientation, sub


class Node:
    __slots__ = ("key", "kind", "dir", "deps", "k", "e", "level", "slot", "last")

    def __init__(self, key, kind, d=None, deps=(), k=0, e=0):
        self.key, self.kind, self.dir, self.deps, self.k, self.e = key, kind, d, deps, k, e
        self.level = 0
        self.slot = None
        self.last = -1


def build_vrr(L):
    """Symbolic VRR DAG; returns (nodes by key, targets list)."""
    l1, l2, l3, l4 = L
    nodes = {}

    def get(e, f, m):
        if min(e) < 0 or min(f) < 0:
            return None
        key = (e, f, m)
        if key in nodes:
            return nodes[key]
        if sum(e) == 0 and sum(f) == 0:
            n = Node(key, "base")
        elif sum(f) == 0:
            i = argmax_dir(e)
            e1 = sub(e, i)
            k = e1[i]
            a0, a1 = get(e1, f, m), get(e1, f, m + 1)
            b0 = b1 = None
            if k > 0:
                b0, b1 = get(sub(e1, i), f, m), get(sub(e1, i), f, m + 1)
            n = Node(key, "os", i, (a0, a1, b0, b1, None), k, 0)
        else:
            i = argmax_dir(f)
            f1 = sub(f, i)
            k = f1[i]
            a0, a1 = get(e, f1, m), get(e, f1, m + 1)
            b0 = b1 = c1 = None
            if k > 0:
                b0, b1 = get(e, sub(f1, i), m), get(e, sub(f1, i), m + 1)
            if e[i] > 0:
                c1 = get(sub(e, i), f1, m + 1)
            n = Node(key, "et", i, (a0, a1, b0, b1, c1), k, e[i])
        nodes[key] = n
        return n

    targets = []
    for le in range(l1, l1 + l2 + 1):
        for e in cart(le):
            for lf in range(l3, l3 + l4 + 1):
                for f in cart(lf):
                    targets.append(get(e, f, 0))
    return nodes, targets


def build_hrr(L, target_of):
    """Symbolic HRR DAG over the accumulated targets C(e,f)."""
    nodes = {}

    def bra(a, b, f):
        key = ("b", a, b, f)
        if key in nodes:
            return nodes[key]
        if sum(b) == 0:
            n = Node(key, "C", deps=(target_of[(a, f)],))
        else:
            i = argmax_dir(b)
            b1 = sub(b, i)
            n = Node(key, "hb", i, (bra(add(a, i), b1, f), bra(a, b1, f)))
        nodes[key] = n
        return n

    def full(a, b, c, d):
        key = ("k", a, b, c, d)
        if key in nodes:
            return nodes[key]
        if sum(d) == 0:
            n = bra(a, b, c)
        else:
            i = argmax_dir(d)
            d1 = sub(d, i)
            n = Node(key, "hk", i, (full(a, b, add(c, i), d1), full(a, b, c, d1)))
        nodes[key] = n
        return n

    return nodes, full


def levels_of(nodes, leaf_kinds):
    order = []
    seen = set()

    def visit(n):
        if id(n) in seen:
            return
        seen.add(id(n))
        for d in n.deps:
            if d is not None and d.kind not in leaf_kinds:
                visit(d)
        lv = 0
        for d in n.deps:
            if d is not None and d.kind not in leaf_kinds:
                lv = max(lv, d.level + 1)
        n.level = lv
        order.append(n)

    for n in list(nodes.values()):
        if n.kind not in leaf_kinds:
            visit(n)
    return order


class SlotAlloc:
    def __init__(self, first):
        self.free = []
        self.next = first
        self.high = first

    def get(self):
        if self.free:
            return self.free.pop()
        s = self.next
        self.next += 1
        self.high = max(self.high, self.next)
        return s

    def put(self, s):
        self.free.append(s)


def gen_coop(la, lb, lc, ld, real):
    """Device routine for one class (FP64 or FP32 recursion).
    Returns (code, nslot)."""
    ls = (la, lb, lc, ld)
    o = orientation(la, lb, lc, ld)
    L = [ls[x] for x in o]
    Lsum = sum(L)
    vnodes, targets = build_vrr(L)
    target_of = {(t.key[0], t.key[1]): t for t in targets}
    # ---------------- VRR levels (base nodes are level 0 leaves) ----------
    base = [vnodes[((0, 0, 0), (0, 0, 0), m)] for m in range(Lsum + 1) if ((0, 0, 0), (0, 0, 0), m) in vnodes]
    order = levels_of(vnodes, {"base"})
    for n in order:
        n.level += 1           # base values are written at level 0
    nlev = max([n.level for n in order], default=0)
    # last use: the level at which the node is read (+ accumulation of targets one level later)
    for n in order:
        for d in n.deps:
            if d is not None:
                d.last = max(d.last, n.level)
    tset = set(id(t) for t in targets)
    for t in targets:
        t.last = max(t.last, t.level + 1)   # accumulated in the next level's step
    for b in base:
        b.last = max(b.last, 1)
    # slots: 0 = zero, 1..NC = accumulators C
    NC = len(targets)
    cslot = {id(t): 1 + k for k, t in enumerate(targets)}
    alloc = SlotAlloc(1 + NC)
    by_level = {}
    for n in order:
        by_level.setdefault(n.level, []).append(n)
    for b in base:
        b.slot = alloc.get()
    frees = {}
    for n in list(base) + order:
        frees.setdefault(n.last, []).append(n)
    for lv in range(1, nlev + 2):
        for n in by_level.get(lv, []):
            n.slot = alloc.get()
        # nodes whose last use is this level can be reused from the next level on
        for n in frees.get(lv, []):
            alloc.put(n.slot)
    vrr_high = alloc.high
    # ---------------- HRR -------------------------------------------------
    hnodes, full = build_hrr(L, target_of)
    comps = [cart(l) for l in ls]
    outs = {}
    for mu, nu, lam, sig in itertools.product(*comps):
        ext = (mu, nu, lam, sig)
        t = [None] * 4
        for pos, role in enumerate(o):
            t[pos] = ext[role]
        outs[(mu, nu, lam, sig)] = full(*t)
    horder = levels_of(hnodes, {"C"})
    for n in horder:
        n.level += 1
    hlev = max([n.level for n in horder], default=0)
    for n in hnodes.values():
        if n.kind == "C":
            n.slot = cslot[id(n.deps[0])]
            n.level = 0
    for n in horder:
        for d in n.deps:
            if d.kind != "C":
                d.last = max(d.last, n.level)
    FINAL = hlev + 1
    for n in outs.values():
        if n.kind != "C":
            n.last = FINAL
    halloc = SlotAlloc(1 + NC)
    hby = {}
    for n in horder:
        hby.setdefault(n.level, []).append(n)
    hfree = {}
    for n in horder:
        hfree.setdefault(n.last, []).append(n)
    for lv in range(1, hlev + 1):
        for n in hby.get(lv, []):
            n.slot = halloc.get()
        for n in hfree.get(lv, []):
            halloc.put(n.slot)
    nslot = max(vrr_high, halloc.high)
    assert nslot < 65536
    # ---------------- emit ------------------------------------------------
    cls = f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"
    prec = "f32" if real == "float" else "f64"
    fx = "f" if real == "float" else ""
    tab_v, tab_a, tab_h = [], [], []
    code = []
    w = code.append
    w(f"// cooperative class ({LNAME[la]}{LNAME[lb]}|{LNAME[lc]}{LNAME[ld]}) {prec}: {len(order)} VRR elements in "
      f"{nlev} levels, {len(horder)} HRR elements in {hlev} levels, {nslot} LDS slots")
    body = []
    b = body.append
    # VRR level loops
    for lv in range(1, nlev + 2):
        groups = {}
        for n in by_level.get(lv, []):
            key = (n.kind, n.dir, n.deps[2] is not None, n.deps[4] is not None)
            groups.setdefault(key, []).append(n)
        for (kind, i, hb, hc), ns in sorted(groups.items(), key=lambda x: str(x[0])):
            off = len(tab_v) // 8
            for n in ns:
                d = n.deps
                tab_v += [n.slot, d[0].slot, d[1].slot, d[2].slot if d[2] else 0, d[3].slot if d[3] else 0,
                          d[4].slot if d[4] else 0, n.k, n.e]
            c1, c2 = ("PA", "WP") if kind == "os" else ("QC", "WQ")
            h1, h2 = ("oo2p", "oo2p_rp") if kind == "os" else ("oo2q", "oo2q_rq")
            expr = f"{c1}{XYZ[i]} * S[t.y] + {c2}{XYZ[i]} * S[t.z]"
            if hb:
                expr += f" + ({real})t2.z * ({h1} * S[t.w] - {h2} * S[t2.x])"
            if hc:
                expr += f" + ({real})t2.w * oo2pq * S[t2.y]"
            b(f"    for (int j = lane; j < {len(ns)}; j += 64) {{")
            b(f"      const uint4 t = fx_unpack_lo(vtab + (long)({off} + j) * 8), t2 = fx_unpack_hi(vtab + (long)({off} + j) * 8);")
            b(f"      S[t.x] = {expr};")
            b("    }")
        # accumulate the previous level's targets
        prev = [t for t in targets if t.level == lv - 1]
        if prev:
            aoff = len(tab_a) // 2
            for t in prev:
                tab_a += [cslot[id(t)], t.slot]
            b(f"    for (int j = lane; j < {len(prev)}; j += 64) {{ const int c = atab[2 * ({aoff} + j)], s = atab[2 * ({aoff} + j) + 1]; S[c] += S[s]; }}")
        b("    fx_wave_sync();")
    vrr_body = body
    # HRR
    body = []
    b = body.append
    for lv in range(1, hlev + 1):
        groups = {}
        for n in hby.get(lv, []):
            groups.setdefault((n.kind, n.dir), []).append(n)
        for (kind, i), ns in sorted(groups.items(), key=lambda x: str(x[0])):
            off = len(tab_h) // 4
            for n in ns:
                tab_h += [n.slot, n.deps[0].slot, n.deps[1].slot, 0]
            g = "AB" if kind == "hb" else "CD"
            b(f"  for (int j = lane; j < {len(ns)}; j += 64) {{")
            b(f"    const ushort4 t = *(const ushort4*)(htab + (long)({off} + j) * 4);")
            b(f"    S[t.x] = S[t.y] + {g}{XYZ[i]}_ * S[t.z];")
            b("  }")
        b("  fx_wave_sync();")
    hrr_body = body
    # contraction slot table: [t = mu*nd + sig][nu*nc + lam]
    na, nb, nc, nd = [len(c) for c in comps]
    tab_c = []
    for im, mu in enumerate(comps[0]):
        for ls_, sig in enumerate(comps[3]):
            for jn, nu in enumerate(comps[1]):
                for kl, lam in enumerate(comps[2]):
                    tab_c.append(outs[(mu, nu, lam, sig)].slot)
    pfac = []
    for jn, nu in enumerate(comps[1]):
        for kl, lam in enumerate(comps[2]):
            pfac.append(comp_factor(nu) * comp_factor(lam))

    def arr(name, vals, typ="uint16_t"):
        rows = []
        for s in range(0, len(vals), 24):
            rows.append(", ".join(str(v) for v in vals[s:s + 24]))
        return f"static __device__ const {typ} {name}[{max(1, len(vals))}] = {{\n  " + ",\n  ".join(rows or ["0"]) + "\n};"

    pre = f"coop_{cls}_{prec}"
    w(arr(f"{pre}_v", tab_v))
    w(arr(f"{pre}_a", tab_a))
    w(arr(f"{pre}_h", tab_h))
    w(arr(f"{pre}_c", tab_c))
    w(f"struct {pre} {{ static constexpr int NSLOT = {nslot}; }};")
    w(f"__device__ __forceinline__ void eri_{cls}_{prec}_coop(const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc,")
    w(f"    const FxShellRef& rd, const FxDevBasis& B, const double* __restrict__ boys_tab,")
    w(f"    const double* __restrict__ Pmat, long ldp, {real}* __restrict__ S, double& kacc) {{")
    w("  const int lane = fx_lane();")
    w(f"  const uint16_t* __restrict__ vtab = {pre}_v;")
    w(f"  const uint16_t* __restrict__ atab = {pre}_a;")
    w(f"  const uint16_t* __restrict__ htab = {pre}_h;")
    roles = ["ra", "rb", "rc", "rd"]
    x = [roles[r] for r in o]
    w(f"  const FxShellRef& x1 = {x[0]}; const FxShellRef& x2 = {x[1]}; const FxShellRef& x3 = {x[2]}; const FxShellRef& x4 = {x[3]};")
    w(f"  for (int j = lane; j <= {NC}; j += 64) S[j] = 0;")
    w("  fx_wave_sync();")
    w("  const double ABx = x1.x - x2.x, ABy = x1.y - x2.y, ABz = x1.z - x2.z;")
    w("  const double CDx = x3.x - x4.x, CDy = x3.y - x4.y, CDz = x3.z - x4.z;")
    w("  const long Nt = B.ntprim;")
    w("  const FxPrimPair* __restrict__ pab = B.pp + (long)x1.pofs * Nt + x2.pofs;")
    w("  const FxPrimPair* __restrict__ pcd = B.pp + (long)x3.pofs * Nt + x4.pofs;")
    w("  for (int i1 = 0; i1 < x1.nprim; ++i1)")
    w("  for (int i2 = 0; i2 < x2.nprim; ++i2) {")
    w("    const FxPrimPair bra = pab[i1 * Nt + i2];")
    w("    const double p = bra.p, op = bra.op, Px = bra.Px, Py = bra.Py, Pz = bra.Pz;")
    w("    for (int i3 = 0; i3 < x3.nprim; ++i3)")
    w("    for (int i4 = 0; i4 < x4.nprim; ++i4) {")
    w("    const FxPrimPair ket = pcd[i3 * Nt + i4];")
    w("    const double q = ket.p, oq = ket.op, Qx = ket.Px, Qy = ket.Py, Qz = ket.Pz;")
    w("    const double ppq = p + q, oppq = 1.0 / ppq, rho = p * q * oppq;")
    w("    const double PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;")
    w("    const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);")
    w("    const double pref = FX_TWO_PI_POW_2_5 * op * oq * sqrt(oppq) * bra.K * ket.K;")
    w(f"    double F[{Lsum + 1}];")
    w(f"    fx_boys<{Lsum}>(T, boys_tab, F);")
    w("    const double Wx = (p * Px + q * Qx) * oppq, Wy = (p * Py + q * Qy) * oppq, Wz = (p * Pz + q * Qz) * oppq;")
    for c in "xyz":
        w(f"    const {real} PA{c} = ({real})(P{c} - x1.{c}), WP{c} = ({real})(W{c} - P{c});")
        w(f"    const {real} QC{c} = ({real})(Q{c} - x3.{c}), WQ{c} = ({real})(W{c} - Q{c});")
    w(f"    const {real} oo2p = ({real})(0.5 * op), oo2q = ({real})(0.5 * oq), oo2pq = ({real})(0.5 * oppq);")
    w(f"    const {real} oo2p_rp = ({real})(0.5 * op * rho * op), oo2q_rq = ({real})(0.5 * oq * rho * oq);")
    for bnode in base:
        w(f"    if (lane == 0) S[{bnode.slot}] = ({real})(pref * F[{bnode.key[2]}]);")
    w("    fx_wave_sync();")
    code += vrr_body
    w("  }")
    w("  }")
    w(f"  const {real} ABx_ = ({real})ABx, ABy_ = ({real})ABy, ABz_ = ({real})ABz;")
    w(f"  const {real} CDx_ = ({real})CDx, CDy_ = ({real})CDy, CDz_ = ({real})CDz;")
    code += hrr_body
    # contraction: lane t owns element (mu, sig) = (t / nd, t % nd)
    w(f"  if (lane < {na * nd}) {{")
    w(f"    const uint16_t* __restrict__ ct = {pre}_c + lane * {nb * nc};")
    w("    double s = 0.0;")
    for jn in range(nb):
        for kl in range(nc):
            j = jn * nc + kl
            fac = pfac[j]
            pv = f"Pmat[{jn} * ldp + {kl}]" + ("" if abs(fac - 1) < 1e-15 else f" * {fac!r}")
            w(f"    s += (double)S[ct[{j}]] * ({pv});")
    w("    kacc += s;")
    w("  }")
    w("  fx_wave_sync();")
    w("}")
    return "\n".join(code), nslot


if __name__ == "__main__":
    import sys
    la, lb, lc, ld = [LNAME.index(ch) for ch in sys.argv[1]]
    code, ns = gen_coop(la, lb, lc, ld, "double")
    print(code.splitlines()[0], "nslot", ns, "bytes/wave", ns * 8)
