"""Seeded synthetic molecular inputs for the exchange build.

This module only draws inputs: atom positions, Gaussian shells (angular
momentum, exponents, raw contraction weights) and a decaying density matrix
P.  It holds none of the exchange method's arithmetic (no normalisation, no
integrals, no norms, no screening); both the plain CPU oracle and the GPU
library consume exactly the arrays produced here.

The paper measures water droplets (H2O)_n at B3LYP/6-31G** with converged
densities (Section V); those are not available, so these seeded systems
stand in for them: 6-31G**-like s/p/d shell mixes on randomly placed atoms,
and a density whose magnitude decays exponentially with the distance between
function centres, which is the structure the metric query of Eq. (8) relies
on (Section III: the method needs decay, not sparsification).

Conventions (fixed here, shared by both sides):
  * lengths are drawn in Angstrom and returned in bohr (a0 = 0.529177210903 A);
  * exponents are in bohr^-2;
  * shells of an atom are consecutive in the order s, p, d; functions of a
    shell are its Cartesian components in lexicographic order
    (p: x, y, z;  d: xx, xy, xz, yy, yz, zz);
  * coefs are raw weights d_p in U[0.1, 1] that multiply *normalised*
    primitives; the consumer renormalises each contracted function;
  * P_ij = u_ij * exp(-|R_i - R_j| / L) with R the atom centre of function
    i (distance 0 within an atom), u_ij = u_ji ~ U(-1, 1) taken from the
    upper triangle of a row-major uniform draw, P_ii = 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
NCART = (1, 3, 6)


@dataclasses.dataclass
class System:
    name: str
    atoms: np.ndarray          # (natom, 3) Angstrom
    l: np.ndarray              # (nshell,) int32
    nprim: np.ndarray          # (nshell,) int32
    center: np.ndarray         # (nshell, 3) float64, bohr
    exps: np.ndarray           # (sum nprim,) float64, bohr^-2
    coefs: np.ndarray          # (sum nprim,) float64, raw weights
    shell_atom: np.ndarray     # (nshell,) int32
    P: np.ndarray | None       # (n, n) float64
    tau: float

    @property
    def nshell(self) -> int:
        return int(self.l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(NCART[x] for x in self.l))

    def func_atom(self) -> np.ndarray:
        return np.repeat(self.shell_atom, [NCART[x] for x in self.l]).astype(np.int32)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def _rsa(rng, natom, draw, min_sep):
    """Random sequential addition: accept candidates from draw() in seed order
    while they keep at least min_sep (Angstrom) from every accepted atom."""
    pts = np.empty((natom, 3))
    k = 0
    tries = 0
    while k < natom:
        c = draw()
        tries += 1
        if tries > 200 * natom + 10000:
            raise RuntimeError("random sequential addition did not converge")
        if k:
            d2 = np.sum((pts[:k] - c) ** 2, axis=1)
            if d2.min() < min_sep * min_sep:
                continue
        pts[k] = c
        k += 1
    return pts


def cube_atoms(rng, natom, edge, min_sep=1.0):
    return _rsa(rng, natom, lambda: rng.uniform(0.0, edge, 3), min_sep)


def box_atoms(rng, natom, dims, min_sep=1.0):
    dims = np.asarray(dims, dtype=float)
    return _rsa(rng, natom, lambda: rng.uniform(0.0, 1.0, 3) * dims, min_sep)


def sphere_atoms(rng, natom, density=0.1, min_sep=1.0):
    """Uniform in a sphere of radius (3N / (4 pi rho))^(1/3) Angstrom."""
    r = (3.0 * natom / (4.0 * math.pi * density)) ** (1.0 / 3.0)

    def draw():
        while True:
            c = rng.uniform(-r, r, 3)
            if c @ c <= r * r:
                return c
    return _rsa(rng, natom, draw, min_sep)


def chain_atoms(rng, natom, spacing=1.5, jitter=0.1):
    x = np.arange(natom, dtype=float) * spacing
    pts = np.zeros((natom, 3))
    pts[:, 0] = x
    pts += rng.uniform(-jitter, jitter, (natom, 3))
    return pts


# ----------------------------------------------------------------------------
# basis
# ----------------------------------------------------------------------------
def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def make_shells(rng, atoms, with_d):
    """Per atom: s (3 primitives, exponents log-U[0.1, 20]),
    p (2 primitives, log-U[0.1, 5]) and optionally Cartesian d
    (1 primitive, exponent U[0.3, 1.5]); weights U[0.1, 1]."""
    ls, nps, ctr, ex, co, sa = [], [], [], [], [], []
    for ia, xyz in enumerate(atoms):
        specs = [(0, 3, "log", 0.1, 20.0), (1, 2, "log", 0.1, 5.0)]
        if with_d:
            specs.append((2, 1, "lin", 0.3, 1.5))
        for l, k, kind, lo, hi in specs:
            e = _loguniform(rng, lo, hi, k) if kind == "log" else rng.uniform(lo, hi, k)
            c = rng.uniform(0.1, 1.0, k)
            ls.append(l)
            nps.append(k)
            ctr.append(xyz * BOHR_PER_ANGSTROM)
            ex.extend(e)
            co.extend(c)
            sa.append(ia)
    return (np.asarray(ls, np.int32), np.asarray(nps, np.int32),
            np.asarray(ctr, np.float64).reshape(-1, 3),
            np.asarray(ex, np.float64), np.asarray(co, np.float64),
            np.asarray(sa, np.int32))


def make_density(rng, atoms, func_atom, decay_angstrom, row_block=2048):
    """Symmetric P with P_ij = u_ij exp(-|R_i - R_j| / L), P_ii = 1."""
    n = func_atom.shape[0]
    P = rng.uniform(-1.0, 1.0, size=(n, n))
    # mirror the strict upper triangle onto the lower one, block by block
    for i0 in range(0, n, row_block):
        i1 = min(n, i0 + row_block)
        blk = P[i0:i1, i0:i1]
        iu = np.triu_indices(i1 - i0, 1)
        blk[(iu[1], iu[0])] = blk[iu]
        if i0:
            P[i0:i1, :i0] = P[:i0, i0:i1].T
    fa = atoms[func_atom]
    for i0 in range(0, n, row_block):
        i1 = min(n, i0 + row_block)
        d = np.sqrt(((fa[i0:i1, None, :] - fa[None, :, :]) ** 2).sum(-1))
        P[i0:i1] *= np.exp(-d / decay_angstrom)
    np.fill_diagonal(P, 1.0)
    return P


def assemble(name, rng, atoms, with_d, decay, tau, density=True):
    l, nprim, center, exps, coefs, sa = make_shells(rng, atoms, with_d)
    sys_ = System(name, atoms, l, nprim, center, exps, coefs, sa, None, tau)
    if density:
        sys_.P = make_density(rng, atoms, sys_.func_atom(), decay)
    return sys_


# ----------------------------------------------------------------------------
# the five workloads (and scaled-down relatives used by tests)
# ----------------------------------------------------------------------------
def tiny_cube(natom=24, edge=8.0, seed=1000, tau=1e-12, with_d=False):
    rng = np.random.default_rng(seed)
    atoms = cube_atoms(rng, natom, edge)
    return assemble(f"cube{natom}", rng, atoms, with_d, 2.0, tau)


def chain(natom=200, seed=1001, tau=1e-8, with_d=False):
    rng = np.random.default_rng(seed)
    atoms = chain_atoms(rng, natom)
    return assemble(f"chain{natom}", rng, atoms, with_d, 2.0, tau)


def cluster(natom=1000, seed=1002, tau=1e-8, with_d=True, density=True):
    rng = np.random.default_rng(seed)
    atoms = sphere_atoms(rng, natom)
    return assemble(f"cluster{natom}{'spd' if with_d else 'sp'}", rng, atoms,
                    with_d, 2.0, tau, density)


def batch_clusters(count=64, seed=1003, tau=1e-8, lo=50, hi=500):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        natom = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        atoms = sphere_atoms(rng, natom)
        out.append(assemble(f"batch{i}_{natom}", rng, atoms, False, 2.0, tau))
    return out


def slab(natom=4000, dims=(40.0, 40.0, 25.0), seed=1004, tau=1e-8, density=True):
    rng = np.random.default_rng(seed)
    atoms = box_atoms(rng, natom, dims)
    return assemble(f"slab{natom}", rng, atoms, False, 2.0, tau, density)


def config(i: int, **kw):
    """The five named workloads: 0 tiny cube, 1 chain, 2 s+p+d cluster,
    3 batch of 64 clusters (a list), 4 s+p slab."""
    return [tiny_cube, chain, cluster, batch_clusters, slab][i](**kw)
