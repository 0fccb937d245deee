"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to mathematics fixed independently of
its code: closed forms of the Boys function and of (ss|ss), derivative
identities of Gaussians (finite differences of the closed form give p and d
integrals), the asymptotic 1/R law (which fixes the normalisation of every
Cartesian component), permutational symmetry, the Schwarz inequality,
positive semi-definiteness, translation and rotation covariance, and, for
the exchange build of Eq. (6) with the metric query of Eq. (8), linearity,
symmetry, the probe identity, the 4-index energy sum and the rigorous bound
on what culling drops.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import synthetic
from synthetic import System


def custom(shells, P=None, tau=1e-10):
    """shells: list of (l, center_bohr(3), exps, coefs)."""
    l = np.array([s[0] for s in shells], np.int32)
    nprim = np.array([len(s[2]) for s in shells], np.int32)
    ctr = np.array([s[1] for s in shells], np.float64).reshape(-1, 3)
    ex = np.concatenate([np.asarray(s[2], float) for s in shells])
    co = np.concatenate([np.asarray(s[3], float) for s in shells])
    sys_ = System("custom", ctr / synthetic.BOHR_PER_ANGSTROM, l, nprim, ctr, ex, co,
                  np.arange(len(shells), dtype=np.int32), P, tau)
    return sys_


# --------------------------------------------------------------------------
# Boys function
# --------------------------------------------------------------------------
def boys_ref(m, T):
    """F_m(T) = Gamma(m+1/2) P(m+1/2, T) / (2 T^(m+1/2)) (regularised
    lower incomplete gamma, scipy)."""
    if T == 0:
        return 1.0 / (2 * m + 1)
    return sp.gamma(m + 0.5) * sp.gammainc(m + 0.5, T) / (2.0 * T ** (m + 0.5))


@pytest.mark.parametrize("T", [0.0, 1e-9, 1e-3, 0.37, 2.5, 7.9, 15.0, 29.99, 30.0, 30.01, 45.0, 120.0, 1e4])
def test_boys_incomplete_gamma(T):
    F = oracle.boys(8, T)
    for m in range(9):
        ref = boys_ref(m, T)
        assert abs(F[m] - ref) <= 1e-13 * abs(ref) + 1e-300, (m, T, F[m], ref)


def test_boys_zero_and_asymptotic_and_downward():
    assert np.allclose(oracle.boys(8, 0.0), [1.0 / (2 * m + 1) for m in range(9)], rtol=0, atol=0)
    # large-T asymptotic F_m ~ (2m-1)!! / 2^(m+1) sqrt(pi / T^(2m+1))
    T = 400.0
    F = oracle.boys(8, T)
    for m in range(9):
        df = float(np.prod(np.arange(2 * m - 1, 0, -2))) if m else 1.0
        assert abs(F[m] / (df / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))) - 1) < 1e-12
    # downward identity F_m = (2T F_{m+1} + e^{-T}) / (2m+1) on both sides of the series/erf switch
    for T in (0.5, 12.0, 29.0, 31.0, 60.0):
        F = oracle.boys(8, T)
        for m in range(8):
            assert abs((2 * T * F[m + 1] + math.exp(-T)) / (2 * m + 1) - F[m]) < 1e-14 * F[m]
    # F_0 from erf
    for T in (0.1, 3.0, 50.0):
        assert abs(oracle.boys(0, T)[0] - 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))) < 1e-15


# --------------------------------------------------------------------------
# (ss|ss) closed form and its derivatives
# --------------------------------------------------------------------------
def ssss(alphas, centers):
    """Closed form over four normalised s primitives:
    2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd F_0(rho |PQ|^2)."""
    a, b, c, d = alphas
    A, B, C, D = [np.asarray(x, float) for x in centers]
    N = [(2 * x / math.pi) ** 0.75 for x in alphas]
    p, q = a + b, c + d
    P = (a * A + b * B) / p
    Q = (c * C + d * D) / q
    Kab = math.exp(-a * b / p * np.dot(A - B, A - B))
    Kcd = math.exp(-c * d / q * np.dot(C - D, C - D))
    rho = p * q / (p + q)
    T = rho * np.dot(P - Q, P - Q)
    F0 = 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    return 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * Kab * Kcd * F0 * N[0] * N[1] * N[2] * N[3]


def test_ssss_closed_form_primitives():
    rng = np.random.default_rng(7)
    for _ in range(20):
        al = np.exp(rng.uniform(math.log(0.1), math.log(20), 4))
        ctr = rng.uniform(-2, 2, (4, 3))
        s = custom([(0, ctr[i], [al[i]], [0.7]) for i in range(4)])
        got = oracle.eri_quartet(s, 0, 1, 2, 3)[0, 0, 0, 0]
        ref = ssss(al, ctr)
        assert abs(got - ref) <= 1e-13 * abs(ref)


def test_ssss_contracted_is_weighted_sum():
    rng = np.random.default_rng(8)
    ex = [np.exp(rng.uniform(math.log(0.1), math.log(20), 3)) for _ in range(4)]
    co = [rng.uniform(0.1, 1, 3) for _ in range(4)]
    ctr = rng.uniform(-2, 2, (4, 3))
    s = custom([(0, ctr[i], ex[i], co[i]) for i in range(4)])
    c = oracle.norm_coefs(s)[:, 0, :3]   # normalised weights of normalised... (radial incl. N)
    got = oracle.eri_quartet(s, 0, 1, 2, 3)[0, 0, 0, 0]
    ref = 0.0
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for m in range(3):
                    al = (ex[0][i], ex[1][j], ex[2][k], ex[3][m])
                    Nprod = np.prod([(2 * x / math.pi) ** 0.75 for x in al])
                    ref += c[0, i] * c[1, j] * c[2, k] * c[3, m] / Nprod * ssss(al, ctr)
    assert abs(got - ref) <= 1e-13 * abs(ref)


def test_same_centre_and_far_field():
    al = 0.83
    s = custom([(0, [0, 0, 0], [al], [1.0])])
    assert abs(oracle.eri_quartet(s, 0, 0, 0, 0)[0, 0, 0, 0] - 2 * math.sqrt(al / math.pi)) < 1e-14
    # two normalised s distributions: (aa|bb) = erf(sqrt(pq/(p+q)) R) / R
    for R in (0.3, 2.0, 9.0):
        s = custom([(0, [0, 0, 0], [al], [1.0]), (0, [0, 0, R], [1.7], [1.0])])
        p, q = 2 * al, 2 * 1.7
        ref = math.erf(math.sqrt(p * q / (p + q)) * R) / R
        assert abs(oracle.eri_quartet(s, 0, 0, 1, 1)[0, 0, 0, 0] - ref) < 1e-14


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 1), (2, 2), (2, 1), (0, 2)])
def test_far_field_fixes_every_component_normalisation(la, lb):
    """(mu mu|nu nu) -> 1/R for R -> inf iff every Cartesian component is
    normalised to (phi|phi) = 1 (charge of phi_mu^2 is 1)."""
    rng = np.random.default_rng(3 + la * 3 + lb)
    R = 2.0e4
    sa = (la, [0, 0, 0], np.exp(rng.uniform(math.log(0.1), math.log(5), 2)), rng.uniform(0.1, 1, 2))
    sb = (lb, [0.3 * R, -0.4 * R, 0.866 * R], np.exp(rng.uniform(math.log(0.1), math.log(5), 2)),
          rng.uniform(0.1, 1, 2))
    s = custom([sa, sb])
    dist = np.linalg.norm(s.center[1] - s.center[0])
    I = oracle.eri_quartet(s, 0, 0, 1, 1)
    for m in range(I.shape[0]):
        for n in range(I.shape[2]):
            assert abs(I[m, m, n, n] * dist - 1.0) < 1e-6


def _fd1(f, x0, i, h):
    def D(hh):
        e = np.zeros_like(x0); e[i] = hh
        return (f(x0 + e) - f(x0 - e)) / (2 * hh)
    d1, d2, d3 = D(h), D(h / 2), D(h / 4)
    r1, r2 = (4 * d2 - d1) / 3, (4 * d3 - d2) / 3
    return (16 * r2 - r1) / 15


def _fd2(f, x0, i, j, h):
    def D(hh):
        if i == j:
            e = np.zeros_like(x0); e[i] = hh
            return (f(x0 + e) - 2 * f(x0) + f(x0 - e)) / hh ** 2
        ei = np.zeros_like(x0); ei[i] = hh
        ej = np.zeros_like(x0); ej[j] = hh
        return (f(x0 + ei + ej) - f(x0 + ei - ej) - f(x0 - ei + ej) + f(x0 - ei - ej)) / (4 * hh * hh)
    d1, d2, d3 = D(h), D(h / 2), D(h / 4)
    r1, r2 = (4 * d2 - d1) / 3, (4 * d3 - d2) / 3
    return (16 * r2 - r1) / 15


def _sys_from_x(x, ls, al):
    return custom([(ls[k], x[3 * k:3 * k + 3], [al[k]], [1.0]) for k in range(4)])


def test_p_and_d_from_centre_derivatives():
    """A normalised p_i primitive equals alpha^{-1/2} d/dA_i of the
    normalised s primitive; d_ii = (d^2/dA_i^2 + 2 alpha) s / (sqrt3 alpha)
    and d_ij = d^2/dA_i dA_j s / alpha (i != j)."""
    rng = np.random.default_rng(11)
    al = np.array([0.9, 0.6, 1.3, 0.45])
    x0 = rng.uniform(-1.0, 1.0, 12)
    f = lambda x: ssss(al, x.reshape(4, 3))
    h = 0.02
    comps_p = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    # (p s|s s)
    I = oracle.eri_quartet(_sys_from_x(x0, [1, 0, 0, 0], al), 0, 1, 2, 3)
    for i in range(3):
        ref = _fd1(f, x0, i, h) / math.sqrt(al[0])
        assert abs(I[i, 0, 0, 0] - ref) < 1e-8 * max(1e-3, abs(ref))
    # (s s|s p)
    I = oracle.eri_quartet(_sys_from_x(x0, [0, 0, 0, 1], al), 0, 1, 2, 3)
    for i in range(3):
        ref = _fd1(f, x0, 9 + i, h) / math.sqrt(al[3])
        assert abs(I[0, 0, 0, i] - ref) < 1e-8 * max(1e-3, abs(ref))
    # (p p|s s) and (p s|p s)
    for ls, (o1, o2), idx in (([1, 1, 0, 0], (0, 3), lambda i, j: (i, j, 0, 0)),
                              ([1, 0, 1, 0], (0, 6), lambda i, j: (i, 0, j, 0)),
                              ([0, 1, 0, 1], (3, 9), lambda i, j: (0, i, 0, j))):
        I = oracle.eri_quartet(_sys_from_x(x0, ls, al), 0, 1, 2, 3)
        k1, k2 = [k for k in range(4) if ls[k]]
        for i in range(3):
            for j in range(3):
                ref = _fd2(f, x0, o1 + i, o2 + j, h) / math.sqrt(al[k1] * al[k2])
                assert abs(I[idx(i, j)] - ref) < 1e-7 * max(1e-3, abs(ref)), (ls, i, j)
    # (d s|s s): xx, xy, xz, yy, yz, zz
    I = oracle.eri_quartet(_sys_from_x(x0, [2, 0, 0, 0], al), 0, 1, 2, 3)
    dcomp = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for c, (i, j) in enumerate(dcomp):
        d2 = _fd2(f, x0, i, j, h)
        ref = (d2 + 2 * al[0] * f(x0)) / (math.sqrt(3) * al[0]) if i == j else d2 / al[0]
        assert abs(I[c, 0, 0, 0] - ref) < 1e-7 * max(1e-3, abs(ref)), c
    # (s s|d s) on the ket side
    I = oracle.eri_quartet(_sys_from_x(x0, [0, 0, 2, 0], al), 0, 1, 2, 3)
    for c, (i, j) in enumerate(dcomp):
        d2 = _fd2(f, x0, 6 + i, 6 + j, h)
        ref = (d2 + 2 * al[2] * f(x0)) / (math.sqrt(3) * al[2]) if i == j else d2 / al[2]
        assert abs(I[0, 0, c, 0] - ref) < 1e-7 * max(1e-3, abs(ref)), c


# --------------------------------------------------------------------------
# the four-index tensor
# --------------------------------------------------------------------------
def small_spd(natom=3, seed=21, edge=3.0):
    rng = np.random.default_rng(seed)
    atoms = synthetic.cube_atoms(rng, natom, edge)
    return synthetic.assemble("spd", rng, atoms, True, 2.0, 1e-10)


@pytest.fixture(scope="module")
def spd():
    s = small_spd()
    return s, oracle.eri_tensor(s)


def test_eightfold_symmetry(spd):
    s, T = spd
    sc = np.abs(T).max()
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2), (3, 2, 1, 0)]:
        assert np.abs(T - T.transpose(perm)).max() < 1e-13 * sc


def test_schwarz_inequality_and_norms(spd):
    s, T = spd
    n = s.nbf
    diag = np.einsum("ijij->ij", T)
    assert diag.min() > 0
    Q = np.sqrt(diag)
    assert np.all(np.abs(T) <= Q[:, :, None, None] * Q[None, None, :, :] * (1 + 1e-12) + 1e-300)
    # shell-block Frobenius norms of Q
    Qn = oracle.schwarz(s)
    off = np.concatenate([[0], np.cumsum([synthetic.NCART[x] for x in s.l])])
    for a in range(s.nshell):
        for b in range(s.nshell):
            blk = diag[off[a]:off[a + 1], off[b]:off[b + 1]]
            assert abs(Qn[a, b] - math.sqrt(blk.sum())) < 1e-13 * Qn[a, b]


def test_supermatrix_positive_semidefinite(spd):
    s, T = spd
    n = s.nbf
    M = T.reshape(n * n, n * n)
    w = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert w.min() > -1e-10 * w.max()


def test_translation_invariance(spd):
    s, T = spd
    s2 = small_spd()
    s2.center = s2.center + np.array([3.1, -7.4, 0.25])
    T2 = oracle.eri_tensor(s2)
    assert np.abs(T - T2).max() < 1e-11 * np.abs(T).max()


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_rotation_covariance(spd):
    """p components transform as a vector, Cartesian d as a symmetric
    tensor (after removing the per-component sqrt(3) normalisation)."""
    s, T = spd
    R = _rotation(np.random.default_rng(5))
    s2 = small_spd()
    s2.center = s2.center @ R.T
    T2 = oracle.eri_tensor(s2)
    dcomp = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    fac = [1.0, math.sqrt(3), math.sqrt(3), 1.0, math.sqrt(3), 1.0]
    Ud = np.zeros((6, 6))
    for c, (a, b) in enumerate(dcomp):
        for cp, (ap, bp) in enumerate(dcomp):
            tsum = R[a, ap] * R[b, bp] + (R[a, bp] * R[b, ap] if ap != bp else 0.0)
            Ud[c, cp] = fac[c] / fac[cp] * tsum
    blocks = [np.eye(1), R, Ud]
    n = s.nbf
    U = np.zeros((n, n))
    o = 0
    for l in s.l:
        k = synthetic.NCART[l]
        U[o:o + k, o:o + k] = blocks[l]
        o += k
    Tr = np.einsum("ia,jb,kc,ld,abcd->ijkl", U, U, U, U, T, optimize=True)
    assert np.abs(Tr - T2).max() < 1e-11 * np.abs(T).max()


# --------------------------------------------------------------------------
# the exchange build
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def spd_k(spd):
    s, T = spd
    return s, T, oracle.exchange(s, tau=-1.0)[0]


def test_bruteforce_exchange_matches_tensor_contraction(spd_k):
    s, T, K = spd_k
    ref = np.einsum("ijkl,jk->il", T, s.P)
    assert np.abs(K - ref).max() < 1e-13 * np.abs(ref).max()


def test_exchange_energy_equals_four_index_sum(spd_k):
    s, T, K = spd_k
    e4 = np.einsum("il,jk,ijkl->", s.P, s.P, T)
    assert abs(np.sum(s.P * K) - e4) < 1e-12 * abs(e4)


def test_probe_density_gives_integral_slices(spd_k):
    s, T, _ = spd_k
    n = s.nbf
    for nu, lam in [(0, 0), (1, 7), (12, 29), (4, 20)]:
        P = np.zeros((n, n))
        P[nu, lam] += 1.0
        P[lam, nu] += 1.0
        K, _ = oracle.exchange(s, P=P, tau=-1.0)
        ref = T[:, nu, lam, :] + T[:, lam, nu, :]
        assert np.abs(K - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_linearity_in_P(spd_k):
    s, _, K1 = spd_k
    rng = np.random.default_rng(2)
    n = s.nbf
    P2 = rng.uniform(-1, 1, (n, n))
    K2, _ = oracle.exchange(s, P=P2, tau=-1.0)
    K3, _ = oracle.exchange(s, P=s.P + 2.5 * P2, tau=-1.0)
    assert np.abs(K3 - (K1 + 2.5 * K2)).max() < 1e-12 * np.abs(K3).max()


@pytest.fixture(scope="module")
def cube10():
    s = synthetic.tiny_cube(natom=10, edge=6.0, seed=77, tau=1e-6)
    Kf, stf = oracle.exchange(s, tau=-1.0)
    return s, Kf, stf


@pytest.mark.parametrize("tau", [1e-8, 1e-6, 1e-4])
def test_culling_error_within_bound_matrix(cube10, tau):
    s, Kf, stf = cube10
    Kt, st = oracle.exchange(s, tau=tau)
    assert st["quartets"] < stf["quartets"]
    E = oracle.bound_matrix(s, tau)
    assert np.all(np.abs(Kt - Kf) <= E * (1 + 1e-9) + 1e-15)
    # symmetric P -> symmetric K also with culling (beta is transpose-symmetric)
    assert np.abs(Kt - Kt.T).max() < 1e-13 * np.abs(Kt).max()


def test_count_matches_exchange(cube10):
    s, _, _ = cube10
    for tau in (1e-7, 1e-5):
        _, st = oracle.exchange(s, tau=tau)
        cnt, prim, near = oracle.count(s, tau=tau)
        assert cnt.sum() == st["quartets"]
        assert prim == st["prim_quartets"]
        # s+p only
        assert cnt[2].sum() == 0 and cnt[:, 2].sum() == 0


def test_blocks_match_full(cube10):
    s, _, _ = cube10
    K, _ = oracle.exchange(s, tau=1e-7)
    off = np.concatenate([[0], np.cumsum([synthetic.NCART[x] for x in s.l])])
    pairs = [(0, 0), (3, 17), (19, 2), (11, 11)]
    blks, _ = oracle.exchange_blocks(s, pairs, tau=1e-7)
    for (a, d), B in zip(pairs, blks):
        assert np.abs(B - K[off[a]:off[a + 1], off[d]:off[d + 1]]).max() < 1e-15 * max(1, np.abs(K).max())


def test_atom_permutation_permutes_K(cube10):
    s, _, _ = cube10
    K, _ = oracle.exchange(s, tau=1e-7)
    rng = np.random.default_rng(9)
    natom = s.atoms.shape[0]
    perm = rng.permutation(natom)
    # rebuild the shell arrays in permuted atom order
    sh_of_atom = [np.nonzero(s.shell_atom == a)[0] for a in range(natom)]
    order = np.concatenate([sh_of_atom[a] for a in perm])
    poff = np.concatenate([[0], np.cumsum(s.nprim)])
    foff = np.concatenate([[0], np.cumsum([synthetic.NCART[x] for x in s.l])])
    fperm = np.concatenate([np.arange(foff[k], foff[k + 1]) for k in order])
    s2 = System("perm", s.atoms[perm], s.l[order], s.nprim[order], s.center[order],
                np.concatenate([s.exps[poff[k]:poff[k + 1]] for k in order]),
                np.concatenate([s.coefs[poff[k]:poff[k + 1]] for k in order]),
                np.arange(len(order), dtype=np.int32), s.P[np.ix_(fperm, fperm)], s.tau)
    K2, _ = oracle.exchange(s2, tau=1e-7)
    assert np.abs(K2 - K[np.ix_(fperm, fperm)]).max() < 1e-13 * np.abs(K).max()


def test_density_block_norms_match_numpy(spd):
    """Eq. (8) density factor: Pn_bc = max(||P_bc||_F, ||P_cb||_F) over the
    shell blocks, against numpy's Frobenius norm on a non-symmetric P."""
    s = spd[0]
    rng = np.random.default_rng(9)
    P = rng.standard_normal((s.nbf, s.nbf))
    Pn = oracle.pnorm(s, P)
    off = np.concatenate([[0], np.cumsum([(l + 1) * (l + 2) // 2 for l in s.l])])
    for b in range(s.nshell):
        for c in range(s.nshell):
            blk = P[off[b]:off[b + 1], off[c]:off[c + 1]]
            blkT = P[off[c]:off[c + 1], off[b]:off[b + 1]]
            ref = max(np.linalg.norm(blk), np.linalg.norm(blkT))
            assert abs(Pn[b, c] - ref) <= 1e-14 * ref
    assert np.array_equal(Pn, Pn.T)


def _culled_beta_sum(s, tau, Qn, Pn):
    """Shell-block sum of beta = (Q_ab Q_cd) P_bc over the culled quartets
    (beta <= tau), from the Schwarz and density norm tables alone, expanded
    to the function block of (a, d)."""
    S = s.nshell
    beta = (Qn[:, :, None, None] * Qn[None, None, :, :]) * Pn[None, :, :, None]   # [a, b, c, d]
    Es = np.where(beta <= tau, beta, 0.0).sum(axis=(1, 2))
    off = np.concatenate([[0], np.cumsum([synthetic.NCART[x] for x in s.l])])
    E = np.zeros((s.nbf, s.nbf))
    for a in range(S):
        for d in range(S):
            E[off[a]:off[a + 1], off[d]:off[d + 1]] = Es[a, d]
    return E, beta


@pytest.mark.parametrize("tau", [1e-8, 1e-6, 1e-4])
def test_bound_matrix_is_the_culled_beta_sum(cube10, tau):
    """The other side of the culling pin (Eq. 8 and the sub-multiplicativity
    argument after it): E is exactly the sum of the bounds of the culled
    quartets, so an E that drops the density factor, counts surviving
    quartets or sums every quartet fails here even though it would still
    bound |K_tau - K_full|."""
    s = cube10[0]
    Qn = oracle.schwarz(s)
    Pn = oracle.pnorm(s, s.P)
    E = oracle.bound_matrix(s, tau, Qn=Qn, Pn=Pn)
    ref, beta = _culled_beta_sum(s, tau, Qn, Pn)
    assert np.any(beta <= tau) and np.any(beta > tau)
    assert np.all(np.abs(E - ref) <= 1e-12 * np.maximum(ref, 1e-300))


def test_bound_matrix_limits(cube10):
    """Below the smallest bound nothing is culled (E = 0); above the largest
    everything is, and E is the full sum over (b, c) of (Q_ab Q_cd) P_bc."""
    s = cube10[0]
    Qn = oracle.schwarz(s)
    Pn = oracle.pnorm(s, s.P)
    beta = (Qn[:, :, None, None] * Qn[None, None, :, :]) * Pn[None, :, :, None]
    pos = beta[beta > 0]
    assert np.all(oracle.bound_matrix(s, 0.5 * pos.min(), Qn=Qn, Pn=Pn) == 0.0)
    E = oracle.bound_matrix(s, 2.0 * beta.max(), Qn=Qn, Pn=Pn)
    full = np.einsum("ab,cd,bc->ad", Qn, Qn, Pn)
    off = np.concatenate([[0], np.cumsum([synthetic.NCART[x] for x in s.l])])
    for a in range(s.nshell):
        for d in range(s.nshell):
            blk = E[off[a]:off[a + 1], off[d]:off[d + 1]]
            assert np.all(np.abs(blk - full[a, d]) <= 1e-12 * full[a, d])


@pytest.mark.parametrize("sep", [20.0, 60.0, 200.0])
def test_schwarz_far_pair_shortcut(sep):
    """The oracle's Schwarz table skips the diagonal integral of a pair whose
    Gaussian-product exponent mu R^2 is at least 575 for every primitive
    pair (the integral, proportional to exp(-2 mu R^2), is below the FP64
    range there).  Each table entry must equal the square root of the sum of
    the diagonal integrals evaluated directly, on both sides of the cut."""
    shells = [(0, [0.0, 0.0, 0.0], [0.5, 2.0], [0.6, 0.4]),
              (1, [sep, 0.0, 0.0], [0.4], [1.0]),
              (2, [0.0, sep, 0.3], [0.9], [1.0])]
    s = custom(shells)
    Qn = oracle.schwarz(s)
    cut = 0
    for a in range(3):
        for b in range(3):
            I = oracle.eri_quartet(s, a, b, a, b)
            na, nb = I.shape[0], I.shape[1]
            diag = np.array([I[i, j, i, j] for i in range(na) for j in range(nb)])
            ref = math.sqrt(np.maximum(diag, 0.0).sum())
            assert abs(Qn[a, b] - ref) <= 1e-13 * ref + 1e-300, (a, b, Qn[a, b], ref)
            mu_r2 = min(x * y / (x + y) for x in shells[a][2] for y in shells[b][2]) * \
                float(np.sum((np.array(shells[a][1]) - np.array(shells[b][1])) ** 2))   # centres in bohr
            if mu_r2 >= 575.0:
                assert Qn[a, b] == 0.0
                cut += 1
    assert cut > 0 or sep < 50.0


@pytest.mark.parametrize("tau", [1e-8, 1e-6])
def test_leafblock_rule_limits_and_bounds(cube10, tau):
    """The paper-literal leaf rule (whole leaf blocks computed): with leaves
    of single shells it is the shell-level rule; with one leaf holding the
    whole basis it is brute force; in between it computes a superset of the
    shell-level quartets (a block norm bounds its sub-blocks), so its K lies
    within the bound matrix of the shell-level culled work."""
    s, Kf, stf = cube10
    Ks, sts = oracle.exchange(s, tau=tau)
    K1, st1 = oracle.exchange_leafblock(s, 1, tau=tau)
    assert st1["near_threshold"] == 0 and st1["leaves"] == s.nshell
    assert st1["quartets"] == sts["quartets"]
    assert np.abs(K1 - Ks).max() <= 1e-14 * np.abs(Ks).max()
    Kall, stall = oracle.exchange_leafblock(s, s.nbf, tau=tau)
    assert stall["leaves"] == 1 and stall["quartets"] == stf["quartets"]
    assert np.abs(Kall - Kf).max() <= 1e-14 * np.abs(Kf).max()
    E = oracle.bound_matrix(s, tau)
    for leaf in (4, 10):
        Kb, stb = oracle.exchange_leafblock(s, leaf, tau=tau)
        assert stb["near_threshold"] == 0
        assert sts["quartets"] <= stb["quartets"] <= stf["quartets"]
        assert np.all(np.abs(Kb - Ks) <= E * (1 + 1e-9) + 1e-15)
        assert np.abs(Kb - Kb.T).max() <= 1e-13 * np.abs(Kb).max()


# --------------------------------------------------------------------------
# Overlaps (the criterion of Eqs. 3-4)
# --------------------------------------------------------------------------
def _overlap_quadrature(sh_a, sh_b):
    """<phi_a|phi_b> for single-primitive shells by Gauss-Hermite quadrature
    around the product centre (exact for these polynomial degrees), with
    each Cartesian component normalised by its own quadrature self-overlap."""
    from numpy.polynomial.hermite import hermgauss
    x, w = hermgauss(12)

    def comps(l):
        return [(i, j, l - i - j) for i in range(l, -1, -1) for j in range(l - i, -1, -1)]

    def integral(la, A, a, ta, lb, B, b, tb):
        p = a + b
        P = (a * np.asarray(A) + b * np.asarray(B)) / p
        val = np.exp(-a * b / p * np.sum((np.asarray(A) - np.asarray(B)) ** 2))
        for k in range(3):
            t = P[k] + x / np.sqrt(p)
            val *= np.sum(w * (t - A[k]) ** ta[k] * (t - B[k]) ** tb[k]) / np.sqrt(p)
        return val
    (la, A, a), (lb, B, b) = sh_a, sh_b
    out = np.zeros((len(comps(la)), len(comps(lb))))
    for i, ta in enumerate(comps(la)):
        na = integral(la, A, a, ta, la, A, a, ta)
        for j, tb in enumerate(comps(lb)):
            nb = integral(lb, B, b, tb, lb, B, b, tb)
            out[i, j] = integral(la, A, a, ta, lb, B, b, tb) / np.sqrt(na * nb)
    return out


def test_overlap_normalisation_and_symmetry():
    s = synthetic.config(0)
    rng = np.random.default_rng(5)
    atoms = synthetic.cube_atoms(rng, 4, 3.0)
    spd = synthetic.assemble("spd4", rng, atoms, True, 2.0, 1e-10)
    for x in (s, spd):
        Sm, S = oracle.overlap(x, full=True)
        assert np.abs(np.diag(S) - 1.0).max() < 1e-13
        assert np.abs(S - S.T).max() < 1e-14
        off = np.concatenate([[0], np.cumsum([synthetic.NCART[t] for t in x.l])])
        for a in range(x.nshell):
            for b in range(x.nshell):
                assert Sm[a, b] == np.abs(S[off[a]:off[a + 1], off[b]:off[b + 1]]).max()


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)])
def test_overlap_against_quadrature(la, lb):
    """Single-primitive shells at arbitrary centres: the Hermite-expansion
    overlap against Gauss-Hermite quadrature of the products."""
    A, B = [0.1, -0.3, 0.4], [0.9, 0.5, -0.2]
    a, b = 0.7, 1.9
    sys_ = custom([(la, A, [a], [1.0]), (lb, B, [b], [1.0])])
    _, S = oracle.overlap(sys_, full=True)
    na = synthetic.NCART[la]
    got = S[:na, na:]
    ref = _overlap_quadrature((la, A, a), (lb, B, b))
    assert np.abs(got - ref).max() < 1e-13, (got, ref)
    if la == lb == 0:   # closed form of two normalised s Gaussians
        R2 = np.sum((np.array(A) - np.array(B)) ** 2)
        assert abs(got[0, 0] - (2 * np.sqrt(a * b) / (a + b)) ** 1.5 * np.exp(-a * b / (a + b) * R2)) < 1e-15


def test_overlap_screen_limits(cube10):
    """tau_ovlp = 0 (or below every pair's largest overlap) is the plain
    metric query; a larger tau_ovlp keeps fewer quartets, never more."""
    s, _, _ = cube10
    tau = 1e-7
    K0, st0 = oracle.exchange(s, tau=tau)
    Sm = oracle.overlap(s)
    prev = None
    for t_ovlp in (0.0, 0.5 * Sm.min(), 1e-6, 1e-3):
        K, st = oracle.exchange_ovlp(s, t_ovlp, tau=tau)
        assert st["beta_quartets"] == st0["quartets"] and st["near_threshold"] == 0
        if t_ovlp <= Sm.min():
            assert st["quartets"] == st0["quartets"]
            assert np.abs(K - K0).max() <= 1e-14 * np.abs(K0).max()   # same quartets, another summation order
        if prev is not None:
            assert st["quartets"] <= prev
        prev = st["quartets"]
    assert prev < st0["quartets"]


@pytest.mark.parametrize("tau", [-1.0, 1e-10, 1e-8, 1e-6])
def test_symmetric_reuse_gives_the_same_K(cube10, tau):
    """Section IV: one evaluation per unique shell quartet, contracted into
    every ordered quartet it stands for that its own bound keeps, gives the
    naive K up to summation order and contracts exactly the naive quartet
    set; the integral evaluations drop to about an eighth."""
    s, Kf, stf = cube10
    Kn, stn = oracle.exchange(s, tau=tau)
    Ks, sts = oracle.exchange_sym8(s, tau=tau)
    assert np.abs(Ks - Kn).max() <= 1e-12 * max(1.0, np.abs(Kn).max())
    assert sts["quartets"] == stn["quartets"]
    assert sts["integrals"] <= sts["quartets"]
    if tau < 0:
        S = s.l.shape[0]
        M = S * (S + 1) // 2
        assert sts["integrals"] == M * (M + 1) // 2     # every canonical quartet
        assert sts["quartets"] == S ** 4
        assert sts["integrals"] * 7 < sts["quartets"]
        # nothing culled; eight distinct images iff a != b, c != d and ab != cd
        Pp = S * (S - 1) // 2
        assert sts["sparse"] == 0 and sts["full"] == Pp * (Pp - 1) // 2
    assert sts["full"] + sts["diagonal"] + sts["sparse"] == sts["integrals"]


def test_symmetric_reuse_with_a_nonsymmetric_density(cube10):
    """The images keep their own bounds, so a non-symmetric density (whose
    K is not symmetric) is handled as the naive loop handles it."""
    s, _, _ = cube10
    rng = np.random.default_rng(5)
    P = s.P + 0.1 * rng.standard_normal(s.P.shape) * np.abs(s.P)
    Kn, stn = oracle.exchange(s, P=P, tau=1e-8)
    Ks, sts = oracle.exchange_sym8(s, P=P, tau=1e-8)
    assert np.abs(Ks - Kn).max() <= 1e-12 * max(1.0, np.abs(Kn).max())
    assert sts["quartets"] == stn["quartets"]
