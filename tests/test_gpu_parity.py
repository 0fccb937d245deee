"""GPU parity: the HIP exchange build (through the C ABI) against the CPU
oracle, element by element, on seeded synthetic inputs.

Bar: FP64 path within 1e-10 max-abs of the oracle; the computed shell
quartet set identical (exact integer counts per angular-momentum class).
The only admissible count difference would come from quartets whose bound
lies within 1e-10 relative of tau (both sides evaluate the same bound
expression, the Schwarz factors from different integral algorithms); the
oracle reports how many such quartets exist, and the tests require none.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

fx = pytest.importorskip("paper_1401_6961_amd")

TOL64 = 1e-10


def say(msg):
    print(msg, flush=True)


def assert_symmetric_path_K(sys_, K):
    """Off-diagonal shell blocks are written as exact transposes; blocks of a
    shell with itself are symmetric to rounding."""
    shell = np.repeat(np.arange(sys_.nshell), [(l + 1) * (l + 2) // 2 for l in sys_.l])
    same = shell[:, None] == shell[None, :]
    assert np.array_equal(K[~same], K.T[~same])
    assert np.abs(K - K.T).max() <= 1e-13


def gpu_exchange(sys_, tau, P=None, tree=None, **opts):
    if tree is None:
        tree = fx.build_quadtree_from(sys_)
    Pt = torch.from_numpy(np.ascontiguousarray(sys_.P if P is None else P)).cuda()
    K = torch.zeros_like(Pt)
    K, st = fx.fx_exchange_ex(tree, Pt, tau, K, fx.make_opts(**opts))
    torch.cuda.synchronize()
    return K.cpu().numpy(), st, tree


def spd_cube(natom, edge, seed, tau=1e-11):
    rng = np.random.default_rng(seed)
    atoms = synthetic.cube_atoms(rng, natom, edge)
    return synthetic.assemble(f"spd{natom}", rng, atoms, True, 2.0, tau)


@pytest.fixture(scope="module")
def spd5():
    return spd_cube(5, 4.0, 31)


def test_schwarz_norms(spd5):
    say("gpu: schwarz spd5")
    tree = fx.build_quadtree_from(spd5)
    Qg = tree.schwarz()
    Qo = oracle.schwarz(spd5)
    assert np.all(np.abs(Qg - Qo) <= 1e-12 * np.maximum(Qo, 1e-300) + 1e-300)


def test_all_classes_fp64(spd5):
    """Every K block built (symmetry off): per-class quartet counts equal the
    oracle's exactly."""
    say("gpu: all 81 classes fp64, spd5 tau=1e-11, symmetry off")
    Ko, sto = oracle.exchange(spd5, tau=1e-11)
    cnt, _, near = oracle.count(spd5, tau=1e-11)
    Kg, st, _ = gpu_exchange(spd5, 1e-11, symmetry=fx.FX_SYM_OFF)
    assert near == 0
    assert st["symmetric_systems"] == 0
    assert np.array_equal(st["class_quartets"], cnt)
    assert st["quartets"] == sto["quartets"] == st["quartets_covered"]
    assert np.abs(Kg - Ko).max() <= TOL64


def test_all_classes_fp64_symmetric(spd5):
    """Symmetric density: only K blocks a <= d are built, each writing its
    transpose.  K is symmetric (exactly off the shell diagonal), matches the
    oracle, and the quartets it accounts for (evaluated + mirrored) are
    exactly the oracle's set."""
    say("gpu: all 81 classes fp64, spd5 tau=1e-11, symmetric path")
    Ko, sto = oracle.exchange(spd5, tau=1e-11)
    Kg, st, _ = gpu_exchange(spd5, 1e-11)
    assert st["symmetric_systems"] == 1
    assert st["quartets_covered"] == sto["quartets"]
    assert st["quartets"] < 0.6 * sto["quartets"]
    assert_symmetric_path_K(spd5, Kg)
    assert np.abs(Kg - Ko).max() <= TOL64


def test_nonsymmetric_density_uses_full_path(spd5):
    """A non-symmetric P is detected on the device; every block is built."""
    say("gpu: non-symmetric density")
    rng = np.random.default_rng(5)
    P = spd5.P + 0.05 * rng.standard_normal(spd5.P.shape) * (np.abs(spd5.P) > 0)
    Ko, sto = oracle.exchange(spd5, tau=1e-11, P=P)
    Kg, st, _ = gpu_exchange(spd5, 1e-11, P=P)
    assert st["symmetric_systems"] == 0
    assert st["quartets"] == sto["quartets"]
    assert np.abs(Kg - Ko).max() <= TOL64


def test_bruteforce_tau0(spd5):
    say("gpu: tau=0 vs oracle brute force")
    Ko, _ = oracle.exchange(spd5, tau=-1.0)
    Kg, st, _ = gpu_exchange(spd5, 0.0)
    assert np.abs(Kg - Ko).max() <= TOL64


def test_probe_density_slices(spd5):
    """P = e_nu e_lam^T + e_lam e_nu^T gives K_{mu sig} = (mu nu|lam sig) + (mu lam|nu sig)."""
    say("gpu: probe densities")
    n = spd5.nbf
    T = oracle.eri_tensor(spd5)
    tree = fx.build_quadtree_from(spd5)
    for nu, lam in [(0, 0), (3, 17), (20, 44), (9, 9)]:
        P = np.zeros((n, n))
        P[nu, lam] += 1.0
        P[lam, nu] += 1.0
        Kg, _, _ = gpu_exchange(spd5, 0.0, P=P, tree=tree)
        ref = T[:, nu, lam, :] + T[:, lam, nu, :]
        assert np.abs(Kg - ref).max() <= TOL64


def test_tiny_cube_config(request):
    say("gpu: 24-atom s+p cube, tau=1e-12")
    s = synthetic.config(0)
    Ko, sto = oracle.exchange(s)
    assert sto["near_threshold"] == 0
    Kg, st, _ = gpu_exchange(s, s.tau, symmetry=fx.FX_SYM_OFF)
    assert st["quartets"] == sto["quartets"]
    assert st["prim_quartets"] == sto["prim_quartets"]
    assert np.abs(Kg - Ko).max() <= TOL64
    Ks, sts, _ = gpu_exchange(s, s.tau)
    assert sts["symmetric_systems"] == 1 and sts["quartets_covered"] == sto["quartets"]
    assert np.abs(Ks - Ko).max() <= TOL64


@pytest.fixture(scope="module")
def chain():
    s = synthetic.config(1)
    Ko, sto = oracle.exchange(s)
    return s, Ko, sto


def test_chain_config(chain):
    say("gpu: 200-atom chain, tau=1e-8")
    s, Ko, sto = chain
    Kg, st, _ = gpu_exchange(s, s.tau)
    assert sto["near_threshold"] == 0
    assert st["quartets_covered"] == sto["quartets"]
    assert np.abs(Kg - Ko).max() <= TOL64
    assert_symmetric_path_K(s, Kg)
    Kf, stf, _ = gpu_exchange(s, s.tau, symmetry=fx.FX_SYM_OFF)
    assert stf["quartets"] == sto["quartets"]
    assert np.abs(Kf - Ko).max() <= TOL64
    assert np.abs(Kf - Kf.T).max() <= 1e-12


def test_chunked_traversal_is_bitwise_identical(chain):
    say("gpu: chunked traversal (frontier cap 2000)")
    s, _, _ = chain
    K1, st1, tree = gpu_exchange(s, s.tau)
    K2, st2, _ = gpu_exchange(s, s.tau, tree=tree, max_frontier_entries=2000)
    assert st2["chunks"] > 0
    assert st1["quartets"] == st2["quartets"]
    assert np.array_equal(K1, K2)


def test_rerun_is_bitwise_identical(chain):
    say("gpu: determinism")
    s, _, _ = chain
    K1, _, tree = gpu_exchange(s, s.tau)
    K2, _, _ = gpu_exchange(s, s.tau, tree=tree)
    assert np.array_equal(K1, K2)


def test_alpha_beta(spd5):
    say("gpu: alpha/beta")
    n = spd5.nbf
    Kg, _, tree = gpu_exchange(spd5, 1e-11)
    Pt = torch.from_numpy(spd5.P).cuda()
    K0 = torch.from_numpy(np.full((n, n), 2.0)).cuda()
    K, _ = fx.fx_exchange_ex(tree, Pt, 1e-11, K0, fx.make_opts(alpha=-0.5, beta=3.0))
    assert np.abs(K.cpu().numpy() - (-0.5 * Kg + 6.0)).max() <= 1e-12


def test_tree_shape_and_order_independence(spd5):
    """Reading of the leaf rule: the quartet set is {beta_q > tau} whatever
    the leaf size or shell order, so K agrees to rounding."""
    say("gpu: leaf size / ordering independence")
    Kref, st0, _ = gpu_exchange(spd5, 1e-9)
    for leaf, order in [(1, 0), (4, 0), (30, 0), (10, 1)]:
        tree = fx.build_quadtree_from(spd5, leaf_max_functions=leaf, ordering=order)
        K, st, _ = gpu_exchange(spd5, 1e-9, tree=tree)
        assert st["quartets"] == st0["quartets"]
        assert np.abs(K - Kref).max() <= 1e-13


def test_mixed_precision_tolerance(chain):
    say("gpu: mixed precision on the chain")
    s, Ko, _ = chain
    K64, st64, tree = gpu_exchange(s, s.tau)
    Km, stm, _ = gpu_exchange(s, s.tau, tree=tree, precision=fx.FX_PREC_MIXED)
    assert stm["quartets"] == st64["quartets"]
    assert stm["quartets_fp32"] > 0
    assert np.abs(Km - Ko).max() <= 1e-7


def test_mixed_precision_all_classes(spd5):
    say("gpu: mixed precision all classes")
    Ko, _ = oracle.exchange(spd5, tau=1e-11)
    Km, stm, _ = gpu_exchange(spd5, 1e-11, precision=fx.FX_PREC_MIXED)
    assert stm["quartets_fp32"] > 0
    assert np.abs(Km - Ko).max() <= 1e-7


def test_cooperative_variants(spd5):
    """The one-quartet-per-wave kernels agree with the oracle like the
    one-quartet-per-lane kernels (both precisions)."""
    say("gpu: cooperative variants, all classes that have them")
    saved = {}
    try:
        for cls in range(81):
            if fx.fx_class_variants_available(cls) & 2:
                for p in (0, 1):
                    saved[(cls, p)] = fx.fx_get_class_variant(cls, p)
                    fx.fx_set_class_variant(cls, p, 1)
        assert len(saved) > 0
        Ko, sto = oracle.exchange(spd5, tau=1e-11)
        Kg, st, _ = gpu_exchange(spd5, 1e-11)
        assert st["quartets_covered"] == sto["quartets"]
        assert np.abs(Kg - Ko).max() <= TOL64
        Km, _, _ = gpu_exchange(spd5, 1e-11, precision=fx.FX_PREC_MIXED)
        assert np.abs(Km - Ko).max() <= 1e-7
    finally:
        for (cls, p), v in saved.items():
            fx.fx_set_class_variant(cls, p, v)


def test_fp32_bound_sum(spd5):
    """Mixed precision, every K block built (no symmetry): the statistic
    fp32_beta_sum equals the sum of beta_q = (Q_ab Q_cd) ||P_bc|| (Eq. 8)
    over the quartets with tau < beta_q < fp32_threshold, in one pass and in
    two passes per class; 0 in FP64."""
    say("gpu: sum of beta over the FP32 quartets")
    tau, thr = 1e-11, 1e-5
    tree = fx.build_quadtree_from(spd5)
    Q = tree.schwarz()
    Pn = oracle.pnorm(spd5, spd5.P)
    beta = (Q[:, :, None, None] * Q[None, None, :, :]) * Pn[None, :, :, None]   # beta[a,b,c,d]
    sel = (beta > tau) & (beta < thr)
    ref = float(beta[sel].sum())
    # quartets within rounding of a threshold could go either way on the device
    near = (np.abs(beta / tau - 1) < 1e-12) | (np.abs(beta / thr - 1) < 1e-12)
    slack = float(beta[near].sum()) + 1e-12 * ref
    saved = {c: fx.fx_get_class_variant(c, 0) for c in range(81)}
    try:
        for v in (2, 0):
            for c in range(81):
                fx.fx_set_class_variant(c, 0, v)
            _, st, _ = gpu_exchange(spd5, tau, tree=tree, precision=fx.FX_PREC_MIXED, fp32_threshold=thr,
                                    symmetry=fx.FX_SYM_OFF)
            assert st["quartets_fp32"] > 0
            assert abs(st["fp32_beta_sum"] - ref) <= slack, (v, st["fp32_beta_sum"], ref)
    finally:
        for c, v in saved.items():
            fx.fx_set_class_variant(c, 0, v)
    _, st64, _ = gpu_exchange(spd5, tau, tree=tree, symmetry=fx.FX_SYM_OFF)
    assert st64["fp32_beta_sum"] == 0.0


def test_one_pass_mixed_matches_two_passes(spd5):
    """Mixed precision with both precisions in one kernel (variant 2) and in
    two kernels per class: the same quartets in each precision, K equal to
    rounding, both within the mixed tolerance of the oracle."""
    say("gpu: mixed precision, one pass vs two passes per class")
    Ko, _ = oracle.exchange(spd5, tau=1e-11)
    saved = {c: fx.fx_get_class_variant(c, 0) for c in range(81)}
    try:
        for c in range(81):
            fx.fx_set_class_variant(c, 0, 2)
        K1, st1, tree = gpu_exchange(spd5, 1e-11, precision=fx.FX_PREC_MIXED)
        for c in range(81):
            fx.fx_set_class_variant(c, 0, 0)
        K2, st2, _ = gpu_exchange(spd5, 1e-11, tree=tree, precision=fx.FX_PREC_MIXED)
    finally:
        for c, v in saved.items():
            fx.fx_set_class_variant(c, 0, v)
    assert st1["quartets"] == st2["quartets"] and st1["quartets_fp32"] == st2["quartets_fp32"] > 0
    assert np.array_equal(st1["class_prec_quartets"], st2["class_prec_quartets"])
    assert np.abs(K1 - K2).max() <= 1e-12
    assert np.abs(K1 - Ko).max() <= 1e-7 and np.abs(K2 - Ko).max() <= 1e-7


@pytest.mark.parametrize("which", ["cube24", "chain200", "chain200_chunked", "spd5_tau_large"])
def test_traversal_partition_covers_n4(which, chain):
    """Eqs. (7a-d): the level-by-level expansion visits the product of the
    four basis trees as a partition -- every task (A,B,C,D) is a surviving
    leaf task, culled, or (symmetric form) the mirror of a traversed task --
    so the sums of |A||B||C||D| over the three sets add up to n^4, with and
    without the symmetric form and with chunked levels."""
    if which == "cube24":
        s, tau, extra = synthetic.config(0), None, {}
    elif which.startswith("chain200"):
        s, tau = chain[0], None
        extra = {"max_frontier_entries": 2000} if which.endswith("chunked") else {}
    else:
        s, tau, extra = spd_cube(5, 4.0, 31), 1e-3, {}
    tau = s.tau if tau is None else tau
    n4 = s.nbf ** 4
    say(f"gpu: traversal partition {which} n={s.nbf} tau={tau}")
    for sym in (fx.FX_SYM_OFF, fx.FX_SYM_AUTO):
        _, st, _ = gpu_exchange(s, tau, symmetry=sym, **extra)
        leaf, culled, mirrored = st["partition"]
        assert leaf + culled + mirrored == n4, (sym, st["partition"], n4)
        assert leaf > 0
        if sym == fx.FX_SYM_OFF:
            assert mirrored == 0
        else:
            assert st["symmetric_systems"] == 1 and mirrored > 0
        if extra:
            assert st["chunks"] > 0


@pytest.mark.parametrize("which,leaf", [("cube24", 4), ("cube24", 10), ("spd5", 10)])
def test_leaf_block_mode_matches_oracle(which, leaf):
    """leaf_screen BLOCK (the paper's rule: whole leaf blocks of a kept leaf
    task are computed) against the oracle's own bisection and leaf test, in
    caller shell order, with and without the symmetric form."""
    s = synthetic.config(0) if which == "cube24" else spd_cube(5, 4.0, 31)
    tau = 1e-6
    say(f"gpu: leaf-block mode {which} leaf={leaf} tau={tau}")
    Ko, sto = oracle.exchange_leafblock(s, leaf, tau=tau)
    assert sto["near_threshold"] == 0
    Ks, sts = oracle.exchange(s, tau=tau)
    assert sto["quartets"] > sts["quartets"]          # the rule computes more than the shell-level one
    tree = fx.build_quadtree_from(s, leaf_max_functions=leaf, ordering=1)
    for sym in (fx.FX_SYM_OFF, fx.FX_SYM_AUTO):
        Kg, st, _ = gpu_exchange(s, tau, tree=tree, leaf_screen=fx.FX_LEAF_BLOCK, symmetry=sym)
        assert st["quartets_covered"] == sto["quartets"], (sym, st["quartets_covered"], sto["quartets"])
        assert np.abs(Kg - Ko).max() <= TOL64


def test_overlap_table_matches_oracle(spd5):
    """Largest |overlap| per shell pair (Obara-Saika on the GPU, Hermite
    expansion in the oracle)."""
    say("gpu: overlap table spd5")
    tree = fx.build_quadtree_from(spd5)
    Sg = tree.overlap()
    So = oracle.overlap(spd5)
    assert np.all(np.abs(Sg - So) <= 1e-13 * So + 1e-14)   # normalised functions: |S| <= 1


@pytest.mark.parametrize("which,tau_ovlp", [("cube24", 1e-6), ("cube24", 1e-3), ("spd5", 1e-4)])
def test_overlap_criterion_matches_oracle(which, tau_ovlp):
    """The metric query plus the overlap criterion of Eqs. (3)-(4): quartets
    whose bra or ket shell pair overlaps less than tau_ovlp everywhere are
    dropped, in the traversal (block maxima) and in the class kernels."""
    s = synthetic.config(0) if which == "cube24" else spd_cube(5, 4.0, 31)
    tau = 1e-8
    say(f"gpu: overlap criterion {which} tau={tau} tau_ovlp={tau_ovlp}")
    Ko, sto = oracle.exchange_ovlp(s, tau_ovlp, tau=tau)
    assert sto["near_threshold"] == 0 and sto["quartets"] < sto["beta_quartets"]
    for sym in (fx.FX_SYM_OFF, fx.FX_SYM_AUTO):
        Kg, st, _ = gpu_exchange(s, tau, symmetry=sym, tau_ovlp=tau_ovlp)
        assert st["quartets_covered"] == sto["quartets"], (sym, st["quartets_covered"], sto["quartets"])
        assert np.abs(Kg - Ko).max() <= TOL64
