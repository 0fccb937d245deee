"""Several densities contracted with the same integrals (fx_exchange_multi):
each K[j] against the oracle, built block by block with the screening norm
the library uses (the largest density-block norm over the densities)."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
fx = pytest.importorskip("paper_1401_6961_amd")

NCART = (1, 3, 6)
TOL64 = 1e-10


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def spd6():
    rng = np.random.default_rng(61)
    atoms = synthetic.cube_atoms(rng, 6, 4.5)
    s = synthetic.assemble("spd6", rng, atoms, True, 2.0, 1e-9)
    P2 = synthetic.make_density(np.random.default_rng(62), s.atoms, s.func_atom(), 1.5)
    return s, P2, fx.build_quadtree_from(s)


def oracle_full(s, P, Pn, tau):
    """K over every shell block (a, d), screened with the given Pn."""
    S = s.nshell
    pairs = np.array([(a, d) for a in range(S) for d in range(S)], np.int32)
    blocks, st = oracle.exchange_blocks(s, pairs, P=P, tau=tau, Pn=Pn)
    off = np.concatenate([[0], np.cumsum([NCART[x] for x in s.l])])
    K = np.zeros((s.nbf, s.nbf))
    for (a, d), b in zip(pairs, blocks):
        K[off[a]:off[a + 1], off[d]:off[d + 1]] = b
    return K, st


def multi(tree, Ps, tau, **kw):
    Pt = [torch.from_numpy(np.ascontiguousarray(P)).cuda() for P in Ps]
    Ks = [torch.zeros_like(P) for P in Pt]
    Ks, st = fx.fx_exchange_multi(tree, Pt, Ks, tau, fx.make_opts(**kw))
    torch.cuda.synchronize()
    return [K.cpu().numpy() for K in Ks], st


@pytest.mark.parametrize("prec", [0, 1])
def test_equal_densities_equal_single_build(spd6, prec):
    """Two copies of one density: both K equal the one-density build, bitwise
    in FP64; in mixed precision to rounding (the one-density build may run
    both precisions in one pass, which sums in another order)."""
    s, _, tree = spd6
    say(f"gpu multi: equal densities, precision {prec}")
    (K1, K2), st = multi(tree, [s.P, s.P], s.tau, precision=prec)
    Pt = torch.from_numpy(s.P).cuda()
    K, st1 = fx.fx_exchange_ex(tree, Pt, s.tau, torch.zeros_like(Pt), fx.make_opts(precision=prec))
    K = K.cpu().numpy()
    assert st["quartets"] == st1["quartets"] and st["quartets_fp32"] == st1["quartets_fp32"]
    assert np.array_equal(K1, K2)
    if prec == 0:
        assert np.array_equal(K1, K)
    else:
        assert np.abs(K1 - K).max() <= 1e-13 * max(1.0, np.abs(K).max())


@pytest.mark.parametrize("symmetric", [True, False])
def test_two_densities_match_oracle(spd6, symmetric):
    s, P2, tree = spd6
    if not symmetric:
        P2 = P2 + 0.05 * np.triu(np.random.default_rng(63).standard_normal(P2.shape), 1)
    say(f"gpu multi: two densities, symmetric={symmetric}")
    Pn = np.maximum(oracle.pnorm(s, s.P), oracle.pnorm(s, P2))
    refs = [oracle_full(s, P, Pn, s.tau) for P in (s.P, P2)]
    (K1, K2), st = multi(tree, [s.P, P2], s.tau)
    assert st["symmetric_systems"] == (1 if symmetric else 0)
    assert st["quartets_covered"] == refs[0][1]["quartets"]
    assert np.abs(K1 - refs[0][0]).max() <= TOL64
    assert np.abs(K2 - refs[1][0]).max() <= TOL64
    (M1, M2), _ = multi(tree, [s.P, P2], s.tau, precision=fx.FX_PREC_MIXED)
    assert np.abs(M1 - refs[0][0]).max() <= 1e-7
    assert np.abs(M2 - refs[1][0]).max() <= 1e-7


def test_cooperative_variant_falls_back(spd6):
    """The one-quartet-per-wave kernels contract one density; with two the
    library runs the one-quartet-per-lane kernels instead."""
    s, P2, tree = spd6
    say("gpu multi: cooperative variants selected")
    saved = {}
    try:
        for cls in range(81):
            if fx.fx_class_variants_available(cls) & 2:
                for p in (0, 1):
                    saved[(cls, p)] = fx.fx_get_class_variant(cls, p)
                    fx.fx_set_class_variant(cls, p, 1)
        (K1, K2), _ = multi(tree, [s.P, P2], s.tau)
    finally:
        for (cls, p), v in saved.items():
            fx.fx_set_class_variant(cls, p, v)
    (R1, R2), _ = multi(tree, [s.P, P2], s.tau)
    assert np.array_equal(K1, R1) and np.array_equal(K2, R2)


def test_rejects_bad_arguments(spd6):
    s, P2, tree = spd6
    say("gpu multi: argument checks")
    Pt = torch.from_numpy(s.P).cuda()
    with pytest.raises(fx.FxError, match="UNSUPPORTED"):
        fx.fx_exchange_multi(tree, [Pt, Pt, Pt], [torch.zeros_like(Pt) for _ in range(3)], s.tau)
    K = torch.zeros_like(Pt)
    with pytest.raises(fx.FxError, match="INVALID"):
        fx.fx_exchange_multi(tree, [Pt, Pt], [K, K], s.tau)
