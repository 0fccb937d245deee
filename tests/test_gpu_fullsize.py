"""Parity at full workload sizes, in the launch configurations the benchmark
times, on sampled K blocks.

The oracle cannot build K for thousands of atoms in seconds, but it builds
any single block K_{a d} (all functions of shells a and d) directly from
the definition with the same screening test (Eq. 6 restricted to the quartets
whose bound of Eq. 8 exceeds tau).  Each test builds the whole K on the GPU
and compares seeded samples of blocks element by element:

* near blocks: a and d on the same atom or on one of its nearest atoms,
  where K is largest and the most quartets survive;
* every (l_a, l_d) combination present;
* random blocks (mostly small or screened to zero).

Bars: FP64 path 1e-10 max-abs, mixed path 1e-7 max-abs.  These tests take
minutes; they are marked slow as well as gpu.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]
fx = pytest.importorskip("paper_1401_6961_amd")

NCART = (1, 3, 6)


def say(msg):
    print(msg, flush=True)


def sample_pairs(s, n_near, n_rand, seed):
    rng = np.random.default_rng(seed)
    S = s.nshell
    atom_xyz = np.array([s.center[np.flatnonzero(s.shell_atom == i)[0]] for i in range(s.shell_atom.max() + 1)])
    shells_of = [np.flatnonzero(s.shell_atom == i) for i in range(len(atom_xyz))]
    pairs = []
    for _ in range(n_near):
        i = int(rng.integers(len(atom_xyz)))
        d2 = ((atom_xyz - atom_xyz[i]) ** 2).sum(1)
        j = int(np.argsort(d2)[rng.integers(0, 4)])
        pairs.append((int(rng.choice(shells_of[i])), int(rng.choice(shells_of[j]))))
    for la in sorted(set(s.l.tolist())):
        for ld in sorted(set(s.l.tolist())):
            i = int(rng.integers(len(atom_xyz)))
            a = [x for x in shells_of[i] if s.l[x] == la]
            j = int(np.argsort(((atom_xyz - atom_xyz[i]) ** 2).sum(1))[1])
            d = [x for x in shells_of[j] if s.l[x] == ld]
            if a and d:
                pairs.append((int(a[0]), int(d[0])))
    pairs += [tuple(int(x) for x in rng.integers(0, S, 2)) for _ in range(n_rand)]
    return np.array(pairs, np.int32)


def compare_blocks(s, K, pairs, Kref_blocks, tol):
    off = np.concatenate([[0], np.cumsum([NCART[x] for x in s.l])])
    worst, nonzero = 0.0, 0
    for (a, d), blk in zip(pairs, Kref_blocks):
        g = K[off[a]:off[a + 1], off[d]:off[d + 1]]
        worst = max(worst, float(np.abs(g - blk).max()))
        nonzero += int(np.abs(blk).max() > 1e-6)
    assert worst <= tol, worst
    return worst, nonzero


def oracle_blocks(s, pairs, Qn, Pn):
    blocks, st = oracle.exchange_blocks(s, pairs, Qn=Qn, Pn=Pn)
    assert st["near_threshold"] == 0
    return blocks


@pytest.fixture(scope="module")
def cluster():
    """1000-atom s+p+d cluster, tau=1e-8, its tree and the oracle's blocks."""
    say("gpu fullsize: 1000-atom s+p+d cluster, generating")
    s = synthetic.config(2)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    pairs = sample_pairs(s, 28, 12, seed=7)
    say("gpu fullsize: cluster oracle blocks")
    ref = oracle_blocks(s, pairs, oracle.schwarz(s), oracle.pnorm(s, s.P))
    return s, tree, P, pairs, ref


@pytest.mark.timeout(600)
def test_cluster_1000_spd_mixed(cluster):
    """Mixed build with the tuned kernel table, as benchmarked."""
    from paper_1401_6961_amd import autotune
    s, tree, P, pairs, ref = cluster
    n_tuned = autotune.apply()
    say(f"gpu fullsize: cluster mixed build ({n_tuned} tuned entries)")
    K, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_MIXED))
    torch.cuda.synchronize()
    assert st["quartets_fp32"] > 0
    w, nz = compare_blocks(s, K.cpu().numpy(), pairs, ref, 1e-7)
    say(f"gpu fullsize: cluster mixed max err {w:.2e} over {len(pairs)} blocks ({nz} non-negligible)")
    assert nz >= 20


@pytest.mark.timeout(600)
def test_cluster_1000_spd_fp64(cluster):
    s, tree, P, pairs, ref = cluster
    say("gpu fullsize: cluster FP64 build")
    K, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_FP64))
    torch.cuda.synchronize()
    K = K.cpu().numpy()
    w, nz = compare_blocks(s, K, pairs, ref, 1e-10)
    say(f"gpu fullsize: cluster FP64 max err {w:.2e} over {len(pairs)} blocks ({nz} non-negligible)")
    assert np.abs(K - K.T).max() <= 1e-12


@pytest.mark.timeout(600)
def test_batched_64_clusters_graph():
    """64 s+p clusters (50..500 atoms) in one batched, graph-captured mixed
    call, as benchmarked; blocks of four systems against the oracle."""
    say("gpu fullsize: 64 batched clusters, generating")
    systems = synthetic.config(3)
    trees = [fx.build_quadtree_from(x) for x in systems]
    Ps = [torch.from_numpy(x.P).cuda() for x in systems]
    Ks = [torch.zeros_like(P) for P in Ps]
    say("gpu fullsize: batched graph-captured build")
    Ks, st = fx.fx_exchange_batched(trees, Ps, Ks, systems[0].tau,
                                    fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=True))
    torch.cuda.synchronize()
    assert st["graph_nodes"] == 1
    sizes = np.array([x.nbf for x in systems])
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 5, 40})
    for i in picks:
        x = systems[i]
        pairs = sample_pairs(x, 10, 4, seed=100 + i)
        ref = oracle_blocks(x, pairs, oracle.schwarz(x), oracle.pnorm(x, x.P))
        w, nz = compare_blocks(x, Ks[i].cpu().numpy(), pairs, ref, 1e-7)
        say(f"gpu fullsize: system {i} (n={x.nbf}) max err {w:.2e} over {nz} non-negligible blocks")


@pytest.fixture(scope="module")
def slab():
    """4000-atom s+p slab and the oracle's blocks."""
    say("gpu fullsize: 4000-atom s+p slab, generating")
    s = synthetic.config(4)
    pairs = sample_pairs(s, 24, 8, seed=11)
    say("gpu fullsize: slab oracle blocks")
    ref = oracle_blocks(s, pairs, oracle.schwarz(s), oracle.pnorm(s, s.P))
    return s, pairs, ref


@pytest.mark.timeout(600)
def test_slab_oracle_blocks_are_informative(slab):
    s, pairs, ref = slab
    assert sum(int(np.abs(b).max() > 1e-6) for b in ref) >= 16


@pytest.mark.timeout(600)
def test_slab_4000_sp_mlp_schedule(slab):
    """Mixed build with a (seeded, untrained) MLP ordering the units:
    ordering never changes which quartets are computed or K."""
    s, pairs, ref = slab
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    rng = np.random.default_rng(3)
    w = (0.2 * rng.standard_normal(fx.lib().fx_costmodel_nparams())).astype(np.float32)
    norm = np.array([10, 2, -8, 6, 3, 1, 3, 2, 10, 2], np.float32)
    model = fx.CostModel.create(w, norm)
    say("gpu fullsize: slab mixed build, MLP schedule")
    K, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P),
                              fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=fx.FX_SCHED_MLP, costmodel=model))
    torch.cuda.synchronize()
    w_, nz = compare_blocks(s, K.cpu().numpy(), pairs, ref, 1e-7)
    say(f"gpu fullsize: slab max err {w_:.2e} over {len(pairs)} blocks ({nz} non-negligible)")


def _exact_counts(s, name):
    """Symmetry off: every ordered quartet is evaluated by its own class
    kernel, so the per-class counts and the primitive-quartet total equal the
    oracle's exhaustive count, up to the quartets whose bound lies within
    1e-10 relative of tau (the only ones whose test can flip between the
    two sides, whose Schwarz factors come from different integral
    algorithms; the oracle counts them)."""
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    say(f"gpu fullsize: {name} counts, GPU build with symmetry off")
    _, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P),
                              fx.make_opts(precision=fx.FX_PREC_MIXED, symmetry=fx.FX_SYM_OFF))
    torch.cuda.synchronize()
    say(f"gpu fullsize: {name} counts, oracle")
    cnt, prim, near = oracle.count(s)
    say(f"gpu fullsize: {name} {int(cnt.sum())} quartets, {near} near tau; GPU {st['quartets']}")
    assert near <= 1e-9 * cnt.sum()
    assert np.abs(st["class_quartets"] - cnt).sum() <= near
    assert st["quartets"] == st["quartets_covered"]
    assert abs(st["quartets"] - int(cnt.sum())) <= near
    assert abs(st["prim_quartets"] - prim) <= near * 16 ** 4
    n4 = s.nbf ** 4
    assert sum(st["partition"]) == n4 and st["partition"][2] == 0


@pytest.mark.timeout(900)
def test_cluster_1000_exact_quartet_counts(cluster):
    _exact_counts(cluster[0], "cluster")


@pytest.mark.timeout(900)
def test_slab_4000_exact_quartet_counts(slab):
    _exact_counts(slab[0], "slab")
