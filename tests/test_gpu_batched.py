"""Batched launches, graph capture and launch options: every system's K from
one batched call equals its own single-system build bitwise (the K-block
reductions do not depend on how units are grouped into launches)."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
fx = pytest.importorskip("paper_1401_6961_amd")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def systems():
    say("gpu: building 6 small clusters (s+p and s+p+d mixed)")
    out = []
    for i, (n, d) in enumerate([(12, False), (30, True), (8, False), (20, True), (45, False), (16, True)]):
        s = synthetic.cluster(n, seed=500 + i, with_d=d)
        tree = fx.build_quadtree_from(s)
        out.append((s, tree, torch.from_numpy(s.P).cuda()))
    return out


def single(tree, s, P, **kw):
    K = torch.zeros_like(P)
    K, st = fx.fx_exchange_ex(tree, P, s.tau, K, fx.make_opts(**kw))
    return K.cpu().numpy(), st


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_equals_single_bitwise(systems, prec):
    say(f"gpu: batched vs single, precision {prec}")
    refs = [single(t, s, P, precision=prec) for s, t, P in systems]
    Ks = [torch.zeros_like(P) for _, _, P in systems]
    Ks, st = fx.fx_exchange_batched([t for _, t, _ in systems], [P for _, _, P in systems], Ks, 1e-8,
                                    fx.make_opts(precision=prec))
    assert st["quartets"] == sum(r[1]["quartets"] for r in refs)
    for K, (Kr, _) in zip(Ks, refs):
        assert np.array_equal(K.cpu().numpy(), Kr)


def test_graph_capture_equals_eager(systems):
    say("gpu: graph-captured class launches")
    Ps = [P for _, _, P in systems]
    trees = [t for _, t, _ in systems]
    K1 = [torch.zeros_like(P) for P in Ps]
    K1, _ = fx.fx_exchange_batched(trees, Ps, K1, 1e-8, fx.make_opts(precision=1))
    for rep in range(3):
        K2 = [torch.zeros_like(P) for P in Ps]
        K2, st = fx.fx_exchange_batched(trees, Ps, K2, 1e-8, fx.make_opts(precision=1, use_graph=True))
        assert st["graph_nodes"] == 1
        torch.cuda.synchronize()
        for a, b in zip(K1, K2):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    s, t, P = systems[1]
    Kg, stg = single(t, s, P, precision=1, use_graph=True)
    Ke, _ = single(t, s, P, precision=1)
    assert stg["graph_nodes"] == 1 and np.array_equal(Kg, Ke)


@pytest.mark.skip(reason="persistent class launches are switched off: a GPU run of the persistent-grid "
                         "path went silent for 180 s and was killed; no cause was found by reading the code")
def test_persistent_launches():
    pass


def test_xcd_remap_does_not_change_K(systems):
    say("gpu: XCD-aware workgroup remap")
    s, t, P = systems[3]
    Kref, _ = single(t, s, P, precision=1)
    saved = {(c, p): fx.fx_get_class_launch(c, p) for c in range(81) for p in (0, 1)}
    try:
        for flags in (1,):
            for c in range(81):
                for p in (0, 1):
                    fx.fx_set_class_launch(c, p, flags)
            K, _ = single(t, s, P, precision=1)
            assert np.array_equal(K, Kref), flags
    finally:
        for (c, p), v in saved.items():
            fx.fx_set_class_launch(c, p, v)
