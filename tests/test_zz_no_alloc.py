"""The allocation-free entry point (fx_exchange_noalloc): its K equals
fx_exchange_ex's bitwise on two calls in a row, the second with a smaller
system (the scratch array keeps the first call's contents), and a system
whose fixed buffers exceed the array is refused before any work."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
fx = pytest.importorskip("paper_1401_6961_amd")


def say(msg):
    print(msg, flush=True)


def _pair(s, **kw):
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    ref, st_ref = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(**kw))
    K = torch.full_like(P, 3.0)
    K, st = fx.fx_exchange_noalloc(tree, P, s.tau, K, fx.make_opts(**kw))
    torch.cuda.synchronize()
    return ref, st_ref, K, st


def test_noalloc_equals_allocating_entry_point_twice():
    big = synthetic.chain(200)
    rng = np.random.default_rng(31)
    small = synthetic.assemble("spd5", rng, synthetic.cube_atoms(rng, 5, 4.0), True, 2.0, 1e-11)
    assert small.nbf < big.nbf
    for s, prec in ((big, fx.FX_PREC_FP64), (small, fx.FX_PREC_MIXED)):
        say(f"gpu: no-alloc entry point, n={s.nbf}, precision {prec}")
        ref, st_ref, K, st = _pair(s, precision=prec)
        assert st["quartets"] == st_ref["quartets"] and st["quartets_covered"] == st_ref["quartets_covered"]
        assert torch.equal(K, ref)
        assert 0 < st["workspace_bytes"] <= fx.lib().fx_noalloc_scratch_bytes()


def test_noalloc_rejects_what_does_not_fit():
    """A 1000-atom s+p+d cluster needs far more than the scratch array
    (density norms alone: 72 MB, unit lists 108 MB, beta != 0 adds 800 MB)."""
    s = synthetic.cluster(1000, density=False)
    tree = fx.build_quadtree_from(s)
    n = s.nbf
    P = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    K = torch.zeros_like(P)
    say("gpu: no-alloc entry point refuses an oversized call")
    with pytest.raises(fx.FxError) as e:
        fx.fx_exchange_noalloc(tree, P, 1e-8, K, fx.make_opts(beta=1.0))
    assert "scratch" in str(e.value)
