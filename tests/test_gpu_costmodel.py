"""GPU cost model: the hand-written FP32 forward/backward kernels against the
FP64 reference, training on the GPU, timing probes, and scheduling that
never changes K."""
import os

import numpy as np
import pytest

import synthetic
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
fx = pytest.importorskip("paper_1401_6961_amd")


def say(msg):
    print(msg, flush=True)


def rand_model(seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPARAM).astype(np.float32)
    norm = np.array([1.0, -2.0, 0.5, 3.0, 2.0, 0.7, 1.5, 0.9, 10.0, 3.0], np.float32)
    f = (rng.normal(0, 2, (3000, 4)) + norm[:4]).astype(np.float32)
    t = rng.normal(10, 3, 3000).astype(np.float32)
    return p, norm, f, t


def test_forward_matches_reference():
    say("gpu: costmodel forward")
    p, norm, f, _ = rand_model()
    m = fx.CostModel.create(p, norm)
    got = m.predict(f)
    ref = mlp.predict(p.astype(np.float64), norm.astype(np.float64), f.astype(np.float64))
    assert np.abs(got - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


def test_gradient_matches_reference():
    say("gpu: costmodel gradient")
    p, norm, f, t = rand_model(1)
    m = fx.CostModel.create(p, norm)
    loss, g = m.loss_grad(f, t)
    lref, gref = mlp.loss_grad(p.astype(np.float64), norm.astype(np.float64), f.astype(np.float64),
                               t.astype(np.float64))
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    assert np.linalg.norm(g - gref) <= 1e-3 * np.linalg.norm(gref)


def test_training_fits_a_smooth_target():
    say("gpu: costmodel training")
    rng = np.random.default_rng(7)
    f = rng.uniform([8, 0, -6, 0], [14, 3, 0, 10], (20000, 4)).astype(np.float32)
    t = (f[:, 0] + f[:, 1] + 0.6 * f[:, 3] + 0.2 * np.maximum(f[:, 2] + 3, 0) ** 2).astype(np.float32)
    data = fx.TaskTimings.from_arrays(f, t)
    m, loss = fx.fx_costmodel_train(data, steps=800, batch=4096, lr=3e-3, seed=3)
    assert loss < 0.02, loss          # mean squared error on standardised targets
    w, norm = m.params()
    pred = m.predict(f[:500])
    assert np.abs(pred - mlp.predict(w.astype(np.float64), norm.astype(np.float64), f[:500])).max() < 1e-3


@pytest.fixture(scope="module")
def recorded():
    say("gpu: recording unit timings (60-atom s+p+d cluster)")
    s = synthetic.cluster(60, seed=2024)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    rec = fx.fx_record_task_timings(tree, P, s.tau, fx.make_opts(precision=fx.FX_PREC_MIXED))
    return s, tree, P, rec


def test_timing_probes(recorded):
    s, tree, P, rec = recorded
    f, t, c = rec.arrays()
    assert len(t) > 1000
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(t))
    assert t.min() >= 0 and t.max() < 40       # log2 ns
    assert set(np.unique(c // 2)).issubset(set(range(81)))


def test_schedules_give_bitwise_identical_K(recorded):
    s, tree, P, rec = recorded
    say("gpu: K under NONE / BOUND / MLP schedules")
    m, _ = fx.fx_costmodel_train(rec, steps=300, batch=4096)
    Ks = []
    for sched, cm in ((fx.FX_SCHED_NONE, None), (fx.FX_SCHED_BOUND, None), (fx.FX_SCHED_MLP, m)):
        K = torch.zeros_like(P)
        K, st = fx.fx_exchange_ex(tree, P, s.tau, K, fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=sched,
                                                                    costmodel=cm))
        Ks.append(K.cpu().numpy())
    assert np.array_equal(Ks[0], Ks[1]) and np.array_equal(Ks[0], Ks[2])


def _r2(pred, y):
    return 1.0 - np.mean((pred - y) ** 2) / np.var(y)


def test_learned_model_predicts_unit_time_better_than_bound_only(recorded):
    """Ablation of the learned part: on a held-out system the MLP's predicted
    unit times explain the measured ones better than the bound-only estimate
    does, even with that estimate given the benefit of an optimal affine fit."""
    s, tree, P, rec = recorded
    say("gpu: learned vs bound-only prediction on a held-out system")
    m, _ = fx.fx_costmodel_train(rec, steps=1500, batch=8192)
    s2 = synthetic.cluster(80, seed=77)
    tree2 = fx.build_quadtree_from(s2)
    P2 = torch.from_numpy(s2.P).cuda()
    f2, t2, _ = fx.fx_record_task_timings(tree2, P2, s2.tau, fx.make_opts(precision=fx.FX_PREC_MIXED)).arrays()
    r2_mlp = _r2(m.predict(f2), t2)
    f1, t1, _ = rec.arrays()
    b1 = f1[:, 0] + f1[:, 1] + f1[:, 3]
    A = np.vstack([b1, np.ones_like(b1)]).T
    coef = np.linalg.lstsq(A, t1, rcond=None)[0]
    r2_bound = _r2(coef[0] * (f2[:, 0] + f2[:, 1] + f2[:, 3]) + coef[1], t2)
    say(f"R^2 held-out: mlp {r2_mlp:.3f}  bound-only {r2_bound:.3f}")
    assert r2_mlp > r2_bound


@pytest.mark.xfail(strict=False, reason="the learned unit order does not yet beat the bound-only order: "
                   "4000-atom s+p slab, 5 alternating runs each, 20.52 s learned vs 20.31 s bound-only; "
                   "1000-atom s+p+d cluster, 14.74 s vs 14.68 s (K bitwise equal); with one unit per "
                   "workgroup the order inside a launch has little leverage")
def test_learned_order_builds_no_slower_than_bound_only():
    """The shipped model's unit order against the bound-only order on a
    250-atom s+p+d cluster, 5 alternating runs each: same K bitwise, and the
    learned order's median no slower."""
    import time
    model = fx.CostModel.load(os.path.join(os.path.dirname(fx.__file__), "costmodel_gfx950.fxmlp"))
    s = synthetic.cluster(250, seed=2250)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    say("gpu: learned vs bound-only unit order, 250-atom cluster, 5 alternating runs")
    opts = {"bound": fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=fx.FX_SCHED_BOUND, use_graph=True),
            "mlp": fx.make_opts(precision=fx.FX_PREC_MIXED, schedule=fx.FX_SCHED_MLP, costmodel=model,
                                use_graph=True)}
    Ks = {k: torch.zeros_like(P) for k in opts}
    for k, o in opts.items():
        fx.fx_exchange_ex(tree, P, s.tau, Ks[k], o, stats=False)
    torch.cuda.synchronize()
    times = {k: [] for k in opts}
    for r in range(5):
        for k in (("bound", "mlp") if r % 2 == 0 else ("mlp", "bound")):
            t0 = time.perf_counter()
            fx.fx_exchange_ex(tree, P, s.tau, Ks[k], opts[k], stats=False)
            torch.cuda.synchronize()
            times[k].append(time.perf_counter() - t0)
    assert torch.equal(Ks["bound"], Ks["mlp"])
    med = {k: float(np.median(v)) for k, v in times.items()}
    say(f"median: learned {med['mlp']:.4f} s, bound-only {med['bound']:.4f} s")
    assert med["mlp"] <= med["bound"]


def test_costmodel_save_load_roundtrip(tmp_path):
    say("gpu: costmodel save/load")
    p, norm, f, _ = rand_model(5)
    m = fx.CostModel.create(p, norm)
    path = tmp_path / "m.fxmlp"
    m.save(str(path))
    m2 = fx.CostModel.load(str(path))
    w2, n2 = m2.params()
    assert np.array_equal(w2, p) and np.array_equal(n2, norm)
    assert np.array_equal(m2.predict(f), m.predict(f))
