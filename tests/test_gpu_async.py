"""Asynchronous calls, whole-call graph capture and replay, and buffer
capacities (the traversal of Eqs. 7a-d keeps every size on the device)."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
fx = pytest.importorskip("paper_1401_6961_amd")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def mid():
    """250-atom s+p+d cluster (about a second per build) and its reference K."""
    s = synthetic.cluster(250, seed=2250)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    Kref, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_MIXED))
    torch.cuda.synchronize()
    return s, tree, P, Kref.clone(), st


def test_call_returns_before_K_is_complete(mid):
    s, tree, P, Kref, st = mid
    say("gpu: asynchronous call")
    K = torch.full_like(P, 7.0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    fx.fx_exchange_ex(tree, P, s.tau, K, fx.make_opts(precision=fx.FX_PREC_MIXED), stats=False)
    pending = not stream.query()
    torch.cuda.synchronize()
    assert pending, "the call waited for its work"
    assert torch.equal(K, Kref)


def test_plain_fx_exchange_is_asynchronous_and_exact(mid):
    s, tree, P, _, _ = mid
    say("gpu: fx_exchange (FP64 defaults)")
    K64, _ = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P))
    K = torch.zeros_like(P)
    fx.fx_exchange(tree, P, s.tau, K)
    torch.cuda.synchronize()
    assert torch.equal(K, K64)


def test_graph_replays_equal_eager(mid):
    """The whole call (norms, traversal, units, class kernels, scaling)
    captured once and replayed: every replay equals the eager result
    bitwise, with eager work and synchronisations between replays."""
    s, tree, P, Kref, _ = mid
    say("gpu: graph capture and replays")
    opts = fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=True)
    K = torch.zeros_like(P)
    for i in range(4):
        K.fill_(float(i + 1))
        fx.fx_exchange_ex(tree, P, s.tau, K, opts, stats=False)
        torch.cuda.synchronize()
        assert torch.equal(K, Kref), f"replay {i}"
        # eager work of the program between replays
        Ke, _ = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_MIXED))
        torch.cuda.synchronize()
        assert torch.equal(Ke, Kref)
    # with statistics the replay is also checked for capacity on the host
    K2, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), opts)
    assert st["graph_nodes"] == 1 and st["overflow"] == 0
    assert torch.equal(K2, Kref)


def test_overflow_without_waiting_gives_nan_and_waiting_splits(mid):
    """A capacity too small for the traversal: a call that does not wait
    writes NaN (never a silently wrong K); a call that waits splits its K
    rows and returns the exact K."""
    s, tree, P, Kref, st0 = mid
    cap = max(st0["frontier"]) // 4      # a quarter of the largest level: row ranges must split
    say(f"gpu: capacity overflow (asynchronous and waiting), cap {cap} of {max(st0['frontier'])}")
    small = fx.make_opts(precision=fx.FX_PREC_MIXED, max_frontier_entries=cap)
    K = torch.zeros_like(P)
    fx.fx_exchange_ex(tree, P, s.tau, K, small, stats=False)
    torch.cuda.synchronize()
    assert torch.isnan(K).all()
    K2, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), small)
    assert st["chunks"] > 0 and st["overflow"] == 1      # split after an overflow; K complete
    assert torch.equal(K2, Kref)
    assert st["quartets"] == st0["quartets"]


def test_workspace_budget_runs_row_ranges(mid):
    """A workspace budget below what one pass needs: the traversal runs over
    K row ranges (cut where the leaf entries of the first call balance, each
    range's sizes measured once), the workspace stays within the budget, and
    K is bitwise the same, eager and replayed."""
    s, tree, P, Kref, st0 = mid
    budget = st0["workspace_bytes"] // 4
    say(f"gpu: workspace budget {budget} of {st0['workspace_bytes']} bytes")
    opts = fx.make_opts(precision=fx.FX_PREC_MIXED, max_workspace_bytes=budget)
    K, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), opts)
    assert st["chunks"] > st0["chunks"] and st["overflow"] == 0
    assert st["workspace_bytes"] <= budget
    assert torch.equal(K, Kref) and st["quartets"] == st0["quartets"]
    g = fx.make_opts(precision=fx.FX_PREC_MIXED, max_workspace_bytes=budget, use_graph=True)
    for i in range(2):
        K.fill_(float(i + 1))
        fx.fx_exchange_ex(tree, P, s.tau, K, g, stats=False)
        torch.cuda.synchronize()
        assert torch.equal(K, Kref), f"replay {i}"


def test_progress_reports_each_row_range(mid, capfd):
    """The progress hook: one line per K row range of an eager call, from the
    library's own callback on the runtime thread."""
    s, tree, P, Kref, st0 = mid
    say("gpu: progress lines per row range")
    budget = st0["workspace_bytes"] // 4
    opts = fx.make_opts(precision=fx.FX_PREC_MIXED, max_workspace_bytes=budget)
    capfd.readouterr()
    fx.set_progress_stderr("probe")
    try:
        K, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), opts)
        torch.cuda.synchronize()
    finally:
        fx.set_progress_stderr(None)
    lines = [x for x in capfd.readouterr().err.splitlines() if x.startswith("probe: K row range")]
    n = st["chunks"] + 1
    assert n > 1 and len(lines) == n
    assert lines[-1] == f"probe: K row range {n} of {n} done"
    assert torch.equal(K, Kref)


def test_group_screen_gives_the_same_K(mid):
    """One shared screen per (l_a, l_d) group against a screen in every class
    kernel (the default): the same quartets in the same order, so K is
    bitwise the same (mixed and FP64, eager and replayed)."""
    s, tree, P, Kref, st0 = mid
    say("gpu: shared group screen on / off")
    assert not fx.get_group_screen()
    K64, st64 = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P))
    fx.set_group_screen(True)
    try:
        Kon, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_MIXED))
        K64on, st64on = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P))
        Kg = torch.zeros_like(P)
        fx.fx_exchange_ex(tree, P, s.tau, Kg, fx.make_opts(precision=fx.FX_PREC_MIXED, use_graph=True), stats=False)
        torch.cuda.synchronize()
    finally:
        fx.set_group_screen(False)
    assert torch.equal(Kon, Kref) and torch.equal(Kg, Kref) and torch.equal(K64on, K64)
    assert np.array_equal(st["class_prec_quartets"], st0["class_prec_quartets"])
    assert st64on["quartets"] == st64["quartets"]


def test_first_call_learns_capacities():
    """A fresh tree: the first call sizes its buffers by a traversal-only
    pass; later calls need no more than 25% above the sizes seen."""
    s = synthetic.chain(200)
    tree = fx.build_quadtree_from(s)
    P = torch.from_numpy(s.P).cuda()
    say("gpu: capacity learning on a fresh tree")
    K1 = torch.zeros_like(P)
    fx.fx_exchange(tree, P, s.tau, K1)
    K2, st = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P))
    torch.cuda.synchronize()
    assert torch.equal(K1, K2) and st["overflow"] == 0 and st["chunks"] == 0
    Ko, _ = oracle.exchange(s)
    assert np.abs(K2.cpu().numpy() - Ko).max() <= 1e-10


def test_caller_allocator_owns_the_workspace(mid):
    """fx_set_allocator: the call's workspace comes from the caller's
    allocator (here PyTorch's caching allocator, on the call's stream), and K
    is the same as with the library's own allocation."""
    import ctypes
    s, tree, P, Kref, _ = mid
    say("gpu: workspace from the PyTorch caching allocator")
    calls = {"alloc": 0, "free": 0}
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

    def alloc(nbytes, stream, ctx):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream)

    def free(ptr, stream, ctx):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    a, f = ALLOC(alloc), FREE(free)
    L = fx.lib()
    L.fx_set_allocator.argtypes = [ALLOC, FREE, ctypes.c_void_p]
    assert L.fx_set_allocator(a, f, None) == 0
    try:
        stream = torch.cuda.current_stream()
        K, _ = fx.fx_exchange_ex(tree, P, s.tau, torch.zeros_like(P), fx.make_opts(precision=fx.FX_PREC_MIXED),
                                 stream=stream)
        torch.cuda.synchronize()
    finally:
        L.fx_set_allocator(ALLOC(), FREE(), None)
    assert calls["alloc"] >= 1 and calls["free"] == calls["alloc"]
    assert torch.equal(K, Kref)
