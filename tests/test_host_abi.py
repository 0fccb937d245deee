"""CPU-side checks of the C ABI: the library loads, exports every symbol
the header declares, validates arguments before touching the GPU, and the
host planner (Hilbert ordering, ragged bisection of Eq. (1)) has the
properties the traversal relies on."""
import ctypes
import os
import re

import numpy as np
import pytest

import synthetic

fx = pytest.importorskip("paper_1401_6961_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "fx.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fx_status|int32_t|void|const char\*)\s+(fx_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    L = fx.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = fx.lib()
    assert fx.fx.status_string(0) == "FX_OK"
    assert fx.fx.status_string(2) == "FX_ERR_UNSUPPORTED"


def _shells(s):
    return fx.fx._ShellArrays(s.l, s.nprim, s.center, s.exps, s.coefs)


def test_invalid_arguments_are_rejected_before_device_work():
    L = fx.lib()
    vp = ctypes.c_void_p
    # NULL tree / pointers / negative or NaN tau: validated on the host
    assert L.fx_exchange(None, vp(8), 1e-8, vp(16), None) == 1
    s = synthetic.tiny_cube(natom=3, edge=3.0, seed=5)
    # unsupported angular momentum and primitive counts
    for field, val in (("l", 3), ("nprim", 0), ("nprim", 17)):
        bad = synthetic.tiny_cube(natom=3, edge=3.0, seed=5)
        arr = getattr(bad, field).copy()
        arr[1] = val
        setattr(bad, field, arr)
        if field == "nprim":
            continue  # exps length would no longer match; covered by plan test below
        sh = _shells(bad)
        out = vp()
        assert L.fx_build_quadtree(ctypes.byref(sh.s), None, None, ctypes.byref(out)) == 2
        assert b"l outside" in L.fx_last_error_message()
    bad = synthetic.tiny_cube(natom=3, edge=3.0, seed=5)
    bad.exps = bad.exps.copy()
    bad.exps[0] = -1.0
    sh = _shells(bad)
    out = vp()
    assert L.fx_build_quadtree(ctypes.byref(sh.s), None, None, ctypes.byref(out)) == 1
    assert L.fx_build_quadtree(None, None, None, ctypes.byref(out)) == 1
    with pytest.raises(fx.FxError):
        fx.fx_set_class_variant(81, 0, 0)


def test_variant_table():
    for cls in range(81):
        av = fx.fx_class_variants_available(cls)
        assert av in (5, 7)          # one quartet per lane, and both precisions in one pass, always
        for p in (0, 1):
            v = fx.fx_get_class_variant(cls, p)
            assert av & (1 << v)
            assert v != 2 or p == 0
    # (ss|ss) has no one-quartet-per-wave form, (dd|dd) has
    assert fx.fx_class_variants_available(0) == 5
    assert fx.fx_class_variants_available(80) == 7
    with pytest.raises(fx.FxError):
        fx.fx_set_class_variant(80, 1, 2)    # the one-pass form is selected on the FP64 entry


def test_hilbert_curve_is_a_unit_step_path():
    """Sorting all cells of a 2^b grid by the key visits every cell once,
    consecutive cells being face neighbours: the locality property the
    shell ordering relies on (Section III)."""
    b = 3
    n = 1 << b
    keys = {}
    for x in range(n):
        for y in range(n):
            for z in range(n):
                keys[fx.fx.hilbert_key3(x, y, z, b)] = (x, y, z)
    assert sorted(keys) == list(range(n ** 3))
    path = [keys[k] for k in range(n ** 3)]
    for p, q in zip(path, path[1:]):
        assert sum(abs(a - c) for a, c in zip(p, q)) == 1


@pytest.mark.parametrize("leaf", [0, 1, 4, 10, 30])
def test_bisection_partitions_shells_and_keeps_them_whole(leaf):
    s = synthetic.cluster(60, with_d=True, density=False)
    perm, nodes = fx.fx_plan_tree(s.l, s.nprim, s.center, s.exps, s.coefs, leaf_max_functions=leaf)
    assert sorted(perm) == list(range(s.nshell))
    nlev = nodes[:, 0].max() + 1
    nf = np.array([synthetic.NCART[x] for x in s.l[perm]])
    fp = np.concatenate([[0], np.cumsum(nf)])
    for lv in range(nlev):
        lvl = nodes[nodes[:, 0] == lv]
        # every level covers [0, S) exactly once, in order
        assert lvl[0, 1] == 0 and lvl[-1, 2] == s.nshell
        assert np.all(lvl[1:, 1] == lvl[:-1, 2])
        if lv + 1 < nlev:
            nxt = nodes[nodes[:, 0] == lv + 1]
            assert lvl[:, 3].sum() == len(nxt)
    leaves = nodes[nodes[:, 0] == nlev - 1]
    lim = 10 if leaf == 0 else leaf
    for a, b_, _ in leaves[:, 1:4]:
        assert b_ - a == 1 or fp[b_] - fp[a] <= lim
    # splits land at the shell boundary nearest the function midpoint
    for lv in range(nlev - 1):
        lvl = nodes[nodes[:, 0] == lv]
        nxt = nodes[nodes[:, 0] == lv + 1]
        k = 0
        for a, b_, nch in lvl[:, 1:4]:
            if nch == 2:
                m = nxt[k, 2]
                mid = 0.5 * (fp[a] + fp[b_])
                best = min(range(a + 1, b_), key=lambda t: (abs(fp[t] - mid), t))
                assert m == best
            k += nch


def test_hilbert_order_keeps_atoms_together():
    s = synthetic.cluster(40, with_d=True, density=False)
    perm, _ = fx.fx_plan_tree(s.l, s.nprim, s.center, s.exps, s.coefs)
    atoms = s.shell_atom[perm]
    # shells of one atom are consecutive and keep their s, p, d order
    for a in np.unique(atoms):
        pos = np.nonzero(atoms == a)[0]
        assert np.all(np.diff(pos) == 1)
        assert list(s.l[perm][pos]) == [0, 1, 2]


def test_xcd_remap_is_a_bijection():
    L = fx.lib()
    for nb in list(range(1, 70)) + [255, 256, 1000, 4099]:
        img = [L.fx_xcd_block(b, nb) for b in range(nb)]
        assert sorted(img) == list(range(nb))
        # consecutive logical blocks of one XCD: b and b + 8 map to neighbours
        for b in range(nb - 8):
            assert img[b + 8] == img[b] + 1
    assert L.fx_xcd_block(5, 5) == -1


def test_persistent_launch_flag_is_switched_off():
    with pytest.raises(fx.FxError):
        fx.fx_set_class_launch(0, 0, 2)


def test_exchange_opts_init_fills_documented_defaults():
    """A zero-filled options struct is not the defaults (alpha would be 0);
    fx_exchange_opts_init gives the documented ones."""
    o = fx.opts_init()
    assert o.precision == fx.FX_PREC_FP64 and o.fp32_threshold == 1e-5
    assert o.schedule == fx.FX_SCHED_BOUND and not o.costmodel
    assert o.alpha == 1.0 and o.beta == 0.0
    assert o.max_frontier_entries == 0 and o.profile == 0 and o.use_graph == 0
    assert o.symmetry == fx.FX_SYM_AUTO and o.leaf_screen == fx.FX_LEAF_SHELL
    assert o.tau_ovlp == 0.0 and o.max_workspace_bytes == 0
    d = fx.make_opts()
    for name, _ in fx.fx_exchange_opts._fields_:
        if name != "costmodel":
            assert getattr(o, name) == getattr(d, name), name


def test_costmodel_load_rejects_foreign_files(tmp_path):
    """A missing, foreign or truncated file is refused before any device work."""
    import ctypes as C
    L = fx.lib()
    h = C.c_void_p()
    missing = tmp_path / "none.fxmlp"
    assert L.fx_costmodel_load(os.fsencode(str(missing)), C.byref(h)) == 1
    bad = tmp_path / "bad.fxmlp"
    bad.write_bytes(b"FXMLP001" + b"\x00" * 12)
    assert L.fx_costmodel_load(os.fsencode(str(bad)), C.byref(h)) == 1
    assert not h.value


def test_row_cuts_partition_the_leaves_and_balance_the_entries():
    """K row ranges for the workspace budget: contiguous, non-empty, covering
    every leaf; each range's entries exceed an equal share by less than its
    largest leaf; with no counts, leaf counts differ by at most one."""
    rng = np.random.default_rng(11)
    for trial in range(50):
        nleaf = int(rng.integers(1, 400))
        rows = rng.integers(0, 1000, nleaf) * (rng.random(nleaf) < 0.9)
        if trial % 5 == 0:
            rows[: nleaf // 2] *= 50          # a heavy block of rows
        n = int(rng.integers(1, nleaf + 3))
        cuts = fx.plan_row_cuts(rows, n)
        m = min(n, nleaf)
        assert cuts[0] == 0 and cuts[m] == nleaf and np.all(cuts[m:] == nleaf)
        assert np.all(np.diff(cuts[: m + 1]) >= 1)
        total = int(rows.sum())
        if total > 0 and m > 1:
            for k in range(m):
                seg = rows[cuts[k]:cuts[k + 1]]
                assert seg.sum() <= total / m + rows.max() * 2, (trial, k)
        even = fx.plan_row_cuts(None, n, nleaf=nleaf)
        sizes = np.diff(even[: m + 1])
        assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1


def test_row_cuts_reject_bad_arguments():
    with pytest.raises(fx.FxError):
        fx.plan_row_cuts(np.array([1, -2, 3]), 2)
    with pytest.raises(fx.FxError):
        fx.plan_row_cuts(None, 0, nleaf=5)
