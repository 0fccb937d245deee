"""CPU-side checks of the tuning table: the generator reads its per-kernel
choices from it, the autotuner's candidates change what they claim to, and
the choice step keeps, per class, the entries of the fastest candidate."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_6961_amd", "csrc")
if CSRC not in sys.path:
    sys.path.insert(0, CSRC)

import gen_eri  # noqa: E402
from paper_1401_6961_amd import autotune  # noqa: E402

TABLE = os.path.join(ROOT, "paper_1401_6961_amd", "tuning_gfx950.json")
L = "spd"


def class_name(c):
    return L[c // 27] + L[(c // 9) % 3] + L[(c // 3) % 3] + L[c % 3]


def kernels():
    return json.load(open(TABLE))["generator"]["kernels"]


def test_generator_sets_follow_the_table():
    k = kernels()
    gen_eri.load_choices(TABLE)
    try:
        for key, e in k.items():
            cls, prec = key.split(":")
            if prec == "mix":
                assert cls in gen_eri.DUAL
                continue
            form = e.get("form", "register")
            assert ((cls, prec) in gen_eri.STAGED) == (form in ("staged", "folded")), key
            assert ((cls, prec) in gen_eri.FOLD) == (form == "folded"), key
            assert gen_eri.MIN_WAVES.get((cls, prec), 1) == e.get("waves", 1), key
            assert gen_eri.GROUPS.get((cls, prec), 3) == e.get("groups", 3), key
        assert gen_eri.DUAL == {key.split(":")[0] for key in k if key.endswith(":mix")}
    finally:
        gen_eri.load_choices()


def test_without_a_table_every_kernel_is_the_register_form(tmp_path):
    gen_eri.load_choices(str(tmp_path / "none.json"))
    try:
        assert not (gen_eri.STAGED or gen_eri.FOLD or gen_eri.DUAL or gen_eri.MIN_WAVES or gen_eri.GROUPS)
    finally:
        gen_eri.load_choices()


def test_generated_class_file_carries_the_kernel_choices(tmp_path):
    """One class file generated from the table: its waves and entry-group
    defines are the table's."""
    k = kernels()
    key = next(x for x, e in k.items() if e.get("groups", 3) != 3)
    cls, prec = key.split(":")
    la, lb, lc, ld = (L.index(x) for x in cls)
    gen_eri.load_choices(TABLE)
    try:
        gen_eri.main(str(tmp_path))
    finally:
        gen_eri.load_choices()
    src = open(tmp_path / f"eri_{cls}.hip").read()
    assert f"#define FX_FILL_GROUPS_{prec} {k[key]['groups']}" in src
    dddd = open(tmp_path / "eri_dddd.hip").read()
    assert f"#define FX_THREAD_MIN_WAVES_f64 {k['dddd:f64']['waves']}" in dddd
    table_h = open(tmp_path / "eri_table.h").read()
    dual = [int(x) for x in table_h.split("fx_class_dual_default[81] = {")[1].split("}")[0].split(",")]
    assert [class_name(c) in {x.split(':')[0] for x in k if x.endswith(':mix')} for c in range(81)] == \
        [bool(x) for x in dual]


def test_candidates_change_what_they_name():
    k = kernels()
    assert autotune.candidate_kernels("current", k) == k
    none = autotune.candidate_kernels("dual_none", k)
    assert not any(x.endswith(":mix") for x in none)
    allm = autotune.candidate_kernels("dual_all", k)
    assert sum(x.endswith(":mix") for x in allm) == 81
    folded = autotune.candidate_kernels("folded", k)
    for key, e in folded.items():
        if key.endswith(":mix"):
            continue
        if "d" in key.split(":")[0]:
            assert e["form"] == "folded" and e["waves"] == 1
        else:
            assert e == k[key]
    with pytest.raises(ValueError):
        autotune.candidate_kernels("nonsense", k)


def test_choose_keeps_the_fastest_candidate_per_class(tmp_path):
    """Synthetic timings: candidate B is faster for even classes only; the
    chosen table takes B's entries there and the current ones elsewhere."""
    base = json.load(open(TABLE))
    table = tmp_path / "table.json"
    table.write_text(json.dumps(base))
    k = base["generator"]["kernels"]
    names = ("current", "folded")
    for i, nm in enumerate(names):
        d = tmp_path / nm
        d.mkdir()
        t = dict(base)
        t["generator"] = dict(base["generator"], kernels=autotune.candidate_kernels(nm, k))
        (d / "table.json").write_text(json.dumps(t))
        cs = np.ones((81, 2))
        if nm == "folded":
            cs[0::2] = 0.5
            cs[1::2] = 2.0
        (d / "times.json").write_text(json.dumps({"class_seconds": cs.tolist()}))
    autotune.generator_choose(str(tmp_path), table_path=str(table), names=names, log=lambda m: None)
    chosen = json.load(open(table))["generator"]["kernels"]
    folded = autotune.candidate_kernels("folded", k)
    for c in range(81):
        cls = class_name(c)
        src = folded if c % 2 == 0 else k
        for prec in ("f64", "f32"):
            assert chosen[f"{cls}:{prec}"] == src[f"{cls}:{prec}"], (cls, prec)
