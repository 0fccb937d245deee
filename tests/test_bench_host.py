"""CPU-side checks of bench.py's host logic: the HBM-traffic record is read
only while the kernel's sources hash to the value recorded with the
counters, and the tuning-table summary names the table it hashes."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_record_needs_the_recorded_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "fx_k_xxxx_f64", "gen_hash": "abc", "traffic_bytes_per_launch": 123.0}
    (prof / "hbm_traffic_xxxx_test.md").write_text("# t\n\n```json\n" + json.dumps(rec) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda k: "abc")
    assert bench.profiled_traffic("fx_k_xxxx_f64") == (123.0, os.path.join("profiles", "hbm_traffic_xxxx_test.md"))
    assert bench.profiled_traffic("fx_k_yyyy_f64") == (None, None)
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda k: "changed")
    assert bench.profiled_traffic("fx_k_xxxx_f64") == (None, None)


def test_committed_traffic_records_parse():
    """Every committed record carries the fields bench.py reads."""
    import glob
    import re
    paths = glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))
    assert paths
    for p in paths:
        m = re.search(r"```json\n(.*?)\n```", open(p).read(), re.S)
        assert m, p
        rec = json.loads(m.group(1))
        assert rec["kernel"].startswith("fx_k_") and rec["traffic_bytes_per_launch"] > 0
        assert len(rec["gen_hash"]) == 16


def test_tuning_table_info_hashes_the_package_table():
    import hashlib
    info = bench.tuning_table_info()
    path = os.path.join(ROOT, info["path"])
    assert info["sha256"] == hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    assert info["launch_entries"] == 162 and info["generator_kernels"] > 162
