"""Host-side logic of bench.py (no GPU): the counter record is used only for
the kernel sources it was taken on, and the reported figures are formed from
it as documented."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def write_record(path, sha, kernels):
    with open(path, "w") as f:
        json.dump({"source_sha256": sha, "kernels": kernels}, f)


def test_source_hash_covers_the_pass_sources_only():
    h = bench.kernel_source_hash()
    assert len(h) == 64 and h == bench.kernel_source_hash()
    csrc = os.path.join(ROOT, "paper_2307_01571_amd", "csrc")
    for name in bench.PASS_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name


def test_counters_follow_the_source_hash(tmp_path, monkeypatch):
    rec = tmp_path / "traffic.json"
    kern = {"col_pass": {"read_bytes": 100.0, "write_bytes": 50.0, "valu_insts": 7.0}}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    write_record(rec, bench.kernel_source_hash(), kern)
    assert bench.measured_counters("col_pass") == {"bytes": 150.0, "valu_insts": 7.0}
    assert bench.measured_counters("row_pass") is None
    write_record(rec, "0" * 64, kern)  # taken on other kernel sources
    assert bench.measured_counters("col_pass") is None
    rec.unlink()
    assert bench.measured_counters("col_pass") is None


def test_valu_peak_is_the_issue_rate():
    # 256 CUs x 4 SIMDs at 2.4 GHz, one wave64 VALU instruction per SIMD every 4 cycles
    assert abs(bench.VALU_PEAK_GINST - 614.4) < 1e-9
