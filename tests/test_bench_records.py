"""Host-side checks of bench.py's committed counter records: the traffic and
VALU records apply only to the forward kernel sources and launch plans they
were measured on (a changed kernel or plan reports null, never a stale
figure), and the records in profiles/ are consistent with each other."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(name):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        return json.load(f)


def _plans(rec):
    return {int(r): {"tile": (v[0], v[1]), "fused": v[2]} for r, v in rec["plans"].items()}


def test_records_share_plans_and_hash():
    t, v = _record("fwd_traffic.json"), _record("fwd_valu.json")
    assert t["plans"] == v["plans"]
    assert t["kernel_hash"] == v["kernel_hash"]
    assert set(v["lane_ops_per_px_sweep"]) == {str(r) for r in bench.RADII}


def test_records_apply_only_to_their_kernels_and_plans(monkeypatch):
    rec = _record("fwd_valu.json")
    plans = _plans(rec)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_hash"])
    got = bench.measured_valu(plans)
    assert got == {int(r): float(x) for r, x in rec["lane_ops_per_px_sweep"].items()}
    assert bench.measured_traffic("rgb2048_T30", plans) == _record("fwd_traffic.json")["per_launch_bytes"]["rgb2048_T30"]
    other = dict(plans)
    other[bench.RADII[0]] = {"tile": (1, 1), "fused": 1}
    assert bench.measured_valu(other) is None
    assert bench.measured_traffic("rgb2048_T30", other) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_valu(plans) is None
    assert bench.measured_traffic("rgb2048_T30", plans) is None


def test_valu_peak_is_the_unpacked_fp32_issue_rate():
    assert abs(bench.VALU_PEAK_TLANE_OPS - 39.3216) < 1e-9


def test_parity_record_applies_only_to_its_kernels_and_plans(monkeypatch, tmp_path):
    rec = {"kernel_hash": "abc", "plans": {"2": [188, 0, 1]}, "headline": {}, "precision": {}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "parity_record.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    plans = {2: {"tile": (188, 0), "fused": 1}}
    assert bench.parity_record(plans) == rec
    assert bench.parity_record({2: {"tile": (120, 0), "fused": 2}}) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.parity_record(plans) is None
