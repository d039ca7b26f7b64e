"""Host-side pieces of bench.py (no GPU): the multi-GPU refusal, the byte
models behind the roofline, and the traffic figures' source check."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_byte_models():
    # detection + law: per sphere candidate record 8, packed state 40 + 6R, cell 4, two counts and the
    # first contact index 12; per contact list entry 4, history read and written 2 (4 + 3R), force
    # record 6R, partner slot 4 and filed entry 8; cell starts once
    assert bench.contacts_bytes(10, 7, 20, 4) == 10 * (8 + 64 + 4 + 12) + 20 * (4 + 32 + 24 + 4 + 8) + 4 * 8
    assert bench.contacts_bytes(10, 7, 20, 8) == 10 * (8 + 88 + 4 + 12) + 20 * (4 + 56 + 48 + 4 + 8) + 4 * 8
    # gather: per sphere state in 40 + 6R and out 36 + 6R, count and first index 8; per contact two record
    # reads and the filed entry
    assert bench.gather_bytes(10, 20, 4) == 10 * (64 + 60 + 8) + 20 * (48 + 8)
    # whole step: B = 2 state + 16 + 3 + Z (4 + 3R); 131 + 16 Z bytes in mixed precision
    assert bench.step_algorithmic_bytes(1, 0.0, 4) == 131
    assert bench.step_algorithmic_bytes(1, 6.0, 4) == pytest.approx(131 + 16 * 6)


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    rec = {"kernel_source_sha256": bench.kernel_source_hash(),
           "kernels": {"k_detect": {"bytes_per_launch": 1.5e9}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(p))
    assert bench.measured_traffic("k_detect") == 1.5e9
    assert bench.measured_traffic("k_gather") is None  # not measured
    p.write_text(json.dumps(dict(rec, kernel_source_sha256="0" * 64)))  # counters of other kernels
    assert bench.measured_traffic("k_detect") is None
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("k_detect") is None


def test_valu_utilisation_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    k = {"valu_utilisation": 0.18, "valu_issue": 0.3, "lane_use": 0.6, "ta_busy": 0.85}
    rec = {"kernel_source_sha256": bench.kernel_source_hash(), "kernels": {"k_contacts_direct": k}}
    p = tmp_path / "v.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "VALU_JSON", str(p))
    v = bench.measured_valu("k_contacts_direct")
    assert v["frac"] == 0.18 and v["issue_frac"] == 0.3 and v["lane_use"] == 0.6
    assert v["peak"] == 157.3 and v["unit"] == "TFLOP/s"
    assert bench.measured_valu("k_gather") is None
    p.write_text(json.dumps(dict(rec, kernel_source_sha256="0" * 64)))
    assert bench.measured_valu("k_contacts_direct") is None


def test_committed_counter_summaries_match_the_kernel_source():
    # the committed traffic and VALU figures were taken with the current kernels
    assert bench.measured_traffic("k_contacts_direct") is not None
    assert bench.measured_valu("k_contacts_direct") is not None
