"""Host-side logic of bench.py (CPU): the one-GPU refusal and the counter-summary
lookup that supplies the roofline's `traffic` only while the kernel sources match."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _record():
    rec = None
    for line in open(bench.PMC_SUMMARY):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
    return rec


def test_counter_summary_has_a_traffic_record():
    rec = _record()
    assert rec is not None and len(rec["source_sha16"]) == 16
    row = rec["kernels"]["k_key_ip"]
    assert row["hbm_bytes_per_launch"] > 0


def test_traffic_reported_only_for_matching_sources(monkeypatch):
    rec = _record()
    monkeypatch.setattr(bench, "source_digest", lambda: rec["source_sha16"])
    val, note = bench.pmc_traffic("k_key_ip")
    assert val == rec["kernels"]["k_key_ip"]["hbm_bytes_per_launch"] and "FETCH_SIZE" in note
    assert bench.pmc_traffic("no_such_kernel")[0] is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    val, note = bench.pmc_traffic("k_key_ip")
    assert val is None and "changed" in note
