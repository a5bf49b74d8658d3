"""Host logic of bench.py (no GPU): the counter-record gate of roofline.traffic and the
one-GPU contract of the command line."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record():
    for line in open(os.path.join(ROOT, "profiles", "hbm_traffic_internal_conductors_2000.md")):
        if line.startswith("traffic-record: "):
            return json.loads(line[len("traffic-record: "):])
    raise AssertionError("no traffic record in the committed counter summary")


def test_traffic_record_matches_the_committed_kernel():
    import bench
    rec = _record()
    lay = types.SimpleNamespace(internal_entries=rec["internal_entries"], rows_per_wave=rec["rows_per_wave"])
    import hashlib
    if hashlib.sha256(bench.internal_kernel_source().encode()).hexdigest() != rec["kernel_source_sha256"]:
        pytest.skip("the internal kernel changed since its counters were taken: the bench reports null traffic")
    t = bench.internal_traffic(rec["workload"], lay)
    assert t is not None
    assert t == pytest.approx(1024.0 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]))
    # one launch reads half of the arena (the rows of M_i or of Z_i), complex64 entries:
    # its HBM bytes cannot be below that
    assert t >= 0.5 * 8.0 * rec["internal_entries"]


def test_traffic_is_null_for_another_workload_or_shape(monkeypatch):
    import bench
    rec = _record()
    ok = dict(internal_entries=rec["internal_entries"], rows_per_wave=rec["rows_per_wave"])
    assert bench.internal_traffic("line_bundle", types.SimpleNamespace(**ok)) is None
    other = dict(ok, internal_entries=ok["internal_entries"] + 1)
    assert bench.internal_traffic(rec["workload"], types.SimpleNamespace(**other)) is None
    other = dict(ok, rows_per_wave=12 - ok["rows_per_wave"])   # 8 <-> 4
    assert bench.internal_traffic(rec["workload"], types.SimpleNamespace(**other)) is None
    # any change to the kernel's source text voids the record
    src = bench.internal_kernel_source()
    monkeypatch.setattr(bench, "internal_kernel_source", lambda: src + " ")
    assert bench.internal_traffic(rec["workload"], types.SimpleNamespace(**ok)) is None


def test_kernel_source_region_spans_the_queue_helpers_and_the_kernel():
    import bench
    src = bench.internal_kernel_source()
    assert src.startswith("struct TileQueue {")
    assert "k_internal(const float2*" in src and src.endswith("\n}\n")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
