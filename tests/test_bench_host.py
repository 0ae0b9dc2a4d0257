"""Host logic of bench.py (CPU only): the traffic record built from the two
counter runs, and its use only for the kernel source it was measured on."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write_counters(path, counter, gate_kib, copy_kib_each):
    """Two gate launches, then the calibration copies split over three
    dispatches each (as a 256 MiB device copy is)."""
    rows = []
    d = 1
    for v in gate_kib:
        rows.append((d, "void itpp::gate_kernel<2, 1024, 4000, double, false>(...)", v))
        d += 1
    rows.append((d, "itpp::select_decide(...)", 1.0))
    d += 1
    for _ in range(3):
        for part in (0.5, 0.25, 0.25):
            rows.append((d, "__amd_rocclr_copyBuffer", copy_kib_each * part))
            d += 1
    with open(path, "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for di, name, v in rows:
            wr.writerow([di, name, counter, v])


def test_summarize_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec_path))
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    true_kib = bench.COPY_BYTES / 1024.0
    # FETCH_SIZE reads half the bytes, WRITE_SIZE all of them
    _write_counters(f, "FETCH_SIZE", [1000.0, 3000.0], true_kib / 2)
    _write_counters(w, "WRITE_SIZE", [500.0, 1500.0], true_kib)
    bench.summarize_pmc(str(f), str(w))
    rec = json.load(open(rec_path))
    assert rec["counters"]["fetch"]["factor"] == pytest.approx(2.0)
    assert rec["counters"]["write"]["factor"] == pytest.approx(1.0)
    assert rec["counters"]["fetch"]["launches"] == 2
    assert rec["bytes_per_launch"] == pytest.approx((2000.0 * 2.0 + 1000.0) * 1024.0)
    assert rec["kernel_source_sha256"] == bench.kernel_source_hash()


def test_summarize_counts_only_launches_that_did_work(tmp_path, monkeypatch):
    """A redone gate leaves launches that return at once (a few bytes): they
    are not gates and do not dilute the per-launch traffic."""
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec_path))
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    true_kib = bench.COPY_BYTES / 1024.0
    _write_counters(f, "FETCH_SIZE", [1000.0, 0.25, 3000.0, 0.5], true_kib / 2)
    _write_counters(w, "WRITE_SIZE", [500.0, 0.0, 1500.0, 0.0], true_kib)
    bench.summarize_pmc(str(f), str(w))
    rec = json.load(open(rec_path))
    assert rec["counters"]["fetch"]["launches"] == 2 and rec["counters"]["fetch"]["empty_launches"] == 2
    assert rec["bytes_per_launch"] == pytest.approx((4000.75 / 2 * 2.0 + 1000.0) * 1024.0)


def test_record_ignored_for_another_kernel_source(tmp_path, monkeypatch):
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec_path))
    json.dump({"kernel_source_sha256": "0" * 64, "bytes_per_launch": 1.0}, open(rec_path, "w"))
    assert bench.measured_traffic() is None
    json.dump({"kernel_source_sha256": bench.kernel_source_hash(), "bytes_per_launch": 1.0}, open(rec_path, "w"))
    assert bench.measured_traffic()["bytes_per_launch"] == 1.0


def test_committed_record_matches_the_kernel_source():
    """The committed traffic figure was taken on the kernel as it stands."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "gate_kernel_traffic_tfim_n64_open_K2e24.json")))
    assert rec["kernel_source_sha256"] == bench.kernel_source_hash()


def test_more_than_one_gpu_exits_with_a_message():
    import subprocess

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
