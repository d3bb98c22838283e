"""Host logic of the measurement chain (no GPU): the counter calibration and
summaries of profsum on synthetic rocprofv3 CSV output, and the source-hash
gate that keeps a traffic figure of another kernel version out of the bench
line."""
import csv
import json
import os

import pytest

from paper_2602_14667_amd import kernel3d_hash, kernel_hash, profsum

COPY = profsum.COPY_BYTES


def write_stats(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_kernel_stats.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        for name, calls, avg in rows:
            w.writerow([name, calls, calls * avg, avg, 0.0, avg * 0.99, avg * 1.01])


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, ctr, kib) in enumerate(rows):
            w.writerow([i, name, ctr, kib])


COPY_K = "rr::k_copy16(uint4 const*, uint4*, long)"


def calibration(prof, fetch_counted, write_counted):
    """Copy kernel of COPY bytes whose counters read fetch_counted and
    write_counted bytes (per dispatch, in KiB)."""
    write_stats(os.path.join(prof, "stats_copy"), [(COPY_K, 20, 1.0e6)])
    write_counters(os.path.join(prof, "pmc_FETCH_SIZE_copy"),
                   [(COPY_K, "FETCH_SIZE", fetch_counted / 1024)] * 5)
    write_counters(os.path.join(prof, "pmc_WRITE_SIZE_copy"),
                   [(COPY_K, "WRITE_SIZE", write_counted / 1024)] * 5)


def test_step_summary_calibrates_counters(tmp_path):
    prof, out = str(tmp_path / "prof"), str(tmp_path / "out")
    os.makedirs(out)
    # the copy's fetch counter reads half its bytes, the write counter all
    calibration(prof, COPY / 2, COPY)
    n = 64
    k32 = "void rr::k_step<rr::CodecF32, false, false, true, false, false>(...)"
    k16 = "void rr::k_step_pair<rr::CodecF16U, true>(...)"
    for st, name, bpn in (("f32", k32, 152), ("f16", k16, 76)):
        alg = bpn * n * n
        write_stats(os.path.join(prof, f"stats_{st}"), [(name, 55, 2000.0), ("other", 3, 10.0)])
        # reads counted at 0.6x of half the algorithmic bytes -> 1.2x after x2
        write_counters(os.path.join(prof, f"pmc_FETCH_SIZE_{st}"),
                       [(name, "FETCH_SIZE", 0.6 * alg / 2 / 1024)] * 5)
        write_counters(os.path.join(prof, f"pmc_WRITE_SIZE_{st}"),
                       [(name, "WRITE_SIZE", alg / 2 / 1024)] * 5)
    profsum.main(prof, out, str(n))
    for st, bpn in (("f32", 152), ("f16", 76)):
        with open(os.path.join(out, f"traffic_step_{st}_{n}.json")) as fh:
            t = json.load(fh)
        alg = bpn * n * n
        assert t["kernel_hash"] == kernel_hash()
        assert t["fetch_factor"] == pytest.approx(2.0)
        assert t["write_factor"] == pytest.approx(1.0)
        assert t["read_bytes"] == pytest.approx(1.2 * alg / 2)
        assert t["write_bytes"] == pytest.approx(alg / 2)
        assert t["bytes_per_launch"] == pytest.approx(1.1 * alg)
        with open(os.path.join(out, f"step_{st}_{n}.md")) as fh:
            md = fh.read()
        assert "1.200x algorithmic" in md and "average launch: 2.0 us" in md


def test_step3d_summary(tmp_path):
    prof, out = str(tmp_path / "prof"), str(tmp_path / "out")
    os.makedirs(out)
    calibration(prof, COPY / 2, COPY)
    n = 16
    k32 = "void rr3::k_step3<rr::CodecF32>(rr3::Dom3, int, ...)"
    k16 = "void rr3::k_step3<rr::CodecF16U>(rr3::Dom3, int, ...)"
    write_stats(os.path.join(prof, "s3_stats"), [(k32, 55, 4000.0), (k16, 55, 2000.0)])
    fetch, write = [], []
    for name, bpn in ((k32, 384), (k16, 192)):
        alg = bpn * n ** 3
        fetch.append((name, "FETCH_SIZE", alg / 4 / 1024))   # -> 1.0x after x2
        write.append((name, "WRITE_SIZE", alg / 2 / 1024))
    write_counters(os.path.join(prof, "s3_pmc_FETCH_SIZE"), fetch * 3)
    write_counters(os.path.join(prof, "s3_pmc_WRITE_SIZE"), write * 3)
    profsum.step3d_summary(prof, out, str(n))
    for st, bpn in (("f32", 384), ("f16", 192)):
        with open(os.path.join(out, f"traffic_step3d_{st}_{n}.json")) as fh:
            t = json.load(fh)
        assert t["kernel_hash"] == kernel3d_hash()
        assert t["bytes_per_launch"] == pytest.approx(bpn * n ** 3)


def test_bench_traffic_gate(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    path = tmp_path / "profiles" / "traffic_step_f32_64.json"
    assert bench.measured_traffic("f32", 64) is None          # absent
    path.write_text(json.dumps({"kernel_hash": "0" * 16, "bytes_per_launch": 123.0}))
    assert bench.measured_traffic("f32", 64) is None          # another kernel version
    path.write_text(json.dumps({"kernel_hash": kernel_hash(), "bytes_per_launch": 123.0}))
    assert bench.measured_traffic("f32", 64) == 123.0
    # the 3D figure is gated by the 3D sources' hash
    p3 = tmp_path / "profiles" / "traffic_step3d_f32_16.json"
    p3.write_text(json.dumps({"kernel_hash": kernel_hash(), "bytes_per_launch": 7.0}))
    assert bench.measured_traffic("f32", 16, dims=3) is None
    p3.write_text(json.dumps({"kernel_hash": kernel3d_hash(), "bytes_per_launch": 7.0}))
    assert bench.measured_traffic("f32", 16, dims=3) == 7.0


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
