"""Host logic of bench.py (no GPU): the one-GPU contract, the workload names, and the use
of the committed counter summary only while the kernel's source is unchanged."""
import os
import subprocess
import sys

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workload_names_match_the_generators():
    assert set(bench.WORKLOADS) == set(W.CONFIGS)


def test_traffic_summary_needs_the_same_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    summary = tmp_path / "profiles" / "traffic_wl.txt"

    def write(sha):
        summary.write_text("# header: ignored\n"
                           "kernel: mg_down\n"
                           "fetch_kib_per_launch: 10.0\nwrite_kib_per_launch: 2.0\n"
                           "fetch_calibration: 2.0\nwrite_calibration: 1.0\n"
                           f"source: k.hip\nsource_sha256: {sha}\n")

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    write(bench.source_sha256("k.hip"))
    assert bench.measured_traffic("wl", "mg_down") == 1024.0 * (10.0 * 2.0 + 2.0 * 1.0)
    assert bench.measured_traffic("wl", "cg_apply") is None      # another kernel
    assert bench.measured_traffic("other", "mg_down") is None    # no summary
    write("0" * 64)                                               # source changed since
    assert bench.measured_traffic("wl", "mg_down") is None
