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


def test_traffic_summary_with_one_block_per_family(tmp_path, monkeypatch):
    """Several families in one summary, each with its own source file: each block is read
    for its own kernel, and a changed source voids only the blocks that name it."""
    (tmp_path / "a.hip").write_text("a\n")
    (tmp_path / "b.hip").write_text("b\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    def block(name, fetch, src, sha):
        return (f"kernel: {name}\nfetch_kib_per_launch: {fetch}\nwrite_kib_per_launch: 1.0\n"
                f"fetch_calibration: 2.0\nwrite_calibration: 1.0\nsource: {src}\nsource_sha256: {sha}\n")

    (tmp_path / "profiles" / "traffic_wl.txt").write_text(
        "# counters\n" + block("mg_smooth2", 10.0, "a.hip", bench.source_sha256("a.hip"))
        + block("cg_update", 20.0, "a.hip", bench.source_sha256("a.hip"))
        + block("gs_update", 30.0, "b.hip", "0" * 64))
    assert bench.measured_traffic("wl", "mg_smooth2") == 1024.0 * (10.0 * 2.0 + 1.0)
    assert bench.measured_traffic("wl", "cg_update") == 1024.0 * (20.0 * 2.0 + 1.0)
    assert bench.measured_traffic("wl", "gs_update") is None     # its source changed since
    assert bench.measured_traffic("wl", "mg_down") is None       # no block for it


def test_extrapolated_cpu_baseline_on_a_small_sample():
    """The extrapolated oracle baseline of the 3D boxes runs on the CPU, labels itself, scales
    by the cell count and combines the per-call costs with the given iteration counts."""
    class A:
        workload = "convective_box_3d"
    w = W.convective_box_3d(n=32)
    stats = [dict(newton_its=6, gmres_its=120, cg_its=900, converged=1)] * 2
    r = bench.cpu_baseline_extrapolated(w, stats, A(), sample_n=16)
    assert r["kind"] == "oracle" and r["extrapolated"] and r["cores"] == 1
    assert "scaled x8" in r["sample"] and "Newton 6.00, GMRES 120.0, CG 900.0" in r["sample"]
    c = r["components_s_at_sample"]
    step = 8 * (6 * (c["residual_and_scalings"] + c["pc_setup"])
                + 120 * (c["fd_jv"] + c["pc_apply_at_gpu_cg_count"] + c["arnoldi_per_iteration"]))
    assert abs(r["seconds_per_step"] - step) <= 1e-9 * step and abs(r["value"] * step - 1.0) < 1e-12
