"""bench.py's own logic, on the CPU: the roofline arithmetic, the traffic
figures read from the committed counter summaries (keyed by the kernel code),
and the refusal of more than one GPU."""
import os
import subprocess
import sys
import types

import pytest

import bench


def stat(launches, ms, alg_bytes):
    return types.SimpleNamespace(launches=launches, ms=ms, alg_bytes=alg_bytes)


def test_roofline_reports_the_dominant_histogram_kernel():
    st = types.SimpleNamespace(hist_large=stat(240, 19.2, 240 * 30e6),
                               hist_small=stat(240, 14.0, 240 * 4e6),
                               hist_col=stat(0, 0.0, 0.0), finalize=stat(240, 8.0, 0.0),
                               permut=stat(0, 0.0, 0.0))
    roof, kernels = bench.roofline(st)
    assert roof["kernel"] == "hist_large" and roof["unit"] == "GB/s"
    assert roof["avg_launch_ms"] == pytest.approx(0.08)
    # 30 MB per launch in 80 us: 375 GB/s of 8000
    assert roof["achieved"] == pytest.approx(375.0)
    assert roof["peak"] == bench.HBM_PEAK_GBS == 8000.0
    assert roof["frac"] == pytest.approx(375.0 / 8000.0, abs=1e-4)
    assert set(kernels) == set(bench.KERNELS)


def test_traffic_read_only_for_the_profiled_kernel_code(monkeypatch):
    found = 0
    for name in os.listdir(os.path.join(bench.ROOT, "profiles")):
        if not name.endswith("_traffic.md"):
            continue
        kernel_file, workload = name[:-len("_traffic.md")].rsplit("_", 1)
        stat_name = [k for k, v in bench.KERNEL_NAMES.items() if v == kernel_file][0]
        with open(os.path.join(bench.ROOT, "profiles", name)) as f:
            text = f.read()
        key = [l.split(":", 1)[1].strip() for l in text.splitlines()
               if l.startswith("kernel_code_sha256")][0]
        monkeypatch.setattr(bench, "kernel_code_digest", lambda: key)
        v = bench.measured_traffic(workload, stat_name)
        assert isinstance(v, float) and v > 0
        monkeypatch.setattr(bench, "kernel_code_digest", lambda: "0" * 64)
        assert bench.measured_traffic(workload, stat_name) is None
        found += 1
    assert found >= 1
    assert bench.measured_traffic("no_such_workload", "hist_large") is None


def test_digest_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    import shutil
    src = os.path.join(bench.ROOT, "paper_2605_09950_amd", "csrc")
    dst = tmp_path / "paper_2605_09950_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("k_forest.hip", "forest_dev.hpp", "dev_common.hpp", "reg_dev.hpp"):
        shutil.copy(os.path.join(src, name), dst / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_code_digest()
    with open(dst / "k_forest.hip", "a") as f:
        f.write("\n// a comment\n\n   \n")
    assert bench.kernel_code_digest() == d0
    with open(dst / "k_forest.hip", "a") as f:
        f.write("static int extra_code_line;\n")
    assert bench.kernel_code_digest() != d0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
