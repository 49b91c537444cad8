"""Host-side checks of bench.py: its one-GPU contract, its options and the
committed traffic figures it reads (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_every_leg_switch():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--no-cpu-baseline", "--no-variants", "--no-uneven", "--no-dense", "--no-stencil",
                 "--no-stiff", "--no-multi-rhs", "--no-warmstart", "--no-mechanisms",
                 "--calibrate-copy"):
        assert flag in r.stdout


def test_traffic_figures_are_consistent():
    """The committed FETCH_SIZE/WRITE_SIZE figures: scaled by the copy calibration,
    for the workload the headline names, and within a few percent above the
    algorithmic bytes (every value read once)."""
    name = "chem_jacobian_b131072_n54_csr_bicgstab_jacobi_fp64"
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    with open(path) as f:
        t = json.load(f)
    cal = t["copy_calibration"]
    gib_kib = cal["bytes_read_and_written"] / 1024
    assert abs(cal["fetch_factor"] - gib_kib / cal["fetch_size_kib"]) < 1e-9
    assert abs(cal["write_factor"] - gib_kib / cal["write_size_kib"]) < 1e-9
    assert abs(t["fetch_bytes_per_launch"] - t["fetch_size_kib_per_dispatch"] * 1024 * cal["fetch_factor"]) < 1e3
    assert abs(t["write_bytes_per_launch"] - t["write_size_kib_per_dispatch"] * 1024 * cal["write_factor"]) < 1e3
    ratio = (t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]) / t["algorithmic_bytes_per_launch"]
    assert 1.0 <= ratio < 1.1
    assert t["workload"] == name and len(t["kernel_source_sha"]) == 16
