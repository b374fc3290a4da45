"""Host logic of the persistent plan: the row-tile partition is optimal (exhaustive DP
on random cases; compiled with the host C++ compiler, no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_row_partition_is_min_max_optimal(tmp_path):
    exe = str(tmp_path / "partition_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2603_25762_amd", "csrc"),
                           os.path.join(ROOT, "tests", "partition_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
