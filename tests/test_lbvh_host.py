"""Host-side check of the LBVH node construction (the same header the build
kernel uses): a valid binary radix tree for sorted unique keys, including
runs of equal Morton codes."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_lbvh_node_construction(tmp_path):
    exe = tmp_path / "lbvh_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", str(exe), os.path.join(HERE, "native", "lbvh_check.cpp")])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
