"""Launch geometry of the library's problem-sized kernels (host only).

Compiles tests/native/launch_geom_check.cpp against csrc/launch_geom.h with
g++ and runs it: at n = q = 2^30 (the node cap) and 2^33 edges no dispatch may
hold 2^32 or more work-items.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_launch_geometry_below_2_32(tmp_path):
    exe = tmp_path / "launch_geom_check"
    src = os.path.join(HERE, "native", "launch_geom_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "TOO LARGE" not in r.stdout
