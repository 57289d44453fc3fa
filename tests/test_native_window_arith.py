"""The exact integer arithmetic of the tiled particle kernels, checked on the host.

The helpers in ``pm_particles.h`` (window-cell division by a high multiply, cell
numbering, fixed-point CIC weights, node indices, the packed window reduction and
the over-capacity window) are compiled into a small host program
(``tests/native/window_arith_check.cpp``) that checks them exhaustively or on
random cases against their plain definitions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_window_arithmetic_is_exact(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "window_arith_check")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(ROOT, "tests", "native", "window_arith_check.cpp"),
           "-I", os.path.join(ROOT, "paper_2404_02783_amd", "csrc"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]
