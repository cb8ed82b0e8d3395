"""The geometry of the spectrum's windowed multishift QR sweep (the rules in
paper_1912_01491_amd/csrc/qr_window.h that the kernels and the host loop use),
checked on the CPU by tests/native/qr_window_check.cpp over many block sizes and
bulge counts: windows inside the block and disjoint, every reflector position of a
round inside its chain's window, the far parts of a round's products disjoint from
the next round's windows, no product split around the other one on a crossing
block, and the window factor's zero pattern inside the band the products skip."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "qr_window_check.cpp")
INC = os.path.join(ROOT, "paper_1912_01491_amd", "csrc")


def test_window_geometry(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "qr_window_check")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-I", INC, SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 failed" in r.stdout
