"""The bit-sliced hybrid median logic of the kernels (csrc/logfx_bits.h)
against the definition of the hybrid median (Sec. 3.4), on every pattern of
the pixels its two subgroups read, for both window sizes.  Host only: the
header is plain C++ and is compiled here with the system compiler."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_median_bits_exhaustive(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "median_bits_check")
    subprocess.run([cxx, "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_1304_3992_amd", "csrc"),
                    os.path.join(ROOT, "tests", "median_bits_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert r.stdout.count(" 0 mismatches") == 4
