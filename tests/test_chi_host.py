"""The susceptibility kernel's per-tetrahedron arithmetic (``tetra_chi_device.h``: clipping at the two
occupation boundaries into sub-tetrahedra, their volumes, their vertices sorted with their barycentric
rows and the weights formed at them, with the corner weights of ``tetra_device.h``) built for the host
with g++ and checked against the FP64 oracle's one-tetrahedron spectral weight on random tetrahedra,
generic, with nearly equal corners, and with a region that is the whole tetrahedron (the kernel's
unclipped path). No GPU needed; the harness is test code only.

Bound: |S_fp32 - S_oracle| <= 1e-4 of vol * max W / (max - min of eps' - eps), the size of one
tetrahedron's contribution (a wrong piece, sign or vertex order gives O(1))."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_10789_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host", "chi_check.cpp")


def test_chi_clipping_against_oracle(tmp_path, oracle_lib):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "chi_check")
    odir = os.path.dirname(oracle_lib.build())
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC, HARNESS,
           "-o", exe, "-L", odir, "-ltetra_oracle", f"-Wl,-rpath,{odir}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    res = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    parts = res.stdout.split()
    print(res.stdout)
    cases, nonzero, worst, whole = int(parts[1]), int(parts[2]), float(parts[3]), int(parts[4])
    assert cases > 50000 and nonzero > 20000 and whole > 5000
    assert worst <= 1e-4
