"""The adjoint's two-phase output indexing (``tetra_faces.h``), built for the host with g++: face slots
are a bijection onto [0, face_count) for every tile shape, and scattering random per-(cube, corner)
values by tiles (complete points stored, face points into the tile's slots) then gathering every
other grid point from the tiles ``face_tiles`` names reproduces the direct sum over each point's
eight cubes on periodic grids of two to five tiles per axis (an off-by-one in a face offset, a wrong
neighbouring tile or a missed point gives an O(1) error or a NaN). No GPU needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_10789_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host", "face_check.cpp")


def test_face_slots_scatter_and_gather(tmp_path):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "face_check")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC, HARNESS, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(res.stdout)
    lines = [l.split() for l in res.stdout.split("\n") if l.startswith("shape")]
    assert len(lines) == 18
    for parts in lines:
        assert float(parts[8]) <= 1e-12 and parts[9] == "1", parts
    assert res.returncode == 0
