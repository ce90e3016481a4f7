"""The kernels' per-tetrahedron arithmetic (``tetra_device.h``: sort, windows, case split, corner weights
in their local frames, the middle case's cubic form, the range-end adjoint from power sums of the
loss gradient, and the integrated weights of the number of states with their step indices, on the
grid and on the midpoints between grid energies) built for the host with g++ and checked against the
FP64 oracle's corner weights and dual-number energy derivatives on random tetrahedra, generic and
with nearly equal corner energies.
No GPU needed; the harness is test code only.

Bounds (FP32 arithmetic against FP64): corner weights within 1e-5 of the tetrahedron's largest
weight; a case range's energy gradient within 5e-4 of the sum of its per-energy |derivatives|, and its
weight gradient within 1e-5 of sum_j |G| |g|; integrated weights within 1e-9 (FP64) and 1e-5 (FP32)
of V_T/(4 V_G),
and their increments over bins 1e3 and 1e5 times narrower than the tetrahedron within 1e-6 of the
tetrahedron's largest increment (a sign or index mistake in any term gives O(1))."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_10789_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host", "device_math_check.cpp")


@pytest.fixture(scope="module")
def harness(tmp_path_factory, oracle_lib):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("dmc") / "device_math_check")
    odir = os.path.dirname(oracle_lib.build())
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC, HARNESS,
           "-o", exe, "-L", odir, "-ltetra_oracle", f"-Wl,-rpath,{odir}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return exe


def test_corner_weights_and_moment_adjoint_against_oracle(harness):
    res = subprocess.run([harness, "20000"], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr
    rows = {}
    for line in res.stdout.split("\n"):
        parts = line.split()
        if len(parts) == 6:
            rows[parts[0]] = (int(parts[1]), *map(float, parts[2:]))
    print(res.stdout)
    nos = {}
    for line in res.stdout.split("\n"):
        parts = line.split()
        if len(parts) == 4:
            nos[parts[0]] = (int(parts[1]), float(parts[2]), int(parts[3]))
    assert set(nos) == {"nos", "nos_half", "nos32", "nos32_half"}
    for grid, (npts, err, bad) in nos.items():
        assert npts > 100000, grid
        # integrated weights relative to V_T/(4 V_G): FP64 and FP32 evaluation
        assert err <= (1e-5 if grid.startswith("nos32") else 1e-9), (grid, err)
        assert bad == 0, grid  # number-of-states steps at the right grid indices
    inc = {}
    for line in res.stdout.split("\n"):
        parts = line.split()
        if len(parts) == 3 and parts[0].startswith("inc_"):
            inc[parts[0]] = (int(parts[1]), float(parts[2]))
    assert set(inc) == {"inc_1e3", "inc_1e5"}
    for grid, (ninc, err) in inc.items():
        assert ninc > 1000, grid
        assert err <= 1e-6, (grid, err)  # increments on bins 1e3 and 1e5 times finer than the tetrahedron
    assert set(rows) == {"first", "middle", "third"}
    for case, (n, werr, gen, deg, berr) in rows.items():
        assert n > 1000, case
        assert werr <= 1e-5, (case, werr)
        assert gen <= 5e-4 and deg <= 5e-4, (case, gen, deg)
        assert berr <= 1e-5, (case, berr)
