"""Sanitizer builds of the host code, on the CPU (no GPU):

* the FP64 oracle (``oracle/tetra_oracle.cpp``) built with g++ ``-fsanitize=address,undefined`` and
  driven through every exported function on ragged grids, a non-finite band, degenerate corners,
  one and three OpenMP threads, and invalid arguments (``tests/host/oracle_sanitize.cpp``);
* the C ABI's host code: every library source compiled with AddressSanitizer and
  UndefinedBehaviorSanitizer on the host side only (device code is built as usual and never runs),
  linked with ``tests/host/abi_sanitize.cpp``, which calls every entry point with one defect at a
  time and checks the documented status, and every size query.

Either run stops at the first report (``-fno-sanitize-recover=all``; leak checking on), so a pass
means no out-of-bounds access, use after free, undefined arithmetic or leak on these paths."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_10789_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _clean(res):
    text = res.stdout + res.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text and "LeakSanitizer" not in text, text[-4000:]
    assert res.returncode == 0, text[-4000:]
    return res.stdout


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "oracle_san")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "tetra_oracle.cpp"),
           os.path.join(ROOT, "tests", "host", "oracle_sanitize.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    out = _clean(subprocess.run([exe], capture_output=True, text=True, timeout=600, env=SAN_ENV))
    assert out.startswith("ok ")


def test_abi_host_code_under_address_and_undefined_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("needs the ROCm compilers")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
             # host side only: the device code is compiled as usual and never runs here
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-I", INCLUDE, "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        res = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(len(srcs), max(1, len(os.sched_getaffinity(0))))) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "abi_san")
    link = [CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-I", INCLUDE, os.path.join(ROOT, "tests", "host", "abi_sanitize.cpp"), *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    res = subprocess.run(link, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    out = _clean(subprocess.run([exe], capture_output=True, text=True, timeout=300, env=SAN_ENV))
    assert out.startswith("ok ") and int(out.split()[1]) >= 100
