"""Build ``libtetra.so`` (the C-ABI library) in-tree with hipcc for gfx950, and the benchmark's
measurement helper ``libtetra_probe.so`` (not part of the DOS library).

Each HIP source is compiled to an object in parallel, then each library's objects are linked.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtetra.so")
PROBE_LIB = os.path.join(PKG, "libtetra_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def probe_sources():
    return sorted(glob.glob(os.path.join(CSRC, "probe", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd[-3:])}")


def build(extra_flags=(), verbose: bool = False) -> str:
    """Compile every HIP source into ``paper_1710_10789_amd/libtetra.so`` (and the probe sources into
    ``libtetra_probe.so``); returns the DOS library's path."""
    with tempfile.TemporaryDirectory(prefix="tetra_build_") as tmpdir:
        libs = {LIB: [], PROBE_LIB: []}
        cmds = []
        for lib, srcs in ((LIB, sources()), (PROBE_LIB, probe_sources())):
            for src in srcs:
                obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
                libs[lib].append(obj)
                cmds.append([HIPCC, *FLAGS, *extra_flags, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj])
        with ThreadPoolExecutor(max_workers=min(len(cmds), max(1, os.cpu_count() or 1))) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        for lib, objs in libs.items():
            tmp = lib + f".tmp{os.getpid()}"
            _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
            os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(sys.argv[1:], verbose=True))
