"""Host checks of bench.py's contract (no GPU): more than one GPU is refused with a message before
anything touches a device, and a committed traffic record is reported only while the kernel source
hash it was measured on matches the tree (a stale record reads as null, never as a wrong figure)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for argv in (["--gpus", "2"], ["--gpus", "8", "--steps", "1"]):
        res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                             timeout=120, cwd=ROOT)
        assert res.returncode != 0
        assert "one GPU" in res.stderr
        assert res.stdout.strip() == ""


def test_traffic_records_match_the_sources():
    sys.path.insert(0, ROOT)
    import bench

    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    for kernel in bench.KERNEL_SOURCES:
        assert kernel in rec, kernel
        assert rec[kernel]["bytes_per_launch"] == rec[kernel]["read_bytes"] + rec[kernel]["write_bytes"]
        fresh = rec[kernel]["source_sha"] == bench.kernel_source_hash(kernel)
        assert bench.load_traffic(kernel) == (rec[kernel]["bytes_per_launch"] if fresh else None), kernel


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    a = bench._code_only("int f(int x) {  // add one\n  return x + 1; /* done */\n}\n")
    b = bench._code_only("int f(int x) {\n  return x + 1;\n}\n")
    c = bench._code_only("int f(int x) {\n  return x + 2;\n}\n")
    assert a == b and a != c
