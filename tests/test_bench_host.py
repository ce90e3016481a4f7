"""Host checks of bench.py's contract (no GPU): more than one GPU is refused with a message before
anything touches a device, and a committed traffic record is reported only while the kernel source
hash it was measured on matches the tree and for the launch configuration (tile shape) it was
measured with (a stale or foreign record reads as null, never as a wrong figure)."""
import json
import os
import subprocess
import sys

import pytest

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
        assert kernel in rec and isinstance(rec[kernel], list) and rec[kernel], kernel
        configs = [r.get("config") for r in rec[kernel]]
        assert len({json.dumps(c, sort_keys=True) for c in configs}) == len(configs), kernel  # one per config
        for r in rec[kernel]:
            assert r["bytes_per_launch"] == pytest.approx(r["read_bytes"] + r["write_bytes"], rel=1e-12)
            fresh = r["source_sha"] == bench.kernel_source_hash(kernel)
            if r.get("config") is not None:
                assert bench.load_traffic(kernel, r["config"]) == (r["bytes_per_launch"] if fresh else None), kernel
                assert bench.load_traffic(kernel, {"tile": [3, 3, 3]}) is None  # no such launch configuration


def test_traffic_records_are_kept_per_configuration(tmp_path):
    """summarize_profiles replaces the record of the profiled configuration and keeps the others."""
    sys.path.insert(0, ROOT)
    import bench

    out = tmp_path / "traffic.json"
    old = {"dos_backward_kernel": [{"source_sha": "x", "config": {"tile": [4, 4, 16]}, "bytes_per_launch": 3.0,
                                    "read_bytes": 1.0, "write_bytes": 2.0},
                                   {"source_sha": "x", "config": {"tile": [8, 4, 8]}, "bytes_per_launch": 7.0,
                                    "read_bytes": 3.0, "write_bytes": 4.0}]}
    out.write_text(json.dumps(old))
    kt, fe, wr, cf, cw = (tmp_path / n for n in ("kt", "fe", "wr", "cf", "cw"))
    for d in (kt, fe, wr, cf, cw):
        d.mkdir()
    (kt / "kt_kernel_stats.csv").write_text("Name,Calls,AverageNs,MinNs,MaxNs\nk,1,1,1,1\n")
    hdr = "Kernel_Name,Counter_Name,Counter_Value\n"
    (cf / "cf_counter_collection.csv").write_text(hdr + f"copyBuffer,FETCH_SIZE,{64 * 1024 * 4 / 2}\n")
    (cw / "cw_counter_collection.csv").write_text(hdr + f"copyBuffer,WRITE_SIZE,{64 * 1024 * 4}\n")
    (fe / "f_counter_collection.csv").write_text(hdr + "dos_backward_kernel<8>,FETCH_SIZE,10\n")
    (wr / "w_counter_collection.csv").write_text(hdr + "dos_backward_kernel<8>,WRITE_SIZE,20\n")
    bench.summarize_profiles(str(kt), str(fe), str(wr), str(cf), str(cw), out_json=str(out),
                             source_shas={"dos_backward_kernel": "y"},
                             configs={"dos_backward_kernel": {"tile": [8, 4, 8]}})
    recs = json.loads(out.read_text())["dos_backward_kernel"]
    assert [r["config"]["tile"] for r in recs] == [[4, 4, 16], [8, 4, 8]]
    assert recs[0]["bytes_per_launch"] == 3.0 and recs[1]["source_sha"] == "y"
    assert recs[1]["read_bytes"] == 10 * 1024 * 2 and recs[1]["write_bytes"] == 20 * 1024


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    a = bench._code_only("int f(int x) {  // add one\n  return x + 1; /* done */\n}\n")
    b = bench._code_only("int f(int x) {\n  return x + 1;\n}\n")
    c = bench._code_only("int f(int x) {\n  return x + 2;\n}\n")
    assert a == b and a != c
