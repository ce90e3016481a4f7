#!/usr/bin/env python3
"""Benchmark of the tetrahedron-DOS hot path on one MI355X.

Workload (default): 64^3 periodic k-grid (1,572,864 tetrahedra), 8 bands x 8 orbitals, 1000
equidistant energies, FP32 band energies and orbital weights in structure-of-arrays layout, from the
seeded random tight-binding model in ``synth`` (a stand-in for the paper's FeSe model, whose hopping
parameters are not published). Inputs are resident in HBM before timing starts.

One step = one forward pass (DOS) plus one backward pass (gradients with respect to band energies
and orbital weights for G = 2 (DOS - DOS_target), the loss of the differentiation workload). The
headline value counts dense-equivalent tetrahedron-band-energy updates, N_tet * nb * ne per pass,
the work the paper's kernel visits; the JSON line also carries the plain-forward rate, the
in-window update rate, a roofline object for the dominant kernel and the FP64 oracle's CPU rate on a
bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fwdbwd|fwd] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
WORKLOAD = "k64_b8_e1000"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


KERNEL_SOURCES = {
    "dos_forward_kernel": ("tetra_forward.hip", "tetra_device.h", "tetra_internal.h", "tetra_weights.h"),
    # the adjoint pass: dos_backward_kernel and its gather pass, both in tetra_backward.hip
    "dos_backward_kernel": ("tetra_backward.hip", "tetra_device.h", "tetra_faces.h", "tetra_internal.h",
                            "tetra_weights.h"),
    "nos_kernel": ("tetra_nos.hip", "tetra_nos_device.h", "tetra_device.h", "tetra_internal.h", "tetra_weights.h"),
    "chi_kernel": ("tetra_chi.hip", "tetra_chi_device.h", "tetra_device.h", "tetra_internal.h", "tetra_weights.h"),
}


def _code_only(text: str) -> str:
    """C++ source without comments and blank space, so that a comment edit keeps a traffic record."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(kernel: str, read=None) -> str:
    """Hash of the code a kernel is built from (comments ignored); a traffic record is used only while
    it matches. ``read(name)`` returns a source file's text (default: the files in the tree)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        if read is None:
            with open(os.path.join(ROOT, "paper_1710_10789_amd", "csrc", name), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(name)
        h.update(name.encode())
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def table1_offsets():
    # Table I (Sec. III.B), corner label L = 1 + o1 + 2*o2 + 4*o3
    rows = [(1, 2, 3, 6), (2, 3, 4, 6), (1, 3, 5, 6), (3, 4, 6, 8), (3, 5, 6, 7), (3, 6, 7, 8)]
    return [[((L - 1) & 1, ((L - 1) >> 1) & 1, ((L - 1) >> 2) & 1) for L in r] for r in rows]


def count_window_updates(eps, grid, e0, de, ne):
    """Number of (tetrahedron, band, energy) triples with E1 < E_j < E4: the in-window work."""
    n1, n2, n3 = grid
    nb = eps.shape[0]
    e = eps.reshape(nb, n1, n2, n3).astype(np.float64)
    total = 0
    for tet in table1_offsets():
        lo = None
        hi = None
        for o in tet:
            c = np.roll(e, shift=(-o[0], -o[1], -o[2]), axis=(1, 2, 3))
            lo = c if lo is None else np.minimum(lo, c)
            hi = c if hi is None else np.maximum(hi, c)
        ok = np.isfinite(lo) & np.isfinite(hi)
        lo, hi = lo[ok], hi[ok]
        # first j with E_j > lo, last j with E_j < hi; refine the float guesses exactly
        jlo = np.clip(np.floor((lo - e0) / de), 0, ne).astype(np.int64)
        jlo -= (jlo > 0) & (e0 + (jlo - 1) * de > lo)
        jlo += (jlo < ne) & (e0 + jlo * de <= lo)
        jhi = np.clip(np.ceil((hi - e0) / de), -1, ne - 1).astype(np.int64)
        jhi += (jhi < ne - 1) & (e0 + (jhi + 1) * de < hi)
        jhi -= (jhi >= 0) & (e0 + jhi * de >= hi)
        total += int(np.maximum(jhi - jlo + 1, 0).sum())
    return total


def algorithmic_flops(uwin, norb):
    """Per in-window update: forward 4*norb FMAs + 4 corner cubics (8*norb + 24 flops); backward the
    orbital sums s_c and dL/db (16*norb), 4 weights (24), 16 cubic partials (96), a 16-term
    contraction (32)."""
    return uwin * (8 * norb + 24), uwin * (16 * norb + 152)


def count_step_updates(eps, grid, e0, de, ne, joff=0.0):
    """Number of (tetrahedron, band, grid index) triples at which a tetrahedron-band's number of states
    changes on the grid E_j = e0 + (j + joff) de, j = 0..ne-1: from the first E_j > E1 to the first
    E_j >= E4, clipped to the grid (everything below the grid counts once, at j = 0)."""
    n1, n2, n3 = grid
    nb = eps.shape[0]
    e = eps.reshape(nb, n1, n2, n3).astype(np.float64)
    origin = e0 + joff * de
    total = 0
    for tet in table1_offsets():
        lo = None
        hi = None
        for o in tet:
            c = np.roll(e, shift=(-o[0], -o[1], -o[2]), axis=(1, 2, 3))
            lo = c if lo is None else np.minimum(lo, c)
            hi = c if hi is None else np.maximum(hi, c)
        ok = np.isfinite(lo) & np.isfinite(hi)
        lo, hi = lo[ok], hi[ok]
        # ja: first j with E_j > lo; js: first j with E_j >= hi (clipped to [-1, ne] before refining)
        ja = np.clip(np.floor((lo - origin) / de), -1, ne).astype(np.int64)
        ja += (origin + ja * de <= lo)
        ja -= (origin + (ja - 1) * de > lo)
        js = np.clip(np.ceil((hi - origin) / de), -1, ne).astype(np.int64)
        js += (origin + js * de < hi)
        js -= (origin + (js - 1) * de >= hi)
        js0 = np.maximum(js, 0)
        ja0 = np.minimum(np.maximum(ja, 0), js0)
        total += int(np.maximum(np.minimum(js0, ne - 1) - ja0 + 1, 0).sum())
    return total


def nos_flops(ustep, norb):
    """Per number-of-states increment: 4 corners x norb FMAs, 4 corner quartics (4 x 4 FMAs) and 4
    differences: 8*norb + 36 flops."""
    return ustep * (8 * norb + 36)


def algorithmic_bytes(nk, nb, norb, ne):
    fwd = 4 * nk * nb + 4 * nk * nb * norb + 4 * ne * norb
    bwd = fwd + 4 * nk * nb + 4 * nk * nb * norb
    return fwd, bwd


def load_traffic(kernel, config=None):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, if it was profiled with
    the current source and (where given) the same launch configuration; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            recs = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    for rec in recs if isinstance(recs, list) else [recs] if recs else []:
        if rec.get("source_sha") != kernel_source_hash(kernel):
            continue
        if config is not None and rec.get("config") != config:
            continue
        return rec.get("bytes_per_launch")
    return None


def cpu_baseline(eps, w, grid, e0, de, ne, mode, G, gpu_fn):
    """The FP64 oracle timed on every host core available to this process (its forward splits over
    k-slabs, its backward over (band, slab) tasks) on the whole workload, and its forward on one core,
    the mean of five runs as in the paper's CPU protocol (Sec. IV.A)."""
    import oracle

    oracle.build()
    cores = len(os.sched_getaffinity(0))
    n1, n2, n3 = grid
    nb = eps.shape[0]
    dense = 6 * n1 * n2 * n3 * nb * ne
    t0 = time.perf_counter()
    ref, _ = oracle.dos(eps, w, grid, e0, de, ne, nthreads=cores)
    t1 = time.perf_counter()
    if mode == "fwdbwd":
        oracle.dos_backward(eps, w, grid, e0, de, G, nthreads=cores)
    t2 = time.perf_counter()
    got = gpu_fn()
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"[bench] oracle on {cores} threads: fwd {t1 - t0:.2f} s, bwd {t2 - t1:.2f} s", file=sys.stderr, flush=True)
    t1s = []
    for _ in range(5):
        t = time.perf_counter()
        oracle.dos(eps, w, grid, e0, de, ne, nthreads=1)
        t1s.append(time.perf_counter() - t)
        print(f"[bench] one-core oracle forward {t1s[-1]:.2f} s", file=sys.stderr, flush=True)
    return {
        "value": dense / (t2 - t0),
        "unit": "updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"the whole workload, one {'forward + backward' if mode == 'fwdbwd' else 'forward'} pass "
                  f"(fwd {t1 - t0:.2f} s, bwd {t2 - t1:.2f} s), FP64, {cores} threads",
        "fwd_value": dense / (t1 - t0),
        "gpu_fwd_err_vs_oracle": err,
        "single_core_fwd_s": float(np.mean(t1s)),
        "single_core_fwd_runs_s": [float(x) for x in t1s],
    }


def _read_csv(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def launch_configs(rec):
    """Launch configuration per kernel of a bench record (what its traffic figures depend on)."""
    cfg = rec.get("config", {})
    out = {}
    if "tile_forward" in cfg:
        out["dos_forward_kernel"] = {"tile": cfg["tile_forward"]}
    if "tile_backward" in cfg:
        out["dos_backward_kernel"] = {"tile": cfg["tile_backward"]}
    return out


def summarize_profiles(kt_dir, fetch_dir=None, write_dir=None, copy_fetch_dir=None, copy_write_dir=None,
                       command="", out_json=None, source_shas=None, configs=None):
    """Markdown summary of rocprofv3 output (kernel-trace stats, and HBM bytes from FETCH_SIZE /
    WRITE_SIZE scaled by what the same counters read for a device copy of known size)."""
    lines = ["| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in _read_csv(glob.glob(os.path.join(kt_dir, "*kernel_stats.csv"))[0]):
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    traffic = {}
    if fetch_dir and write_dir and copy_fetch_dir and copy_write_dir:
        def per_kernel(d, counter):
            acc = {}
            for r in _read_csv(glob.glob(os.path.join(d, "*counter_collection.csv"))[0]):
                if r["Counter_Name"] == counter:
                    acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
            return {k: sum(v) / len(v) for k, v in acc.items()}

        cf = per_kernel(copy_fetch_dir, "FETCH_SIZE")
        cw = per_kernel(copy_write_dir, "WRITE_SIZE")
        ck = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()][0]
        copy_bytes = 64 * 1024 * 1024 * 4
        f_fetch = copy_bytes / (cf[ck] * 1024)
        f_write = copy_bytes / (cw[ck] * 1024)
        fe = per_kernel(fetch_dir, "FETCH_SIZE")
        wr = per_kernel(write_dir, "WRITE_SIZE")
        lines += ["", f"Copy calibration: a 256 MiB device copy reads FETCH_SIZE {cf[ck]:.0f} KiB "
                      f"(factor {f_fetch:.3f}) and WRITE_SIZE {cw[ck]:.0f} KiB (factor {f_write:.3f}).", "",
                  "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MB | HBM write MB |", "|---|---|---|---|---|"]
        for k in fe:
            if k not in wr:
                continue
            rd, wt = fe[k] * 1024 * f_fetch, wr[k] * 1024 * f_write
            lines.append(f"| `{k[:90]}` | {fe[k]:.0f} | {wr[k]:.0f} | {rd / 1e6:.2f} | {wt / 1e6:.2f} |")
            for short, pat in (("dos_forward_kernel", "dos_forward_kernel"), ("dos_backward_kernel", "dos_backward_kernel"),
                               ("dos_backward_kernel", "bwd_gather_kernel"), ("nos_kernel", "nos_kernel"),
                               ("chi_kernel", "chi_kernel")):
                if pat in k:  # the kernels launched by one call add up (instantiations, gather pass)
                    sha = (source_shas or {}).get(short) or kernel_source_hash(short)
                    rec = traffic.setdefault(short, {"source_sha": sha, "config": (configs or {}).get(short),
                                                     "bytes_per_launch": 0.0, "read_bytes": 0.0, "write_bytes": 0.0})
                    rec["bytes_per_launch"] += rd + wt
                    rec["read_bytes"] += rd
                    rec["write_bytes"] += wt
    if out_json and traffic:
        try:  # keep the records of kernels and launch configurations this run did not profile
            with open(out_json) as f:
                merged = json.load(f)
        except (OSError, ValueError):
            merged = {}
        for short, rec in traffic.items():
            old = merged.get(short)
            old = old if isinstance(old, list) else [old] if old else []
            merged[short] = [r for r in old if r.get("config") != rec["config"]] + [rec]
        with open(out_json, "w") as f:
            json.dump(merged, f, indent=1)
    text = "\n".join(lines)
    if command:
        text = f"Command: `{command}`\n\n" + text
    print(text)
    return text


def _time_events(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        fn()
    ev[1].record()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / steps


def precision_measurement(args, torch, tetra, dev, with_oracle=True):
    """128^3 grid, 16 bands x 16 orbitals, 2000 energies: plain FP32, FP16 weights with a per-band scale,
    and the exact accumulation of each; with ``with_oracle``, errors against the FP64 oracle (FP16
    against the oracle on both the FP32 and the dequantised weights). Returns a dict."""
    from paper_1710_10789_amd import tune

    c = synth.config("k128_b16_e2000")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    t0 = time.perf_counter()
    eps_np, w_np = synth.band_structure(norb, c["seed"], grid, progress=True)
    t_gen = time.perf_counter() - t0
    e0, de = synth.energy_grid(eps_np, ne)
    nb, nk = eps_np.shape
    dense = 6 * nk * nb * ne
    print(f"[precision] band structure ready ({t_gen:.1f} s)", file=sys.stderr, flush=True)
    uwin = count_window_updates(eps_np, grid, e0, de, ne)
    eps = torch.from_numpy(eps_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    w16, scale = tetra.half_weights(w)
    out = torch.empty((ne, norb), device=dev)
    tile, _ = tune.tune_forward(eps, w16, grid, e0, de, ne, w_scale=scale, reps=2)
    ws = torch.empty(tetra.forward_workspace_bytes(grid, nb, norb, e0, de, ne, exact=True), dtype=torch.uint8,
                     device=dev)
    runs = {
        "fp32": lambda: tetra.dos_forward(eps, w, grid, e0, de, ne, out=out, tile=tile),
        "fp16": lambda: tetra.dos_forward(eps, w16, grid, e0, de, ne, w_scale=scale, out=out, tile=tile),
        "fp16_exact": lambda: tetra.dos_forward(eps, w16, grid, e0, de, ne, w_scale=scale, out=out, exact=True,
                                                tile=tile, workspace=ws),
        "fp32_exact": lambda: tetra.dos_forward(eps, w, grid, e0, de, ne, out=out, exact=True, tile=tile,
                                                workspace=ws),
    }
    print("[precision] timing", file=sys.stderr, flush=True)
    ms = {k: _time_events(torch, f, args.steps, args.warmup) for k, f in runs.items()}
    results = {}
    for k, f in runs.items():
        f()
        torch.cuda.synchronize()
        results[k] = out.cpu().numpy().astype(np.float64)
    rec = {
        "workload": "k128_b16_e2000: 128^3 periodic k-grid, 16 bands x 16 orbitals, 2000 energies",
        "dense_updates_per_pass": dense,
        "in_window_updates_per_pass": uwin,
        "tile": list(tetra.TILE_SHAPES[tile]),
        "host_eigh_s": t_gen,
        "ms": ms,
        "exact_over_plain": {"fp32": ms["fp32_exact"] / ms["fp32"], "fp16": ms["fp16_exact"] / ms["fp16"]},
        "updates_per_s": {k: dense / (v * 1e-3) for k, v in ms.items()},
        "hbm_gbs_algorithmic": {"fp32": (4 * nk * nb * (1 + norb)) / (ms["fp32"] * 1e-3) / 1e9,
                                "fp16": (4 * nk * nb + 2 * nk * nb * norb) / (ms["fp16"] * 1e-3) / 1e9},
    }
    if with_oracle:
        import oracle

        oracle.build()
        cores = len(os.sched_getaffinity(0))
        print(f"[precision] FP64 oracle on {cores} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ref, _ = oracle.dos(eps_np, w_np, grid, e0, de, ne, nthreads=cores)
        t_or = time.perf_counter() - t0
        deq = (w16.float() * scale[:, None, None]).cpu().numpy()
        del w_np
        ref_dq, _ = oracle.dos(eps_np, deq, grid, e0, de, ne, nthreads=cores)
        del deq
        err = {k: float(np.abs(v - ref).max() / np.abs(ref).max()) for k, v in results.items()}
        for k in ("fp16", "fp16_exact"):
            err[k + "_vs_dequantised"] = float(np.abs(results[k] - ref_dq).max() / np.abs(ref_dq).max())
        rec["error_vs_fp64_oracle"] = err
        rec["cpu_baseline"] = {"value": dense / t_or, "unit": "updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"the whole workload, one forward pass, FP64 ({t_or:.1f} s)"}
    del eps, w, w16, scale, out, ws
    torch.cuda.empty_cache()
    return rec


def bench_precision(args, torch, tetra, dev):
    """The precision workload on its own JSON line (value: the FP16 + exact forward)."""
    p = precision_measurement(args, torch, tetra, dev, with_oracle=not args.no_cpu_baseline)
    ms = p["ms"]["fp16_exact"]
    rec = {
        "metric": "tetra-band-energy updates/s, precision variant (FP16 weights, exact accumulation)",
        "value": p["dense_updates_per_pass"] / (ms * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "dtype": "f32 math, f16 weights",
        "data": "synthetic (seeded random 16-orbital tight-binding model)",
        "config": {"workload": p["workload"], "dense_updates_per_pass": p["dense_updates_per_pass"],
                   "in_window_updates_per_pass": p["in_window_updates_per_pass"], "tile": p["tile"],
                   "host_eigh_s": p["host_eigh_s"]},
    }
    for k in ("ms", "exact_over_plain", "updates_per_s", "hbm_gbs_algorithmic", "error_vs_fp64_oracle",
              "cpu_baseline"):
        if k in p:
            rec[k] = p[k]
    print(json.dumps(rec), flush=True)


def worst_case_forward_ms(torch, tetra, eps_np, w_np, grid, e0, de, ne, tile, steps=7):
    """The paper's worst case (Sec. IV.A, GPU setup excluded): host-to-device copies of the inputs from
    pinned host memory, the forward, and the device-to-host copy of the DOS; per-call event times over
    ``steps`` calls: the paper's statistic (mean of the five shortest of seven) and the median."""
    dev = torch.device("cuda:0")
    h_eps = torch.empty(eps_np.shape, dtype=torch.float32, pin_memory=True)
    h_w = torch.empty(w_np.shape, dtype=torch.float32, pin_memory=True)
    h_eps.numpy()[...] = eps_np
    h_w.numpy()[...] = w_np
    nb, norb = w_np.shape[0], w_np.shape[1]
    h_dos = torch.empty((ne, norb), dtype=torch.float32, pin_memory=True)
    d_eps = torch.empty(eps_np.shape, dtype=torch.float32, device=dev)
    d_w = torch.empty(w_np.shape, dtype=torch.float32, device=dev)
    d_dos = torch.empty((ne, norb), dtype=torch.float32, device=dev)

    def call():
        d_eps.copy_(h_eps, non_blocking=True)
        d_w.copy_(h_w, non_blocking=True)
        tetra.dos_forward(d_eps, d_w, grid, e0, de, ne, out=d_dos, tile=tile)
        h_dos.copy_(d_dos, non_blocking=True)

    call()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        call()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    bytes_moved = 4 * (eps_np.size + w_np.size + ne * norb)
    srt = np.sort(ts)
    return {"mean_5_shortest_of_7": float(srt[:5].mean()), "median": float(np.median(ts)),
            "pcie_bytes": bytes_moved,
            "what": "H2D of eps and w from pinned host memory + forward + D2H of dos, per call"}


def bench_paper_shape(args, torch, tetra, dev):
    """The paper's largest benchmark shape (Sec. IV, Table II): 60 x 60 x 10 k-points, 8 bands and 8
    orbitals of the seeded model (the paper's FeSe model has no published parameters), 1024 energies;
    forward only, inputs resident (the paper's best case). Context, not the headline metric."""
    from paper_1710_10789_amd import tune

    c = synth.config("k60x60x10_b8_e1024")
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps_np, w_np = synth.band_structure(norb, c["seed"], grid)
    e0, de = synth.energy_grid(eps_np, ne)
    nb, nk = eps_np.shape
    dense = 6 * nk * nb * ne
    eps = torch.from_numpy(eps_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    out = torch.empty((ne, norb), device=dev)
    tile, _ = tune.tune_forward(eps, w, grid, e0, de, ne, reps=3)
    ms = _time_events(torch, lambda: tetra.dos_forward(eps, w, grid, e0, de, ne, out=out, tile=tile), args.steps,
                      args.warmup)
    print(json.dumps({
        "metric": "tetra-band-energy updates/s, the paper's 60x60x10 shape, forward",
        "value": dense / (ms * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic (seeded random 8-orbital tight-binding model)",
        "config": {"workload": "k60x60x10_b8_e1024: 60 x 60 x 10 periodic k-grid, 8 bands x 8 orbitals, 1024 energies",
                   "dense_updates_per_pass": dense, "in_window_updates_per_pass": count_window_updates(eps_np, grid, e0, de, ne),
                   "tile": list(tetra.TILE_SHAPES[tile])},
        "context": "the paper reports 732.0 ms (kernels only) for this k-grid size with 5 of 8 orbitals on a GTX 970",
    }), flush=True)


def nos_record(args, torch, tetra, dev, with_oracle=True):
    """Number of states and bin-averaged DOS at the headline shape (64^3 x 8 bands x 8 orbitals x 1000
    energies): one pass of each, inputs resident; tile shape by a short sweep outside the timed
    region. The FP64 oracle (dense in energy) is timed on the whole workload."""
    c = synth.config(WORKLOAD)
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps_np, w_np = synth.band_structure(norb, c["seed"], grid)
    e0, de = synth.energy_grid(eps_np, ne)
    nb, nk = eps_np.shape
    dense = 6 * nk * nb * ne
    u_nos = count_step_updates(eps_np, grid, e0, de, ne)
    u_bin = count_step_updates(eps_np, grid, e0, de, ne + 1, joff=-0.5)
    eps = torch.from_numpy(eps_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    out_n = torch.empty((ne, norb), device=dev)
    out_b = torch.empty((ne, norb), device=dev)
    if args.tiles:  # every launch of the run with the given shape (for profiles)
        tile, sweep = int(args.tiles.split(",")[0]), None
    else:
        sweep = {}
        for r in range(2):  # best of two sweeps in opposite orders
            for t in (range(6) if r == 0 else range(5, -1, -1)):
                ms_t = _time_events(torch, lambda t=t: tetra.dos_binned(eps, w, grid, e0, de, ne, out=out_b, tile=t),
                                    3, 1)
                sweep[t] = min(sweep.get(t, float("inf")), ms_t)
        tile = min(sweep, key=sweep.get)
    stream = torch.cuda.current_stream(dev)
    runs = {"nos": lambda: tetra.nos_forward(eps, w, grid, e0, de, ne, out=out_n, tile=tile),
            "binned": lambda: tetra.dos_binned(eps, w, grid, e0, de, ne, out=out_b, tile=tile)}
    ms = {}
    for k, f in runs.items():
        for _ in range(args.warmup):
            f()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        for e in ev:
            e[0].record(stream)
            f()
            e[1].record(stream)
        torch.cuda.synchronize()
        ms[k] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    flops = nos_flops(u_bin, norb)
    achieved = flops / (ms["binned"] * 1e-3) / 1e12
    rec = {
        "metric": "tetra-band-energy updates/s, number of states at 64^3 k, 8 bands, 1000 E",
        "value": dense / (ms["nos"] * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms["nos"],
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic (seeded random 8-orbital tight-binding model; eigh on the host, untimed)",
        "config": {"workload": f"{WORKLOAD}: 64^3 periodic k-grid, 8 bands x 8 orbitals, 1000 energies, FP32 SoA",
                   "dense_updates_per_pass": dense, "step_updates_nos": u_nos, "step_updates_binned": u_bin,
                   "tile": list(tetra.TILE_SHAPES[tile])},
        "ms": ms,
        "binned_updates_per_s": dense / (ms["binned"] * 1e-3),
        "roofline": {"bound": "alu", "kernel": "nos_kernel, both precisions (bin averages; events include the zero fill)",
                     "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": load_traffic("nos_kernel"),
                     "algorithmic_flops_per_launch": flops, "avg_launch_ms": ms["binned"]},
        "tile_sweep_ms": sweep,
        "kernel_source_sha": {"nos_kernel": kernel_source_hash("nos_kernel")},
    }
    if with_oracle:
        import oracle

        oracle.build()
        cores = len(os.sched_getaffinity(0))
        print(f"[nos] FP64 oracle on {cores} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ref = oracle.nos(eps_np, w_np, grid, e0, de, ne, nthreads=cores)
        t_or = time.perf_counter() - t0
        runs["nos"]()
        torch.cuda.synchronize()
        got = out_n.cpu().numpy().astype(np.float64)
        rec["cpu_baseline"] = {"value": dense / t_or, "unit": "updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"the whole workload, one number-of-states pass ({ne} energies), FP64 "
                                         f"({t_or:.1f} s)"}
        rec["nos_err_vs_oracle"] = float(np.abs(got - ref).max() / np.abs(ref).max())
    return rec


def bench_nos(args, torch, tetra, dev):
    print(json.dumps(nos_record(args, torch, tetra, dev, with_oracle=not args.no_cpu_baseline)), flush=True)


def chi_record(args, torch, tetra, dev, with_oracle=True):
    """Susceptibility spectral weight at the headline model: 64^3 grid, 8 bands x 8 orbitals, transfer
    q = (16, 16, 0) grid steps, 500 transfer energies from 0 to the band width, Fermi energy at half
    filling; every band pair. One JSON line (not the headline metric)."""
    c = synth.config("chi_k64_b8_w500")
    grid, norb, nw, q = c["grid"], c["norb"], c["nw"], c["q"]
    eps_np, w_np = synth.band_structure(norb, c["seed"], grid)
    ef, w0, dw = synth.chi_grid(eps_np, nw)
    nb, nk = eps_np.shape
    dense = 6 * nk * nb * nb * nw
    eps = torch.from_numpy(eps_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    out = torch.empty((nw, norb), device=dev)
    # the first pass's workspace (per-(tile, band) energy ranges), allocated once, outside the timed region
    ws = torch.empty(max(tetra.chi_workspace_bytes(grid, nb, norb, w0, dw, nw, tile=t)
                         for t in range(len(tetra.TILE_SHAPES))), dtype=torch.uint8, device=dev)
    # tile shape: each of the six timed (best of three launches), outside the timed region
    times = []
    for tile in range(len(tetra.TILE_SHAPES)):
        times.append(_time_events(torch, lambda: tetra.chi_spectral(eps, w, grid, q, ef, w0, dw, nw, out=out,
                                                                     tile=tile, workspace=ws), 3, 1))
    tile = int(np.argmin(times))
    ms = _time_events(torch, lambda: tetra.chi_spectral(eps, w, grid, q, ef, w0, dw, nw, out=out, tile=tile,
                                                        workspace=ws), args.steps, args.warmup)
    got = out.cpu().numpy().astype(np.float64)
    rec = {
        "metric": "susceptibility spectral-weight (tetrahedron, band pair, transfer energy) updates/s at 64^3, "
                  "8 bands x 8 orbitals, 500 w",
        "value": dense / (ms * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic (seeded random 8-orbital tight-binding model; eigh on the host, untimed)",
        "config": {"workload": "chi_k64_b8_w500: 64^3 periodic k-grid, 8 bands x 8 orbitals, q = (16, 16, 0), "
                               "500 transfer energies, E_F at half filling; tetra_chi_spectral_ws (first pass of "
                               "per-(tile, band) energy ranges, then chi_kernel)",
                   "dense_updates_per_pass": dense, "tile": list(tetra.TILE_SHAPES[tile])},
        "tile_ms": times,
        "kernel_source_sha": {"chi_kernel": kernel_source_hash("chi_kernel")},
    }
    if with_oracle:
        import oracle

        oracle.build()
        cores = len(os.sched_getaffinity(0))
        print(f"[chi] FP64 oracle on {cores} threads", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ref, upd = oracle.chi(eps_np, w_np, grid, q, ef, w0, dw, nw, nthreads=cores)
        t_or = time.perf_counter() - t0
        flops = algorithmic_flops(upd, norb)[0]
        achieved = flops / (ms * 1e-3) / 1e12
        rec["config"]["in_window_updates_per_pass"] = upd
        rec["roofline"] = {"bound": "alu", "kernel": "chi_kernel", "achieved": achieved,
                           "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": load_traffic("chi_kernel"),
                           "algorithmic_flops_per_launch": flops, "avg_launch_ms": ms,
                           "timed_over": "the whole call: zero fill, chi_ranges_kernel (first pass), chi_kernel"}
        rec["error_vs_fp64_oracle"] = float(np.abs(got - ref).max() / np.abs(ref).max())
        rec["cpu_baseline"] = {"value": dense / t_or, "unit": "updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"the whole workload, one pass, FP64 ({t_or:.1f} s)"}
    return rec


def bench_chi(args, torch, tetra, dev):
    print(json.dumps(chi_record(args, torch, tetra, dev, with_oracle=not args.no_cpu_baseline)), flush=True)


def batched_record(args, torch, tetra, dev):
    """32 independently seeded 8-orbital models, cubic grids from {24,32,48,64,96}^3 and 256..2048
    energies, through one persistent launch captured in a HIP graph, tile shapes per problem from the
    autotuner."""
    from paper_1710_10789_amd import tune

    specs = synth.batched_items()
    probs, dense, uwin = [], 0, 0
    t0 = time.perf_counter()
    for seed, grid, ne in specs:
        eps_np, w_np = synth.band_structure(8, seed, grid, progress=True)
        e0, de = synth.energy_grid(eps_np, ne)
        probs.append((torch.from_numpy(eps_np).to(dev), torch.from_numpy(w_np).to(dev), grid, e0, de, ne))
        dense += 6 * eps_np.shape[1] * 8 * ne
        uwin += count_window_updates(eps_np, grid, e0, de, ne)
    t_gen = time.perf_counter() - t0
    tiles = tune.tiles_for_batch(probs)
    ws = torch.empty(tetra.batched_workspace_bytes(probs), dtype=torch.uint8, device=dev)
    outs = [torch.empty((p[5], 8), device=dev) for p in probs]
    tetra.dos_batched(probs, workspace=ws, out=outs, tiles=tiles)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tetra.dos_batched(probs, workspace=ws, out=outs, tiles=tiles)
    torch.cuda.current_stream().wait_stream(s)
    ms_graph = _time_events(torch, g.replay, args.steps, args.warmup)
    ms_eager = _time_events(torch, lambda: tetra.dos_batched(probs, workspace=ws, out=outs, tiles=tiles),
                            args.steps, args.warmup)
    ms_single = _time_events(torch, lambda: [tetra.dos_forward(*p, tile=t) for p, t in zip(probs, tiles)],
                             args.steps, args.warmup)
    return {
        "metric": "tetra-band-energy updates/s, batched (32 models, one persistent graph-captured launch)",
        "value": dense / (ms_graph * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic (32 seeded random 8-orbital tight-binding models)",
        "config": {"workload": "batch32: grids from {24,32,48,64,96}^3, 256..2048 energies",
                   "grids": [sp[1][0] for sp in specs], "energies": [sp[2] for sp in specs],
                   "dense_updates_per_pass": dense, "in_window_updates_per_pass": uwin,
                   "tiles": tiles, "host_eigh_s": t_gen},
        "ms": {"graph": ms_graph, "eager_batched": ms_eager, "one_launch_per_model": ms_single},
    }


def bench_batched(args, torch, tetra, dev):
    print(json.dumps(batched_record(args, torch, tetra, dev)), flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-profiles":
        ap = argparse.ArgumentParser()
        ap.add_argument("--summarize-profiles", action="store_true")
        ap.add_argument("--kt", required=True)
        ap.add_argument("--fetch")
        ap.add_argument("--write")
        ap.add_argument("--copy-fetch")
        ap.add_argument("--copy-write")
        ap.add_argument("--command", default="")
        ap.add_argument("--traffic-json")
        ap.add_argument("--bench-json", help="bench output of the profiled tree (its kernel source hashes)")
        a = ap.parse_args()
        shas = configs = None
        if a.bench_json:
            with open(a.bench_json) as f:
                rec = json.loads(f.read().strip().splitlines()[-1])
            shas = rec.get("kernel_source_sha")
            configs = launch_configs(rec)
        summarize_profiles(a.kt, a.fetch, a.write, a.copy_fetch, a.copy_write, a.command, a.traffic_json, shas,
                           configs)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["fwdbwd", "fwd"], default="fwdbwd")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiles", help="forward,backward tile shape ids (skips the autotuner)")
    ap.add_argument("--no-precision", action="store_true",
                    help="headline run without the extra keys of the other workloads (precision 128^3 x 16 x 16 "
                         "x 2000, batched 32 models, number of states, susceptibility)")
    ap.add_argument("--workload", choices=["headline", "precision", "batched", "paper", "nos", "chi"], default="headline",
                    help="headline: 64^3 x 8 x 8 x 1000 fwd+bwd (the metric); precision: 128^3 x 16 x 16 x 2000 "
                         "with FP16 weights and exact accumulation; batched: 32 models, one persistent launch; "
                         "paper: the paper's 60 x 60 x 10 x 8 x 1024 forward, for context; nos: number of states "
                         "and bin-averaged DOS at the headline shape; chi: susceptibility spectral weight at the "
                         "headline model")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 256 MiB (5 times) to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the tetrahedron DOS path is built and timed on a single "
              "MI355X (--gpus 1); multi-GPU sharding is described, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1710_10789_amd as tetra

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = 64 * 1024 * 1024  # floats: 256 MiB read + 256 MiB written per copy
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}), flush=True)
        return
    if args.workload == "precision":
        return bench_precision(args, torch, tetra, dev)
    if args.workload == "batched":
        return bench_batched(args, torch, tetra, dev)
    if args.workload == "paper":
        return bench_paper_shape(args, torch, tetra, dev)
    if args.workload == "nos":
        return bench_nos(args, torch, tetra, dev)
    if args.workload == "chi":
        return bench_chi(args, torch, tetra, dev)
    c = synth.config(WORKLOAD)
    grid, norb, ne = c["grid"], c["norb"], c["ne"]
    eps_np, w_np = synth.band_structure(norb, c["seed"], grid)
    teps_np, tw_np = synth.band_structure(norb, 1, grid)  # target model of the loss
    e0, de = synth.energy_grid(eps_np, ne)  # the headline workload's own grid; target DOS on it
    nb, nk = eps_np.shape
    n_tet = 6 * nk
    dense = n_tet * nb * ne
    uwin = count_window_updates(eps_np, grid, e0, de, ne)
    f_fwd, f_bwd = algorithmic_flops(uwin, norb)
    b_fwd, b_bwd = algorithmic_bytes(nk, nb, norb, ne)

    eps = torch.from_numpy(eps_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    teps, tw = torch.from_numpy(teps_np).to(dev), torch.from_numpy(tw_np).to(dev)
    dos = torch.empty((ne, norb), dtype=torch.float32, device=dev)
    ge = torch.empty_like(eps)
    gw = torch.empty_like(w)

    # tile shapes from the autotuner (outside the timed region); with --tiles every launch of the
    # run uses the given shapes, so a profile of the run sees one configuration per kernel
    from paper_1710_10789_amd import tune

    if args.tiles:
        tile_f, tile_b = (int(x) for x in args.tiles.split(","))
        times_f = times_b = None
    else:
        tile_f, times_f = tune.tune_forward(eps, w, grid, e0, de, ne, reps=3)
    target = tetra.dos_forward(teps, tw, grid, e0, de, ne, tile=tile_f)
    tetra.dos_forward(eps, w, grid, e0, de, ne, out=dos, tile=tile_f)
    G = (2.0 * (dos - target)).contiguous()
    if not args.tiles:
        tile_b, times_b = tune.tune_backward(eps, w, grid, e0, de, G, reps=3)
    # workspace of the adjoint's two-phase output (0 bytes where it does not apply), allocated once
    ws_b = torch.empty(max(tetra.backward_workspace_bytes(grid, nb, norb, e0, de, ne, tile=tile_b), 1),
                       dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    use_bwd = args.mode == "fwdbwd"

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        tetra.dos_forward(eps, w, grid, e0, de, ne, out=dos, tile=tile_f)
        if ev is not None:
            ev[1].record(stream)
        if use_bwd:
            tetra.dos_backward(eps, w, grid, e0, de, G, grad_eps=ge, grad_w=gw, tile=tile_b, workspace=ws_b)
            if ev is not None:
                ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    bwd_ms = np.array([e[1].elapsed_time(e[2]) for e in events]) if use_bwd else np.zeros(args.steps)
    ms_per_step = wall * 1e3 / args.steps
    step_ms = fwd_ms + bwd_ms
    t_fwd = float(fwd_ms.mean()) * 1e-3
    t_bwd = float(bwd_ms.mean()) * 1e-3

    if use_bwd and t_bwd > t_fwd:
        # the adjoint pass: its kernel and, where the two-phase output applies, the gather pass
        kname, klabel, flops, t_k = "dos_backward_kernel", "dos_backward_kernel + bwd_gather_kernel", f_bwd, t_bwd
    else:
        kname, klabel, flops, t_k = "dos_forward_kernel", "dos_forward_kernel", f_fwd, t_fwd
    achieved = flops / t_k / 1e12
    # the counter traffic depends on the launch configuration: reported only for the profiled one
    traffic_cfg = {"tile": list(tetra.TILE_SHAPES[tile_b if kname == "dos_backward_kernel" else tile_f])}
    roofline = {
        "bound": "alu",
        "kernel": klabel,
        "achieved": achieved,
        "peak": PEAK_FP32_VALU_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VALU_TFLOPS,
        "traffic": load_traffic(kname, traffic_cfg),
        "traffic_config": traffic_cfg,
        "algorithmic_flops_per_launch": flops,
        "avg_launch_ms": t_k * 1e3,
    }

    # LDS-atomic ceiling of the forward: its deposits are U_win * ceil(norb/2) 64-bit LDS atomic adds
    # (two orbitals per word), timed against the conflict-free rate of the probe kernel
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    p_blocks, p_iters = cus * 40, 1024
    from paper_1710_10789_amd import probe

    ms_probe = _time_events(torch, lambda: probe.probe_lds_atomics(p_blocks, p_iters, device=dev), 5, 2)
    rate = p_blocks * 256 * 4 * p_iters / (ms_probe * 1e-3)
    fwd_atomics = uwin * ((norb + 1) // 2)
    lds_ceiling = {"lane_atomics_per_s": rate, "forward_lane_atomics": fwd_atomics,
                   "ceiling_ms": fwd_atomics / rate * 1e3, "forward_ms": t_fwd * 1e3,
                   "frac": (fwd_atomics / rate) / t_fwd,
                   "probe": f"{p_blocks} workgroups x 256 lanes x {4 * p_iters} conflict-free ds_add_u64"}

    # the FP32 rate these kernels can issue: they are built without packed FP32, so their ceiling is
    # that of independent non-packed FMAs (half the published figure), timed here with the probe
    f_blocks, f_iters = cus * 32, 4096
    ms_fma = _time_events(torch, lambda: probe.probe_fma_f32(f_blocks, f_iters, device=dev), 5, 2)
    fma_tflops = f_blocks * 256 * f_iters * 16 * 2 / (ms_fma * 1e-3) / 1e12
    fma_rate = {"tflops": fma_tflops, "frac_of_published": fma_tflops / PEAK_FP32_VALU_TFLOPS,
                "forward_frac": f_fwd / t_fwd / 1e12 / fma_tflops,
                "adjoint_frac": (f_bwd / t_bwd / 1e12 / fma_tflops) if use_bwd else None,
                "probe": f"{f_blocks} workgroups x 256 lanes x {f_iters} x 16 independent v_fma_f32"}
    roofline["attainable_tflops"] = fma_tflops
    roofline["frac_attainable"] = achieved / fma_tflops

    out = {
        "metric": "tetra-band-energy updates/s at 64^3 k, 8 bands, 1000 E; fwd+bwd vs plain fwd",
        # dense-equivalent (tetrahedron, band, energy) triples of the workload per second of a step
        "value": dense / (ms_per_step * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random 8-orbital tight-binding model; eigh on the host, untimed)",
        "config": {
            "workload": f"{WORKLOAD}: 64^3 periodic k-grid, 8 bands x 8 orbitals, 1000 energies, FP32 SoA",
            "step": "forward + backward" if use_bwd else "forward",
            "n_tetrahedra": n_tet,
            "tile_forward": list(tetra.TILE_SHAPES[tile_f]),
            "tile_backward": list(tetra.TILE_SHAPES[tile_b]),
            "dense_updates_per_pass": dense,
            "in_window_updates_per_pass": uwin,
        },
        "fwd_ms": t_fwd * 1e3,
        "bwd_ms": t_bwd * 1e3 if use_bwd else None,
        # per-step event times (forward + backward): median, minimum, and the paper's statistic
        # (Sec. IV.A: seven runs, mean of the five shortest) over the first seven timed steps
        "step_event_ms": {"mean": float(step_ms.mean()), "median": float(np.median(step_ms)),
                          "min": float(step_ms.min()),
                          "mean_5_shortest_of_7": float(np.sort(step_ms[:7])[:5].mean()) if len(step_ms) >= 7 else None},
        "fwd_updates_per_s": dense / t_fwd,
        "fwdbwd_updates_per_s": dense / (t_fwd + t_bwd) if use_bwd else None,
        "fwdbwd_over_fwd": (dense / (t_fwd + t_bwd)) / (dense / t_fwd) if use_bwd else None,
        "in_window_updates_per_s_fwd": uwin / t_fwd,
        "roofline": roofline,
        "roofline_fwd": {"achieved": f_fwd / t_fwd / 1e12, "frac": f_fwd / t_fwd / 1e12 / PEAK_FP32_VALU_TFLOPS,
                         "hbm_gbs_algorithmic": b_fwd / t_fwd / 1e9},
        "roofline_bwd": ({"achieved": f_bwd / t_bwd / 1e12, "frac": f_bwd / t_bwd / 1e12 / PEAK_FP32_VALU_TFLOPS,
                          "hbm_gbs_algorithmic": b_bwd / t_bwd / 1e9} if use_bwd else None),
        "lds_atomic_ceiling": lds_ceiling,
        "fp32_fma_rate": fma_rate,
        "kernel_source_sha": {k: kernel_source_hash(k) for k in KERNEL_SOURCES},
        "autotune_ms": {"forward": times_f, "backward": times_b},
        "fwd_worst_case_ms": worst_case_forward_ms(torch, tetra, eps_np, w_np, grid, e0, de, ne, tile_f),
    }
    if not args.no_cpu_baseline:
        def gpu_fn():
            torch.cuda.synchronize()
            return dos.cpu().numpy().astype(np.float64)

        out["cpu_baseline"] = cpu_baseline(eps_np, w_np, grid, e0, de, ne, args.mode,
                                           G.cpu().numpy().astype(np.float64), gpu_fn)
        # the paper's best-case speedup (Sec. IV.A): one-core CPU time over the GPU kernel time of
        # the same forward pass, inputs resident on the device
        out["cpu_baseline"]["single_core_fwd_speedup"] = out["cpu_baseline"]["single_core_fwd_s"] / t_fwd
        out["cpu_baseline"]["single_core_fwd_speedup_worst_case"] = (
            out["cpu_baseline"]["single_core_fwd_s"] / (out["fwd_worst_case_ms"]["mean_5_shortest_of_7"] * 1e-3))
    if not args.no_precision:
        # the precision workload (not part of the headline value): times and errors of its four variants
        del eps, w, teps, tw, dos, ge, gw, ws_b, target, G
        torch.cuda.empty_cache()
        out["precision_k128_b16_e2000"] = precision_measurement(args, torch, tetra, dev,
                                                                with_oracle=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        # the other workloads' own lines, as extra keys (their values are not the headline value)
        for key, fn in (("batched_batch32", lambda: batched_record(args, torch, tetra, dev)),
                        ("nos_k64_b8_e1000", lambda: nos_record(args, torch, tetra, dev, with_oracle=False)),
                        ("chi_k64_b8_w500", lambda: chi_record(args, torch, tetra, dev,
                                                               with_oracle=not args.no_cpu_baseline))):
            print(f"[bench] extra workload {key}", file=sys.stderr, flush=True)
            out[key] = fn()
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
