"""Autotuner for the tile shape of the forward and adjoint kernels.

For a problem class (GPU name, kernel, weight dtype, bands, orbitals, k-point bucket, energy-count
bucket) every tile shape of ``TILE_SHAPES`` is timed on the current stream with HIP events (the best
of two sweeps in opposite orders), and the fastest is kept in a JSON cache (``$TETRA_TUNE_CACHE``, default ``~/.cache/tetra_tune.json``).
Lookups of an untuned class fall back to the default shape 0.
"""
from __future__ import annotations

import json
import math
import os

from . import TILE_SHAPES, dos_backward, dos_forward

_CACHE_PATH = os.environ.get("TETRA_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tetra_tune.json"))
_cache = None


def _load():
    global _cache
    if _cache is None:
        try:
            with open(_CACHE_PATH) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def _save():
    try:
        os.makedirs(os.path.dirname(_CACHE_PATH), exist_ok=True)
        tmp = _CACHE_PATH + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)
        os.replace(tmp, _CACHE_PATH)
    except OSError:
        pass  # an unwritable cache only means tuning again next time


def problem_key(kernel, eps, w, grid, ne) -> str:
    import torch

    nk = int(grid[0]) * int(grid[1]) * int(grid[2])
    name = torch.cuda.get_device_name(eps.device) if eps.is_cuda else "cpu"
    return "|".join([name, kernel, str(w.dtype).replace("torch.", ""), f"nb{w.shape[0]}", f"norb{w.shape[1]}",
                     f"nk2^{int(round(math.log2(max(nk, 1))))}", f"ne2^{int(round(math.log2(max(int(ne), 1))))}"])


def best_tile(kernel, eps, w, grid, ne, default: int = 0) -> int:
    rec = _load().get(problem_key(kernel, eps, w, grid, ne))
    return int(rec["tile"]) if rec else default


def _time(fn, reps):
    import torch

    fn()  # warm-up
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def _sweep(make, reps, rounds):
    """Best time per tile shape over ``rounds`` sweeps, alternating the order of the shapes, so that
    clock ramp-up and cache state do not favour the shapes timed last."""
    n = len(TILE_SHAPES)
    best = [float("inf")] * n
    for r in range(rounds):
        order = range(n) if r % 2 == 0 else range(n - 1, -1, -1)
        for t in order:
            best[t] = min(best[t], _time(make(t), reps))
    return best


def _record(key, times):
    best = min(range(len(times)), key=lambda i: times[i])
    _load()[key] = {"tile": best, "shape": list(TILE_SHAPES[best]), "ms": times}
    _save()
    return best


def tune_forward(eps, w, grid, e0, de, ne, w_scale=None, reps: int = 3, rounds: int = 2):
    """Time every tile shape of the forward kernel on this problem; returns (best, [ms per shape])."""
    import torch

    out = torch.empty((int(ne), w.shape[1]), dtype=torch.float32, device=eps.device)
    times = _sweep(lambda t: (lambda: dos_forward(eps, w, grid, e0, de, ne, w_scale=w_scale, out=out, tile=t)),
                   reps, rounds)
    return _record(problem_key("forward", eps, w, grid, ne), times), times


def tune_backward(eps, w, grid, e0, de, grad_dos, w_scale=None, reps: int = 3, rounds: int = 2):
    """Time every tile shape of the adjoint kernel on this problem; returns (best, [ms per shape])."""
    import torch

    ge = torch.empty_like(eps)
    gw = torch.empty(w.shape, dtype=torch.complex64 if w.is_complex() else torch.float32, device=eps.device)
    times = _sweep(lambda t: (lambda: dos_backward(eps, w, grid, e0, de, grad_dos, w_scale=w_scale, grad_eps=ge,
                                                   grad_w=gw, tile=t)), reps, rounds)
    return _record(problem_key("backward", eps, w, grid, grad_dos.shape[0]), times), times


def tiles_for_batch(problems, tune_missing: bool = True, reps: int = 2):
    """Tile shape per batched problem: the forward's tuned shape of its class (tuned on first sight)."""
    tiles = []
    for pr in problems:
        eps, w, grid, e0, de, ne = pr[:6]
        w_scale = pr[6] if len(pr) > 6 else None
        key = problem_key("forward", eps, w, grid, ne)
        if key not in _load() and tune_missing:
            tune_forward(eps, w, grid, e0, de, ne, w_scale=w_scale, reps=reps)
        tiles.append(best_tile("forward", eps, w, grid, ne))
    return tiles
