"""ctypes front end of ``libtetra_probe.so``, the benchmark's measurement helpers.

Not part of the DOS library: ``tetra_probe_lds_atomics`` times conflict-free 64-bit LDS atomic adds
(the instruction of the kernels' histogram deposits), a ceiling the benchmark reports beside the
forward kernel's time; ``tetra_probe_fma_f32`` times independent non-packed FP32 FMAs, the issue
rate that bounds the kernels (all built without packed FP32 instructions).
"""
from __future__ import annotations

import ctypes
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtetra_probe.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_PATH):
            raise ImportError(f"{_PATH} is missing; build it with `python -m paper_1710_10789_amd.build`")
        L = ctypes.CDLL(_PATH)
        L.tetra_probe_lds_atomics.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.tetra_probe_lds_atomics.restype = ctypes.c_int
        L.tetra_probe_fma_f32.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.tetra_probe_fma_f32.restype = ctypes.c_int
        _lib = L
    return _lib


def probe_lds_atomics(blocks, iters, device=None, out=None):
    """Launch the probe on the current stream (``blocks`` x 256 lanes x ``iters`` x 4 conflict-free
    64-bit LDS atomic adds); returns the int64 checksum tensor ``[blocks]``."""
    import torch

    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(int(blocks), dtype=torch.int64, device=dev)
    if out.dtype != torch.int64 or tuple(out.shape) != (int(blocks),) or out.device != dev:
        raise ValueError("out must be an int64 tensor [blocks] on the device")
    st = lib().tetra_probe_lds_atomics(int(blocks), int(iters), out.data_ptr(),
                                       ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        raise RuntimeError(f"tetra_probe_lds_atomics failed ({st})")
    return out


def probe_fma_f32(blocks, iters, device=None, out=None):
    """Launch the FMA probe on the current stream (``blocks`` x 256 lanes x ``iters`` x 16 independent
    FP32 FMAs); returns the float32 tensor ``[blocks * 256]`` of per-lane results."""
    import torch

    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    n = int(blocks) * 256
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=dev)
    if out.dtype != torch.float32 or tuple(out.shape) != (n,) or out.device != dev:
        raise ValueError("out must be a float32 tensor [blocks * 256] on the device")
    st = lib().tetra_probe_fma_f32(int(blocks), int(iters), out.data_ptr(),
                                   ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        raise RuntimeError(f"tetra_probe_fma_f32 failed ({st})")
    return out
