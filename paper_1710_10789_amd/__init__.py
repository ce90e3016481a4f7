"""Tetrahedron-method orbital-resolved density of states on MI355X (gfx950).

Python binding of the C-ABI library ``libtetra.so`` (declared in ``include/tetra.h``). This module
only marshals arguments: it checks tensor shapes, dtypes and devices, and passes device pointers and
the current HIP stream to the library. Every step of the computation runs in the library's HIP
kernels. PyTorch provides device memory and streams.

The library must have been built (``python -m paper_1710_10789_amd.build``); importing the functions
below on a machine without it raises, there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "TetraError",
    "TETRA_EXACT",
    "TETRA_DETERMINISTIC",
    "TETRA_W_F32",
    "TETRA_W_F16",
    "TETRA_W_C32",
    "library_path",
    "lib",
    "make_desc",
    "dos_forward",
    "forward_workspace_bytes",
    "dos_forward_noalloc",
    "NOALLOC_MAX_BINS",
    "dos_backward",
    "backward_workspace_bytes",
    "nos_forward",
    "dos_binned",
    "chi_spectral",
    "chi_workspace_bytes",
    "dos",
    "dos_batched",
    "batched_workspace_bytes",
    "from_eigh",
    "half_weights",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libtetra.so")

TETRA_OK = 0
TETRA_W_F32 = 0
TETRA_W_F16 = 1
TETRA_W_C32 = 2
TETRA_EXACT = 1
TETRA_DETERMINISTIC = 2
TETRA_ERR_SCRATCH = -5
MAX_NORB = 16
NOALLOC_MAX_BINS = 262144  # ne*norb limit of the exact path of dos_forward_noalloc (TETRA_NOALLOC_MAX_BINS)
# tile shapes (cubes along grid axes 1, 2, 3) selectable through the flags' bits 8..11
TILE_SHAPES = ((4, 4, 16), (8, 8, 4), (4, 8, 8), (8, 4, 8), (4, 16, 4), (16, 4, 4))


def _tile_flag(tile):
    if tile is None:
        return 0
    t = int(tile)
    if not 0 <= t < len(TILE_SHAPES):
        raise ValueError(f"tile must be in 0..{len(TILE_SHAPES) - 1}")
    return t << 8


class TetraError(RuntimeError):
    def __init__(self, func, status, detail=""):
        self.status = status
        msg = f"{func} failed: {_status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class TetraDesc(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int),
        ("n2", ctypes.c_int),
        ("n3", ctypes.c_int),
        ("nb", ctypes.c_int),
        ("norb", ctypes.c_int),
        ("e0", ctypes.c_float),
        ("de", ctypes.c_float),
        ("ne", ctypes.c_int),
    ]


class TetraItem(ctypes.Structure):
    _fields_ = [
        ("d", TetraDesc),
        ("eps", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("w_scale", ctypes.c_void_p),
        ("dos", ctypes.c_void_p),
        ("tile", ctypes.c_int),
    ]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load ``libtetra.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing; build it with `python -m paper_1710_10789_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        p, i, u = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint
        L.tetra_dos_forward.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, u, p]
        L.tetra_dos_forward.restype = i
        L.tetra_dos_forward_workspace.argtypes = [ctypes.POINTER(TetraDesc), u]
        L.tetra_dos_forward_workspace.restype = ctypes.c_size_t
        L.tetra_dos_forward_ws.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, u, p, ctypes.c_size_t, p]
        L.tetra_dos_forward_ws.restype = i
        L.tetra_dos_forward_noalloc.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, u, p]
        L.tetra_dos_forward_noalloc.restype = i
        L.tetra_pack_f16.argtypes = [i, i, i, p, p, p, p]
        L.tetra_pack_f16.restype = i
        L.tetra_nos_forward.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, u, p]
        L.tetra_nos_forward.restype = i
        L.tetra_dos_binned.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, u, p]
        L.tetra_dos_binned.restype = i
        L.tetra_chi_spectral.argtypes = [ctypes.POINTER(TetraDesc), i, i, i, ctypes.c_float, p, p, i, p, p, u, p]
        L.tetra_chi_spectral.restype = i
        L.tetra_chi_spectral_workspace.argtypes = [ctypes.POINTER(TetraDesc), u]
        L.tetra_chi_spectral_workspace.restype = ctypes.c_size_t
        L.tetra_chi_spectral_ws.argtypes = [ctypes.POINTER(TetraDesc), i, i, i, ctypes.c_float, p, p, i, p, p, u, p,
                                            ctypes.c_size_t, p]
        L.tetra_chi_spectral_ws.restype = i
        L.tetra_dos_backward.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, p, p, u, p]
        L.tetra_dos_backward.restype = i
        L.tetra_dos_backward_workspace.argtypes = [ctypes.POINTER(TetraDesc), u]
        L.tetra_dos_backward_workspace.restype = ctypes.c_size_t
        L.tetra_dos_backward_ws.argtypes = [ctypes.POINTER(TetraDesc), p, p, i, p, p, p, p, u, p, ctypes.c_size_t, p]
        L.tetra_dos_backward_ws.restype = i
        L.tetra_dos_batched_workspace.argtypes = [ctypes.POINTER(TetraItem), i, i, u]
        L.tetra_dos_batched_workspace.restype = ctypes.c_size_t
        L.tetra_dos_batched.argtypes = [ctypes.POINTER(TetraItem), i, i, u, p, ctypes.c_size_t, p]
        L.tetra_dos_batched.restype = i
        L.tetra_status_string.argtypes = [i]
        L.tetra_status_string.restype = ctypes.c_char_p
        L.tetra_last_hip_error.argtypes = []
        L.tetra_last_hip_error.restype = ctypes.c_char_p
        L.tetra_version.argtypes = []
        L.tetra_version.restype = i
        _lib = L
    return _lib


def _status_string(status):
    try:
        return lib().tetra_status_string(int(status)).decode()
    except Exception:  # noqa: BLE001 - message only
        return "unknown status"


def _check(func, status):
    if status != TETRA_OK:
        detail = lib().tetra_last_hip_error().decode() if status == -4 else ""
        raise TetraError(func, status, detail)


def make_desc(grid, nb, norb, e0, de, ne) -> TetraDesc:
    n1, n2, n3 = (int(x) for x in grid)
    return TetraDesc(n1, n2, n3, int(nb), int(norb), float(e0), float(de), int(ne))


def _torch():
    import torch

    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require(t, name, shape, dtypes, device=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _shapes(eps, w, grid):
    n1, n2, n3 = (int(x) for x in grid)
    nk = n1 * n2 * n3
    if eps.dim() != 2 or w.dim() != 3:
        raise ValueError("eps must be [nb, nk] and w [nb, norb, nk]")
    nb, norb = w.shape[0], w.shape[1]
    return nk, nb, norb


def _weight_dtypes(torch):
    return (torch.float32, torch.float16, torch.complex64)


def _wtype_of(torch, w):
    return {torch.float16: TETRA_W_F16, torch.complex64: TETRA_W_C32}.get(w.dtype, TETRA_W_F32)


def _weights_type(torch, w, w_scale, nb, dev):
    wtype = _wtype_of(torch, w)
    if wtype == TETRA_W_F16:
        if w_scale is None:
            raise ValueError("float16 weights need w_scale")
        _require(w_scale, "w_scale", (nb,), (torch.float32,), dev)
    elif w_scale is not None:
        raise ValueError("w_scale is only used with float16 weights")
    return wtype


def _integrated(func, eps, w, grid, e0, de, ne, w_scale, out, tile):
    torch = _torch()
    nk, nb, norb = _shapes(eps, w, grid)
    dev = eps.device
    _require(eps, "eps", (nb, nk), (torch.float32,), dev)
    _require(w, "w", (nb, norb, nk), _weight_dtypes(torch), dev)
    wtype = _weights_type(torch, w, w_scale, nb, dev)
    if out is None:
        out = torch.empty((int(ne), norb), dtype=torch.float32, device=dev)
    _require(out, "out", (int(ne), norb), (torch.float32,), dev)
    d = make_desc(grid, nb, norb, e0, de, ne)
    st = getattr(lib(), func)(
        ctypes.byref(d), eps.data_ptr(), w.data_ptr(), wtype,
        w_scale.data_ptr() if w_scale is not None else None, out.data_ptr(), _tile_flag(tile),
        _stream_handle(dev))
    _check(func, st)
    return out


def nos_forward(eps, w, grid, e0, de, ne, *, w_scale=None, out=None, tile=None):
    """Orbital-resolved number of states ``[ne, norb]`` (FP32) at E_j = e0 + j*de: the states of each
    orbital up to E_j per k-point. Arguments as for ``dos_forward``."""
    return _integrated("tetra_nos_forward", eps, w, grid, e0, de, ne, w_scale, out, tile)


def dos_binned(eps, w, grid, e0, de, ne, *, w_scale=None, out=None, tile=None):
    """Bin-averaged orbital-resolved DOS ``[ne, norb]``: (N(E_j + de/2) - N(E_j - de/2)) / de, the
    number of states gained across the bin of width de centred on E_j, divided by de. Arguments as
    for ``dos_forward``."""
    return _integrated("tetra_dos_binned", eps, w, grid, e0, de, ne, w_scale, out, tile)


def chi_workspace_bytes(grid, nb, norb, w0, dw, nw, *, tile=None):
    """Bytes of the workspace ``chi_spectral`` passes to ``tetra_chi_spectral_ws`` (the energy range of
    every (tile, band) at k and at k + q)."""
    d = make_desc(grid, nb, norb, w0, dw, nw)
    return int(lib().tetra_chi_spectral_workspace(ctypes.byref(d), _tile_flag(tile)))


def chi_spectral(eps, w, grid, q, e_fermi, w0, dw, nw, *, w_scale=None, out=None, tile=None, workspace=None,
                 ranges=True):
    """Orbital-resolved susceptibility spectral weight ``S [nw, norb]`` (FP32) at transfer energies
    w_j = w0 + j*dw for the transfer ``q`` (three integers, grid steps) and Fermi energy ``e_fermi``:
    the imaginary part of the bare Lindhard susceptibility at zero temperature is ``-pi S``. Sums every
    band pair (n, n') with weights b_n(k) b_n'(k + q). Arguments otherwise as for ``dos_forward``.

    ``ranges`` (default): ``tetra_chi_spectral_ws`` with a workspace (``workspace``, a uint8 tensor of
    at least ``chi_workspace_bytes(...)`` bytes, or one taken from torch's allocator), whose first pass
    lets the (tile, band pair) units that cannot contribute leave before loading anything;
    ``ranges=False``: ``tetra_chi_spectral``."""
    torch = _torch()
    nk, nb, norb = _shapes(eps, w, grid)
    dev = eps.device
    _require(eps, "eps", (nb, nk), (torch.float32,), dev)
    _require(w, "w", (nb, norb, nk), _weight_dtypes(torch), dev)
    wtype = _weights_type(torch, w, w_scale, nb, dev)
    if out is None:
        out = torch.empty((int(nw), norb), dtype=torch.float32, device=dev)
    _require(out, "out", (int(nw), norb), (torch.float32,), dev)
    q1, q2, q3 = (int(x) for x in q)
    d = make_desc(grid, nb, norb, w0, dw, nw)
    ws_ptr, ws_bytes = None, 0
    if ranges:
        need = int(lib().tetra_chi_spectral_workspace(ctypes.byref(d), _tile_flag(tile)))
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        _check_workspace(workspace, need, dev)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    elif workspace is not None:
        raise ValueError("workspace is for ranges=True")
    st = lib().tetra_chi_spectral_ws(ctypes.byref(d), q1, q2, q3, float(e_fermi), eps.data_ptr(), w.data_ptr(), wtype,
                                     w_scale.data_ptr() if w_scale is not None else None, out.data_ptr(),
                                     _tile_flag(tile), ws_ptr, ws_bytes, _stream_handle(dev))
    _check("tetra_chi_spectral_ws", st)
    return out


def _check_workspace(workspace, need, dev):
    if workspace.dtype != _torch().uint8 or workspace.device != dev or workspace.numel() < need \
            or not workspace.is_contiguous():
        raise ValueError(f"workspace must be a contiguous uint8 tensor on {dev} of at least {need} bytes")


def forward_workspace_bytes(grid, nb, norb, e0, de, ne, *, exact=False, deterministic=False, tile=None):
    """Device bytes ``dos_forward`` needs for its exact accumulation (0 without ``exact`` or
    ``deterministic``)."""
    d = make_desc(grid, nb, norb, e0, de, ne)
    flags = (TETRA_EXACT if exact else 0) | (TETRA_DETERMINISTIC if deterministic else 0) | _tile_flag(tile)
    return int(lib().tetra_dos_forward_workspace(ctypes.byref(d), flags))


def dos_forward(eps, w, grid, e0, de, ne, *, w_scale=None, exact=False, deterministic=False, out=None, tile=None,
                workspace=None):
    """Orbital-resolved DOS ``[ne, norb]`` (FP32) on the current HIP stream.

    eps: float32 ``[nb, nk]``; w: float32 or float16 orbital weights ``[nb, norb, nk]`` (float16 needs
    ``w_scale`` float32 ``[nb]``), or complex64 amplitudes a (the weights are ``|a|^2``, formed in the
    kernels); grid: (n1, n2, n3) with nk = n1*n2*n3; E_j = e0 + j*de. ``exact`` selects the
    exact cross-workgroup accumulation, ``deterministic`` asks for a bitwise reproducible result (the
    same exact path); both use a device workspace (``workspace``, a uint8 tensor of at least
    ``forward_workspace_bytes`` bytes, or one allocated here). ``tile`` an index into ``TILE_SHAPES``
    (default 0).
    """
    torch = _torch()
    nk, nb, norb = _shapes(eps, w, grid)
    dev = eps.device
    _require(eps, "eps", (nb, nk), (torch.float32,), dev)
    _require(w, "w", (nb, norb, nk), _weight_dtypes(torch), dev)
    wtype = _weights_type(torch, w, w_scale, nb, dev)
    if out is None:
        out = torch.empty((int(ne), norb), dtype=torch.float32, device=dev)
    _require(out, "out", (int(ne), norb), (torch.float32,), dev)
    d = make_desc(grid, nb, norb, e0, de, ne)
    flags = (TETRA_EXACT if exact else 0) | (TETRA_DETERMINISTIC if deterministic else 0) | _tile_flag(tile)
    need = int(lib().tetra_dos_forward_workspace(ctypes.byref(d), flags))
    ws_ptr, ws_bytes = None, 0
    if need:
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        _check_workspace(workspace, need, dev)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    st = lib().tetra_dos_forward_ws(
        ctypes.byref(d), eps.data_ptr(), w.data_ptr(), wtype,
        w_scale.data_ptr() if w_scale is not None else None, out.data_ptr(), flags, ws_ptr, ws_bytes,
        _stream_handle(dev))
    _check("tetra_dos_forward_ws", st)
    return out


def dos_forward_noalloc(eps, w, grid, e0, de, ne, out, *, w_scale=None, exact=False, deterministic=False,
                        tile=None):
    """``dos_forward`` through ``tetra_dos_forward_noalloc``: the exact path's workspace is the
    library's static device scratch, so nothing is allocated (``out`` is required). Exact calls that
    overlap on one device race on that scratch; ne*norb above ``NOALLOC_MAX_BINS`` raises
    (``TETRA_ERR_SCRATCH``) with ``exact`` or ``deterministic``."""
    torch = _torch()
    nk, nb, norb = _shapes(eps, w, grid)
    dev = eps.device
    _require(eps, "eps", (nb, nk), (torch.float32,), dev)
    _require(w, "w", (nb, norb, nk), _weight_dtypes(torch), dev)
    wtype = _weights_type(torch, w, w_scale, nb, dev)
    _require(out, "out", (int(ne), norb), (torch.float32,), dev)
    d = make_desc(grid, nb, norb, e0, de, ne)
    flags = (TETRA_EXACT if exact else 0) | (TETRA_DETERMINISTIC if deterministic else 0) | _tile_flag(tile)
    st = lib().tetra_dos_forward_noalloc(
        ctypes.byref(d), eps.data_ptr(), w.data_ptr(), wtype,
        w_scale.data_ptr() if w_scale is not None else None, out.data_ptr(), flags, _stream_handle(dev))
    _check("tetra_dos_forward_noalloc", st)
    return out


def backward_workspace_bytes(grid, nb, norb, e0, de, ne, *, tile=None):
    """Device bytes of the adjoint's two-phase output (0 where it does not apply: a grid side not a
    multiple of the tile's, or a single tile along an axis)."""
    d = make_desc(grid, nb, norb, e0, de, ne)
    return int(lib().tetra_dos_backward_workspace(ctypes.byref(d), _tile_flag(tile)))


def dos_backward(eps, w, grid, e0, de, grad_dos, *, w_scale=None, need_eps=True, need_w=True,
                 grad_eps=None, grad_w=None, tile=None, two_phase=True, workspace=None, deterministic=False):
    """``(dL/deps [nb, nk] or None, dL/dw [nb, norb, nk] or None)`` for ``grad_dos = dL/dDOS``.

    dL/dw is float32 for float32 or float16 weights (of the dequantised weights) and complex64 for
    complex amplitudes, ``2 a dL/db`` (the gradient with respect to the real and imaginary parts).

    ``two_phase`` (where it applies, see ``backward_workspace_bytes``): tile-boundary points go through
    a workspace (``workspace``, a uint8 device tensor of at least that size, or one allocated here)
    and a gather pass instead of global atomics; the gradients are then bitwise reproducible and
    ``deterministic=True`` is accepted (it raises where the two-phase output does not apply)."""
    torch = _torch()
    nk, nb, norb = _shapes(eps, w, grid)
    dev = eps.device
    ne = grad_dos.shape[0]
    _require(eps, "eps", (nb, nk), (torch.float32,), dev)
    _require(w, "w", (nb, norb, nk), _weight_dtypes(torch), dev)
    _require(grad_dos, "grad_dos", (ne, norb), (torch.float32,), dev)
    wtype = _weights_type(torch, w, w_scale, nb, dev)
    gw_dtype = torch.complex64 if wtype == TETRA_W_C32 else torch.float32
    if need_eps and grad_eps is None:
        grad_eps = torch.empty((nb, nk), dtype=torch.float32, device=dev)
    if need_w and grad_w is None:
        grad_w = torch.empty((nb, norb, nk), dtype=gw_dtype, device=dev)
    if grad_eps is not None:
        _require(grad_eps, "grad_eps", (nb, nk), (torch.float32,), dev)
    if grad_w is not None:
        _require(grad_w, "grad_w", (nb, norb, nk), (gw_dtype,), dev)
    d = make_desc(grid, nb, norb, e0, de, ne)
    flags = _tile_flag(tile) | (TETRA_DETERMINISTIC if deterministic else 0)
    need = int(lib().tetra_dos_backward_workspace(ctypes.byref(d), flags)) if two_phase else 0
    ws_ptr, ws_bytes = None, 0
    if need:
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        _check_workspace(workspace, need, dev)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
    st = lib().tetra_dos_backward_ws(
        ctypes.byref(d), eps.data_ptr(), w.data_ptr(), wtype,
        w_scale.data_ptr() if w_scale is not None else None, grad_dos.data_ptr(),
        grad_eps.data_ptr() if grad_eps is not None else None,
        grad_w.data_ptr() if grad_w is not None else None, flags, ws_ptr, ws_bytes, _stream_handle(dev))
    _check("tetra_dos_backward_ws", st)
    return grad_eps, grad_w


def _batch_items(problems, out, tiles=None):
    torch = _torch()
    n = len(problems)
    items = (TetraItem * n)()
    outs = []
    wtype = None
    for i, pr in enumerate(problems):
        eps, w, grid, e0, de, ne = pr[:6]
        w_scale = pr[6] if len(pr) > 6 else None
        nk, nb, norb = _shapes(eps, w, grid)
        dev = eps.device
        _require(eps, f"items[{i}].eps", (nb, nk), (torch.float32,), dev)
        _require(w, f"items[{i}].w", (nb, norb, nk), _weight_dtypes(torch), dev)
        wt = _wtype_of(torch, w)
        if wtype is None:
            wtype = wt
        elif wt != wtype:
            raise TypeError("all items of a batch need the same weight dtype")
        if wt == TETRA_W_F16:
            _require(w_scale, f"items[{i}].w_scale", (nb,), (torch.float32,), dev)
        o = out[i] if out is not None else torch.empty((int(ne), norb), dtype=torch.float32, device=dev)
        _require(o, f"out[{i}]", (int(ne), norb), (torch.float32,), dev)
        outs.append(o)
        items[i].d = make_desc(grid, nb, norb, e0, de, ne)
        items[i].eps = eps.data_ptr()
        items[i].w = w.data_ptr()
        items[i].w_scale = w_scale.data_ptr() if w_scale is not None else None
        items[i].dos = o.data_ptr()
        items[i].tile = 0 if tiles is None else _tile_flag(tiles[i]) >> 8
    return items, outs, wtype


def batched_workspace_bytes(problems) -> int:
    """Device workspace ``dos_batched`` needs for these problems (see ``tetra_dos_batched_workspace``)."""
    items, _, wtype = _batch_items(problems, None)
    return int(lib().tetra_dos_batched_workspace(items, len(problems), wtype, 0))


def dos_batched(problems, *, workspace=None, out=None, tiles=None):
    """DOS of many independent problems in one persistent launch per orbital count.

    problems: sequence of ``(eps, w, grid, e0, de, ne)`` or ``(eps, w, grid, e0, de, ne, w_scale)``
    with the same meaning as in :func:`dos_forward`. ``workspace`` is an optional uint8 device tensor
    of at least :func:`batched_workspace_bytes` bytes (allocated here when omitted). ``tiles`` gives
    each problem's tile shape (see :mod:`paper_1710_10789_amd.tune`). Returns the list of
    ``[ne, norb]`` results (``out`` if given).
    """
    torch = _torch()
    if len(problems) == 0:
        return []
    items, outs, wtype = _batch_items(problems, out, tiles)
    dev = problems[0][0].device
    need = int(lib().tetra_dos_batched_workspace(items, len(problems), wtype, 0))
    if need == 0:
        raise TetraError("tetra_dos_batched_workspace", -1)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if not workspace.is_cuda or workspace.device != dev:
        raise ValueError("workspace must be a tensor on the problems' device")
    # the library checks the size (TETRA_ERR_WORKSPACE)
    st = lib().tetra_dos_batched(items, len(problems), wtype, 0, workspace.data_ptr(), workspace.numel(),
                                 _stream_handle(dev))
    _check("tetra_dos_batched", st)
    return outs


def _autograd_function():
    torch = _torch()

    class _TetraDOS(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps, w, grid, e0, de, ne, exact, tiles, w_scale):
            ctx.save_for_backward(eps, w, w_scale)
            ctx.args = (tuple(grid), float(e0), float(de), tiles[1])
            return dos_forward(eps.contiguous(), w.contiguous(), grid, e0, de, ne, w_scale=w_scale, exact=exact,
                               tile=tiles[0])

        @staticmethod
        def backward(ctx, g):
            eps, w, w_scale = ctx.saved_tensors
            grid, e0, de, btile = ctx.args
            need_w = ctx.needs_input_grad[1]
            ge, gw = dos_backward(eps.contiguous(), w.contiguous(), grid, e0, de, g.contiguous(), w_scale=w_scale,
                                  need_eps=ctx.needs_input_grad[0], need_w=need_w, tile=btile)
            if gw is not None and w.dtype == _torch().float16:
                # dL/d(stored FP16 value) = scale_n dL/db (the kernel's gradient is of b = scale_n w16)
                gw = (gw * w_scale[:, None, None]).to(w.dtype)
            return ge, gw, None, None, None, None, None, None, None

    return _TetraDOS


_FN = None


def dos(eps, w, grid, e0, de, ne, exact=False, tile=None, backward_tile=None, w_scale=None):
    """Differentiable orbital-resolved DOS ``[ne, norb]`` (float32 weights, float16 weights with their
    per-band ``w_scale``, or complex64 amplitudes).

    Gradients with respect to ``eps`` and ``w`` come from the adjoint kernel. For float16 weights the
    gradient with respect to ``w`` is that of the stored values (``scale_n dL/db``, rounded to
    float16); ``w_scale`` itself is treated as a constant.
    """
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(eps, w, tuple(grid), e0, de, ne, exact, (tile, backward_tile), w_scale)


def from_eigh(evals, evecs, amplitudes=False):
    """Structure-of-arrays inputs from ``torch.linalg.eigh`` output.

    evals ``[nk, nb]`` and eigenvectors ``[nk, norb, nb]`` (columns are bands) -> eps ``[nb, nk]`` and
    w ``[nb, norb, nk]``: the weights |a|^2 (eq. matrixelements) in float32, or with ``amplitudes`` the
    eigenvector components a themselves in complex64 (the kernels square them). Differentiable (a
    layout change); not part of the DOS path.
    """
    eps = evals.transpose(0, 1).contiguous().float()
    if amplitudes:
        a = evecs if evecs.is_complex() else evecs.to(_torch().complex64)
        return eps, a.permute(2, 1, 0).contiguous().to(_torch().complex64)
    w = (evecs.real ** 2 + evecs.imag ** 2) if evecs.is_complex() else evecs ** 2
    return eps, w.permute(2, 1, 0).contiguous().float()


def half_weights(w, *, out=None, scale=None):
    """FP16 weights with a per-band power-of-two scale, by the library's pack kernel
    (``tetra_pack_f16``): ``(w16 [nb, norb, nk], scale [nb])``.

    scale_n = 2^ceil(log2 max_{m,k} |w[n, m, k]|) (clamped to 2^-126..2^126; 1 for an all-zero band),
    w16 = RNE(w / scale_n), so the scaling itself is exact and the only error is FP16 rounding.
    """
    torch = _torch()
    if w.dim() != 3:
        raise ValueError("w must be [nb, norb, nk]")
    nb, norb, nk = (int(x) for x in w.shape)
    dev = w.device
    _require(w, "w", (nb, norb, nk), (torch.float32,), dev)
    if out is None:
        out = torch.empty((nb, norb, nk), dtype=torch.float16, device=dev)
    if scale is None:
        scale = torch.empty(nb, dtype=torch.float32, device=dev)
    _require(out, "out", (nb, norb, nk), (torch.float16,), dev)
    _require(scale, "scale", (nb,), (torch.float32,), dev)
    _check("tetra_pack_f16", lib().tetra_pack_f16(nb, norb, nk, w.data_ptr(), out.data_ptr(), scale.data_ptr(),
                                                  _stream_handle(dev)))
    return out, scale
