"""ctypes front end of the FP64 CPU oracle (``oracle/tetra_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's CPU
baseline. The product package never imports it, and it imports nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tetra_oracle.cpp")
_LIB = os.path.join(_HERE, "libtetra_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP64, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d, i, ll = ctypes.c_double, ctypes.c_int, ctypes.c_longlong
        p = ctypes.c_void_p
        lib.tetra_oracle_table.argtypes = [p]
        lib.tetra_oracle_corner_weights.argtypes = [p, d, d, p, p]
        lib.tetra_oracle_corner_weights_grad.argtypes = [p, d, d, p, p]
        lib.tetra_oracle_tet_dos.argtypes = [p, p, d, d]
        lib.tetra_oracle_tet_dos.restype = d
        lib.tetra_oracle_tet_nos.argtypes = [p, p, d, d]
        lib.tetra_oracle_tet_nos.restype = d
        lib.tetra_oracle_dos.argtypes = [i, i, i, i, i, d, d, i, p, p, p, i]
        lib.tetra_oracle_dos.restype = ll
        lib.tetra_oracle_nos.argtypes = [i, i, i, i, i, d, d, i, p, p, p, i]
        lib.tetra_oracle_nos.restype = i
        lib.tetra_oracle_dos_backward.argtypes = [i, i, i, i, i, d, d, i, p, p, p, p, p, i]
        lib.tetra_oracle_dos_backward.restype = i
        lib.tetra_oracle_tet_chi.argtypes = [p, p, p, d, d, d]
        lib.tetra_oracle_tet_chi.restype = d
        lib.tetra_oracle_chi.argtypes = [i, i, i, i, i, i, i, i, d, d, d, i, p, p, p, i]
        lib.tetra_oracle_chi.restype = ll
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _threads(nthreads):
    if nthreads is None:
        return max(1, len(os.sched_getaffinity(0)))
    return int(nthreads)


def table():
    """Table I as 0-based cube-corner slots ``o1 + 2*o2 + 4*o3``, shape [6, 4]."""
    out = np.zeros(24, dtype=np.int32)
    _load().tetra_oracle_table(_ptr(out))
    return out.reshape(6, 4)


def corner_weights(e_sorted, E, vol):
    """``(w[4], g[4])``: integrated corner weights and dw/dE for sorted corner energies."""
    e = np.ascontiguousarray(e_sorted, dtype=np.float64)
    w = np.zeros(4)
    g = np.zeros(4)
    _load().tetra_oracle_corner_weights(_ptr(e), float(E), float(vol), _ptr(w), _ptr(g))
    return w, g


def corner_weights_grad(e_sorted, E, vol):
    """``(g[4], dg[4, 4])`` with ``dg[l, i] = d(dw_l/dE)/dE_i`` (sorted energies)."""
    e = np.ascontiguousarray(e_sorted, dtype=np.float64)
    g = np.zeros(4)
    dg = np.zeros(16)
    _load().tetra_oracle_corner_weights_grad(_ptr(e), float(E), float(vol), _ptr(g), _ptr(dg))
    return g, dg.reshape(4, 4)


def tet_dos(e, b, E, vol):
    """``sum_l b_l dw_l/dE`` for one tetrahedron, corners in any order."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _load().tetra_oracle_tet_dos(_ptr(e), _ptr(b), float(E), float(vol))


def tet_nos(e, b, E, vol):
    """``sum_l b_l w_l(E)`` for one tetrahedron, corners in any order."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _load().tetra_oracle_tet_nos(_ptr(e), _ptr(b), float(E), float(vol))


def _grid_args(eps, w, grid):
    eps = np.ascontiguousarray(eps, dtype=np.float32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    n1, n2, n3 = (int(x) for x in grid)
    nk = n1 * n2 * n3
    nb = eps.shape[0]
    if eps.shape != (nb, nk) or w.ndim != 3 or w.shape[0] != nb or w.shape[2] != nk:
        raise ValueError(f"shape mismatch: eps {eps.shape}, w {w.shape}, grid {grid}")
    return eps, w, n1, n2, n3, nb, w.shape[1]


def dos(eps, w, grid, e0, de, ne, nthreads=None):
    """FP64 orbital-resolved DOS ``[ne, norb]`` and the in-window update count."""
    eps, w, n1, n2, n3, nb, norb = _grid_args(eps, w, grid)
    out = np.zeros((ne, norb), dtype=np.float64)
    cnt = _load().tetra_oracle_dos(n1, n2, n3, nb, norb, float(e0), float(de), int(ne),
                                   _ptr(eps), _ptr(w), _ptr(out), _threads(nthreads))
    if cnt < 0:
        raise ValueError("oracle rejected arguments")
    return out, int(cnt)


def nos(eps, w, grid, e0, de, ne, nthreads=None):
    """FP64 orbital-resolved number of states ``[ne, norb]`` (integrated weights, dense)."""
    eps, w, n1, n2, n3, nb, norb = _grid_args(eps, w, grid)
    out = np.zeros((ne, norb), dtype=np.float64)
    rc = _load().tetra_oracle_nos(n1, n2, n3, nb, norb, float(e0), float(de), int(ne),
                                  _ptr(eps), _ptr(w), _ptr(out), _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return out


def dos_binned(eps, w, grid, e0, de, ne, nthreads=None):
    """FP64 bin-averaged DOS ``[ne, norb]``: (N(E_j + de/2) - N(E_j - de/2)) / de with N the number of
    states above (Sec. II: the DOS is the energy derivative of the orbital-resolved particle number),
    from N on the ne + 1 bin edges e0 - de/2 + i de (exact in FP64 for FP32 e0, de)."""
    edges = nos(eps, w, grid, float(e0) - 0.5 * float(de), de, int(ne) + 1, nthreads)
    return np.diff(edges, axis=0) / float(de)


def dos_backward(eps, w, grid, e0, de, G, nthreads=None):
    """``(dL/deps [nb, nk], dL/dw [nb, norb, nk])`` in FP64 for ``G = dL/dDOS [ne, norb]``."""
    eps, w, n1, n2, n3, nb, norb = _grid_args(eps, w, grid)
    G = np.ascontiguousarray(G, dtype=np.float64)
    ne = G.shape[0]
    if G.shape != (ne, norb):
        raise ValueError("G must be [ne, norb]")
    ge = np.zeros(eps.shape, dtype=np.float64)
    gw = np.zeros(w.shape, dtype=np.float64)
    rc = _load().tetra_oracle_dos_backward(n1, n2, n3, nb, norb, float(e0), float(de), int(ne),
                                           _ptr(eps), _ptr(w), _ptr(G), _ptr(ge), _ptr(gw), _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return ge, gw


def tet_chi(e, ep, W, ef, E, vol):
    """One tetrahedron's susceptibility spectral weight at transfer energy E: corner energies ``e``
    (band n at k) and ``ep`` (band n' at k + q), interpolated weight ``W``, Fermi energy ``ef``."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    ep = np.ascontiguousarray(ep, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    return _load().tetra_oracle_tet_chi(_ptr(e), _ptr(ep), _ptr(W), float(ef), float(E), float(vol))


def chi(eps, w, grid, q, ef, w0, dw, nw, nthreads=None):
    """FP64 orbital-resolved susceptibility spectral weight ``S[nw, norb]`` at w_j = w0 + j*dw for the
    transfer ``q`` (grid steps), Fermi energy ``ef``; and the number of (sub-tetrahedron, band pair,
    energy) updates in open windows. Im chi_0 = -pi S."""
    eps, w, n1, n2, n3, nb, norb = _grid_args(eps, w, grid)
    out = np.zeros((nw, norb), dtype=np.float64)
    q1, q2, q3 = (int(x) for x in q)
    cnt = _load().tetra_oracle_chi(n1, n2, n3, nb, norb, q1, q2, q3, float(ef), float(w0), float(dw), int(nw),
                                   _ptr(eps), _ptr(w), _ptr(out), _threads(nthreads))
    if cnt < 0:
        raise ValueError("oracle rejected arguments")
    return out, int(cnt)
