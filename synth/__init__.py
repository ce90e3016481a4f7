"""Seeded synthetic inputs for the tetrahedron DOS: band energies and orbital weights.

This module only *prepares inputs*. It holds none of the tetrahedron method's arithmetic, so the
FP64 oracle and the HIP path can both consume what it produces without sharing any code.

The paper benchmarks an eight-orbital FeSe tight-binding model (Sec. II.A, eq. kinetichamiltonian),
diagonalised on the CPU outside the timed region (Sec. IV.A). Its hopping parameters are not given,
so a random Hermitian tight-binding model of the same shape stands in for it:

* ``t_0 = (A + A^H)/2 + diag(U[-2, 2])`` eV, ``A`` complex Gaussian with E|z|^2 = sigma^2, sigma = 0.3 eV;
* ``t_R`` complex Gaussian for R in (+x, +y, +z, +x+y, +x-y) in that order, ``t_{-R} = t_R^H``;
* ``H(k) = sum_R t_R exp(i k.R)`` on a periodic grid ``k_a = 2 pi i_a / N_a``, row-major (i1 slowest);
* ``eigh`` in complex128 -> ascending band energies ``E_n(k)`` and ``b_mn(k) = |a^m_n(k)|^2``
  (eq. matrixelements), cast to FP32 and laid out structure-of-arrays:
  ``eps[nb][nk]`` and ``w[nb][norb][nk]`` with ``k = (i1*n2 + i2)*n3 + i3`` (``amplitudes`` gives
  the eigenvector components ``a[nb][norb][nk]`` themselves, complex64, for small grids).
"""
from __future__ import annotations

import hashlib
import os
import sys
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# Nearest-neighbour-type hopping vectors; the negative ones follow from hermiticity.
_R_POS = ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0))
_CACHE_VERSION = "tb-v1"


def hoppings(norb: int, seed: int, sigma: float = 0.3):
    """Hopping matrices ``{R: t_R}`` (eV) of the seeded random model, 11 R vectors in total."""
    rng = np.random.default_rng(seed)

    def cg():
        return (rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))) * (sigma / np.sqrt(2.0))

    a = cg()
    t0 = (a + a.conj().T) / 2 + np.diag(rng.uniform(-2.0, 2.0, norb))
    hops = {(0, 0, 0): t0}
    for r in _R_POS:
        tr = cg()
        hops[r] = tr
        hops[tuple(-x for x in r)] = tr.conj().T
    return hops


def _kfrac(grid, lo, hi):
    n1, n2, n3 = grid
    k = np.arange(lo, hi, dtype=np.int64)
    i3 = k % n3
    i2 = (k // n3) % n2
    i1 = k // (n2 * n3)
    return np.stack([i1 / n1, i2 / n2, i3 / n3], axis=1)


def _diag_chunk(hops, grid, lo, hi):
    kf = _kfrac(grid, lo, hi)
    t0 = hops[(0, 0, 0)]
    norb = t0.shape[0]
    h = np.empty((hi - lo, norb, norb), dtype=np.complex128)
    h[:] = t0
    for r in _R_POS:
        tr = hops[r]
        ph = np.exp(2j * np.pi * (kf @ np.asarray(r, dtype=np.float64)))
        h += ph[:, None, None] * tr + ph.conj()[:, None, None] * tr.conj().T
    evals, evecs = np.linalg.eigh(h)  # ascending per k; columns are eigenvectors
    return evals, np.abs(evecs) ** 2  # [nc, nb], [nc, norb, nb]


def hamiltonians(hops, grid):
    """Bloch Hamiltonians ``H(k) = sum_R t_R exp(2 pi i k.R)`` ``[nk, norb, norb]`` (complex128) of a
    hopping set on the periodic grid, k in the library's order (i3 fastest)."""
    n1, n2, n3 = grid
    kf = _kfrac(grid, 0, n1 * n2 * n3)
    t0 = hops[(0, 0, 0)]
    h = np.empty((kf.shape[0],) + t0.shape, dtype=np.complex128)
    h[:] = t0
    for r in _R_POS:
        ph = np.exp(2j * np.pi * (kf @ np.asarray(r, dtype=np.float64)))
        h += ph[:, None, None] * hops[r] + ph.conj()[:, None, None] * hops[r].conj().T
    return h


def amplitudes(norb: int, seed: int, grid):
    """Band energies ``eps [nb, nk]`` (float32) and eigenvector components ``a [nb, norb, nk]``
    (complex64, a[n, m, k] = <m|n,k>) of the seeded model, for small grids (no cache)."""
    evals, evecs = np.linalg.eigh(hamiltonians(hoppings(norb, seed), grid))
    eps = np.ascontiguousarray(evals.T, dtype=np.float32)
    a = np.ascontiguousarray(evecs.transpose(2, 1, 0), dtype=np.complex64)
    return eps, a


def _cache_path(norb, seed, grid):
    root = os.environ.get("TETRA_SYNTH_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tetra_synth"))
    tag = hashlib.sha1(repr((_CACHE_VERSION, norb, seed, tuple(grid))).encode()).hexdigest()[:16]
    return os.path.join(root, f"tb_{norb}o_s{seed}_{grid[0]}x{grid[1]}x{grid[2]}_{tag}.npz")


def band_structure(norb: int, seed: int, grid, cache: bool = True, workers: int | None = None,
                   progress: bool = False):
    """Return ``(eps, w)``: FP32 ``eps[nb][nk]`` and ``w[nb][norb][nk]`` (nb == norb) of the seeded model.

    The diagonalisation runs on the host (numpy ``eigh`` in complex128), chunked over threads, and is
    cached as ``.npz`` because it dominates set-up time for large grids. ``progress`` prints a line to
    stderr after every tenth of the chunks.
    """
    grid = tuple(int(x) for x in grid)
    path = _cache_path(norb, seed, grid)
    if cache and os.path.exists(path):
        with np.load(path) as z:
            return z["eps"], z["w"]
    nk = grid[0] * grid[1] * grid[2]
    hops = hoppings(norb, seed)
    eps = np.empty((norb, nk), dtype=np.float32)
    w = np.empty((norb, norb, nk), dtype=np.float32)
    chunk = 8192
    bounds = [(lo, min(nk, lo + chunk)) for lo in range(0, nk, chunk)]
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))

    done = [0]
    lock = threading.Lock()

    def run(b):
        lo, hi = b
        ev, bw = _diag_chunk(hops, grid, lo, hi)
        eps[:, lo:hi] = ev.T.astype(np.float32)
        w[:, :, lo:hi] = bw.transpose(2, 1, 0).astype(np.float32)
        if progress:
            with lock:
                done[0] += 1
                if done[0] * 10 // len(bounds) != (done[0] - 1) * 10 // len(bounds):
                    print(f"[synth] eigh {grid} norb {norb}: {done[0]}/{len(bounds)} chunks", file=sys.stderr,
                          flush=True)

    if workers == 1 or len(bounds) == 1:
        for b in bounds:
            run(b)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(run, bounds))
    if cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, eps=eps, w=w)
            os.replace(tmp, path)
        except OSError:
            pass  # an unwritable cache only costs the next caller the diagonalisation
    return eps, w


def energy_grid(eps_list, ne: int, pad: float = 0.1):
    """Equidistant grid ``E_j = e0 + j*de`` (j = 0..ne-1) spanning the band range padded by ``pad``.

    ``e0`` and ``de`` are returned as exactly FP32-representable Python floats, so every consumer
    sees the same grid.
    """
    if isinstance(eps_list, np.ndarray):
        eps_list = [eps_list]
    lo = float(min(float(np.min(e)) for e in eps_list))
    hi = float(max(float(np.max(e)) for e in eps_list))
    span = hi - lo if hi > lo else 1.0  # a single energy level still gets a usable grid
    e0 = float(np.float32(lo - pad * span))
    de = float(np.float32((hi + pad * span - e0) / max(ne - 1, 1)))
    return e0, de


def cosine_band(grid, t: float = 1.0):
    """One band ``-2t(cos k1 + cos k2 + cos k3)`` with one orbital of weight 1 (FP32 SoA)."""
    n1, n2, n3 = grid
    k1, k2, k3 = np.meshgrid(*(2 * np.pi * np.arange(n) / n for n in grid), indexing="ij")
    e = (-2.0 * t * (np.cos(k1) + np.cos(k2) + np.cos(k3))).reshape(1, -1).astype(np.float32)
    return e, np.ones((1, 1, n1 * n2 * n3), dtype=np.float32)


def separable_band(values_i1, n2: int, n3: int):
    """One band depending on the slowest grid index only: ``eps[k] = values_i1[i1]``, weight 1."""
    v = np.asarray(values_i1, dtype=np.float32)
    n1 = v.shape[0]
    e = np.repeat(v, n2 * n3).reshape(1, n1 * n2 * n3)
    return e, np.ones((1, 1, n1 * n2 * n3), dtype=np.float32)


# Workloads, named by what they are. Sizes follow the benchmark set-up of Sec. IV.A (an 8-band
# model, an equidistant energy grid) scaled to one MI355X.
CONFIGS = {
    # small parity case: 16^3 grid, 8 orbitals/bands, 200 energies
    "k16_b8_e200": dict(grid=(16, 16, 16), norb=8, ne=200, seed=0),
    # headline case: 64^3 grid (1.57M tetrahedra), 8 orbitals/bands, 1000 energies
    "k64_b8_e1000": dict(grid=(64, 64, 64), norb=8, ne=1000, seed=0),
    # precision case: 128^3 grid, 16 orbitals/bands, 2000 energies, FP16 weights + Kahan
    "k128_b16_e2000": dict(grid=(128, 128, 128), norb=16, ne=2000, seed=0),
    # differentiation case: 64^3 grid, 8 orbitals/bands, 500 energies, target model seed 1
    "k64_b8_e500_fit": dict(grid=(64, 64, 64), norb=8, ne=500, seed=0, target_seed=1),
    # the paper's largest benchmark shape (60 x 60 x 10 k-points, 8 bands, 1024 energies), context only
    "k60x60x10_b8_e1024": dict(grid=(60, 60, 10), norb=8, ne=1024, seed=0),
    # susceptibility case: the headline model, transfer q = (16, 16, 0) grid steps, 500 transfer energies
    # from 0 to the band width, Fermi energy at half filling
    "chi_k64_b8_w500": dict(grid=(64, 64, 64), norb=8, nw=500, seed=0, q=(16, 16, 0)),
}


def chi_grid(eps, nw: int):
    """``(e_fermi, w0, dw)`` of a susceptibility workload: the Fermi energy at half filling (the median
    of the finite band energies) and transfer energies w_j = w0 + j*dw from 0 to the band width, all
    exactly FP32-representable."""
    fin = eps[np.isfinite(eps)]
    ef = float(np.float32(np.median(fin)))
    width = float(np.float32(fin.max()) - np.float32(fin.min()))
    return ef, 0.0, float(np.float32(width / (nw - 1)))


def config(name: str):
    return dict(CONFIGS[name])


def batched_items(n_models: int = 32, seed: int = 4242, first_model_seed: int = 100,
                  sizes=(24, 32, 48, 64, 96), ne_range=(256, 2048), scale: float = 1.0):
    """(model seed, grid, ne) for the batched workload: uneven cubic grids and energy-grid lengths.

    ``scale`` < 1 shrinks grid edges (rounded, >= 2) for quick tests while keeping the mix.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_models):
        n = int(rng.choice(np.asarray(sizes)))
        ne = int(rng.integers(ne_range[0], ne_range[1] + 1))
        if scale != 1.0:
            n = max(2, int(round(n * scale)))
        out.append((first_model_seed + i, (n, n, n), ne))
    return out
