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
from .tb import (
    hoppings,
    hamiltonians,
    amplitudes,
    band_structure,
    energy_grid,
    chi_grid,
    cosine_band,
    separable_band,
    CONFIGS,
    config,
    batched_items,
)

__all__ = [
    "hoppings",
    "hamiltonians",
    "amplitudes",
    "band_structure",
    "energy_grid",
    "chi_grid",
    "cosine_band",
    "separable_band",
    "CONFIGS",
    "config",
    "batched_items",
]
