"""Pins of the oracle's analytic gradient of L = sum_{j,m} G[j,m] DOS[j,m] with respect to the band
energies and orbital weights: exact linearity in the weights, central finite differences in the
energies away from kinks. CPU only."""
import numpy as np
import pytest

import synth

GRID = (5, 4, 3)


def _setup(seed):
    eps, w = synth.band_structure(3, seed, GRID)
    e0, de = synth.energy_grid(eps, 40)
    G = np.random.default_rng(seed + 50).normal(size=(40, 3))
    return eps, w, e0, de, G


def _loss(oracle_lib, eps, w, e0, de, G):
    d, _ = oracle_lib.dos(eps, w, GRID, e0, de, G.shape[0])
    return float((G * d).sum())


def _neighbours(k):
    """k-points sharing a tetrahedron with k (the 3x3x3 block around it, periodic)."""
    n1, n2, n3 = GRID
    i1, i2, i3 = k // (n2 * n3), (k // n3) % n2, k % n3
    out = []
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                out.append((((i1 + a) % n1) * n2 + (i2 + b) % n2) * n3 + (i3 + c) % n3)
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_weight_gradient_is_exact(oracle_lib, seed):
    eps, w, e0, de, G = _setup(seed)
    _, gw = oracle_lib.dos_backward(eps, w, GRID, e0, de, G)
    L0 = _loss(oracle_lib, eps, w, e0, de, G)
    rng = np.random.default_rng(seed)
    for _ in range(25):
        n, m, k = rng.integers(3), rng.integers(3), rng.integers(eps.shape[1])
        w2 = w.copy()
        w2[n, m, k] = np.float32(w2[n, m, k] + np.float32(0.25))
        delta = float(w2[n, m, k]) - float(w[n, m, k])
        fd = (_loss(oracle_lib, eps, w2, e0, de, G) - L0) / delta
        assert fd == pytest.approx(gw[n, m, k], rel=1e-9, abs=1e-12 * np.abs(gw).max())


@pytest.mark.parametrize("seed", [1, 2])
def test_energy_gradient_matches_central_differences(oracle_lib, seed):
    eps, w, e0, de, G = _setup(seed)
    ge, _ = oracle_lib.dos_backward(eps, w, GRID, e0, de, G)
    h = 2e-4
    Ej = e0 + de * np.arange(G.shape[0])
    rng = np.random.default_rng(seed + 7)
    checked = 0
    for _ in range(200):
        n, k = rng.integers(3), rng.integers(eps.shape[1])
        x = float(eps[n, k])
        partners = [float(eps[n, q]) for q in _neighbours(k) if q != k]
        if np.min(np.abs(Ej - x)) < 10 * h or np.min(np.abs(np.array(partners) - x)) < 10 * h:
            continue  # kink: a grid energy or a partner corner is within reach of the perturbation
        ep, em = eps.copy(), eps.copy()
        ep[n, k] = np.float32(x + h)
        em[n, k] = np.float32(x - h)
        span = float(ep[n, k]) - float(em[n, k])
        fd = (_loss(oracle_lib, ep, w, e0, de, G) - _loss(oracle_lib, em, w, e0, de, G)) / span
        assert fd == pytest.approx(ge[n, k], rel=2e-4, abs=1e-6 * np.abs(ge).max())
        checked += 1
        if checked == 40:
            break
    assert checked >= 20


def test_gradient_of_separable_band_closed_form(oracle_lib):
    """For eps = f(i1) and b = 1 the DOS is (1/n1) sum_i 1[E in (f_i, f_i+1)] / |f_i+1 - f_i|, whose
    derivative with respect to f_i is known in closed form."""
    n1, n2, n3 = 5, 2, 3
    f = np.array([-0.8, -0.1, 0.35, 0.9, 0.2], dtype=np.float32)
    idx = np.repeat(np.arange(n1), n2 * n3)
    eps = f[idx][None, :]
    w = np.ones((1, 1, eps.shape[1]), dtype=np.float32)
    e0, de, ne = -1.0, 0.0371, 60
    G = np.random.default_rng(3).normal(size=(ne, 1))
    ge, _ = oracle_lib.dos_backward(eps, w, (n1, n2, n3), e0, de, G)
    ff = f.astype(np.float64)
    ref = np.zeros(n1)
    for j in range(ne):
        E = e0 + j * de
        for i in range(n1):
            a, b = ff[i], ff[(i + 1) % n1]
            lo, hi = min(a, b), max(a, b)
            if lo < E < hi:
                # d/da of 1/(n1 |b - a|) = sign(b - a) / (n1 (b - a)^2)
                s = 1.0 / (n1 * (b - a) ** 2) * np.sign(b - a)
                ref[i] += G[j, 0] * s
                ref[(i + 1) % n1] -= G[j, 0] * s
    got = ge[0].reshape(n1, n2 * n3).sum(axis=1)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("grid", [(1, 3, 4), (2, 3, 3), (3, 2, 5), (5, 4, 3), (6, 3, 2)])
def test_oracle_results_do_not_depend_on_the_thread_count(oracle_lib, grid):
    """The forward's slabs and the backward's (band, slab) phases sum every element in a fixed order,
    so one thread and eight give the same bits (odd and even slab counts, a single slab)."""
    eps, w = synth.band_structure(3, 21, grid)
    e0, de = synth.energy_grid(eps, 60)
    G = np.random.default_rng(3).normal(size=(60, 3))
    d1, c1 = oracle_lib.dos(eps, w, grid, e0, de, 60, nthreads=1)
    d8, c8 = oracle_lib.dos(eps, w, grid, e0, de, 60, nthreads=8)
    assert c1 == c8 and np.array_equal(d1, d8)
    e1, w1 = oracle_lib.dos_backward(eps, w, grid, e0, de, G, nthreads=1)
    e8, w8 = oracle_lib.dos_backward(eps, w, grid, e0, de, G, nthreads=8)
    assert np.array_equal(e1, e8) and np.array_equal(w1, w8)
    assert np.abs(e1).max() > 0 and np.abs(w1).max() > 0
