"""Pins of the oracle's grid-level DOS (eq. tetmethoorbitalresolved over the Table I tetrahedra of a
periodic grid) against brute force, closed forms, invariances and fine-grid histograms. CPU only."""
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _table_offsets():
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_tetrahedra.txt"), dtype=int)[:, 1:]
    # reading: label = 1 + o1 + 2*o2 + 4*o3, o_a the offset along grid axis a (axis 1 slowest)
    return [[((L - 1) & 1, ((L - 1) >> 1) & 1, ((L - 1) >> 2) & 1) for L in row] for row in rows]


def _brute_force_dos(oracle_lib, eps, w, grid, e0, de, ne):
    """Python loop over cubes/tetrahedra/bands/orbitals/energies around the pinned one-tetrahedron oracle."""
    n1, n2, n3 = grid
    nk = n1 * n2 * n3
    nb, norb = w.shape[0], w.shape[1]
    vol = 1.0 / (6 * nk)
    dos = np.zeros((ne, norb))
    tets = _table_offsets()
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                for tet in tets:
                    ks = [((i1 + o1) % n1 * n2 + (i2 + o2) % n2) * n3 + (i3 + o3) % n3 for o1, o2, o3 in tet]
                    for n in range(nb):
                        e = eps[n, ks].astype(np.float64)
                        for m in range(norb):
                            b = w[n, m, ks].astype(np.float64)
                            for j in range(ne):
                                dos[j, m] += oracle_lib.tet_dos(e, b, e0 + j * de, vol)
    return dos


def _random_inputs(rng, grid, nb, norb):
    nk = int(np.prod(grid))
    eps = rng.uniform(-1, 1, (nb, nk)).astype(np.float32)
    w = rng.uniform(0, 1, (nb, norb, nk)).astype(np.float32)
    return eps, w


@pytest.mark.parametrize("grid", [(3, 2, 4), (1, 3, 2), (2, 1, 1)])
def test_grid_equals_brute_force_assembly(oracle_lib, grid):
    rng = np.random.default_rng(sum(grid))
    eps, w = _random_inputs(rng, grid, 2, 3)
    e0, de, ne = -1.2, 0.083, 30
    ref = _brute_force_dos(oracle_lib, eps, w, grid, e0, de, ne)
    got, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_non_finite_energy_drops_only_its_tetrahedra(oracle_lib):
    rng = np.random.default_rng(3)
    grid = (3, 3, 2)
    eps, w = _random_inputs(rng, grid, 2, 2)
    eps[1, 5] = np.nan
    eps[0, 7] = np.inf
    e0, de, ne = -1.2, 0.1, 26
    ref = _brute_force_dos(oracle_lib, eps, w, grid, e0, de, ne)
    got, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_window_count_matches_direct_count(oracle_lib):
    rng = np.random.default_rng(4)
    grid = (4, 3, 5)
    n1, n2, n3 = grid
    eps, w = _random_inputs(rng, grid, 3, 1)
    e0, de, ne = -1.1, 0.05, 45
    _, cnt = oracle_lib.dos(eps, w, grid, e0, de, ne)
    Ej = e0 + de * np.arange(ne)
    total = 0
    for tet in _table_offsets():
        ks = []
        for o1, o2, o3 in tet:
            i1, i2, i3 = np.meshgrid((np.arange(n1) + o1) % n1, (np.arange(n2) + o2) % n2,
                                     (np.arange(n3) + o3) % n3, indexing="ij")
            ks.append(((i1 * n2 + i2) * n3 + i3).ravel())
        e = np.stack([eps[:, k] for k in ks]).astype(np.float64)  # [4, nb, ncubes]
        lo, hi = e.min(axis=0), e.max(axis=0)
        total += int(((Ej[None, None, :] > lo[..., None]) & (Ej[None, None, :] < hi[..., None])).sum())
    assert cnt == total


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_separable_band_closed_form(oracle_lib, axis):
    """eps depends on one grid index only: the DOS is (1/n_a) sum_i 1[E between f_i, f_i+1] / |f_i+1 - f_i|."""
    rng = np.random.default_rng(40 + axis)
    dims = [5, 3, 4]
    na = dims[axis]
    f = rng.uniform(-1, 1, na).astype(np.float32)
    idx = np.meshgrid(*(np.arange(d) for d in dims), indexing="ij")[axis].ravel()
    eps = f[idx][None, :].astype(np.float32)
    w = np.ones((1, 1, eps.shape[1]), dtype=np.float32)
    e0, de, ne = -1.3, 0.0173, 150
    got, _ = oracle_lib.dos(eps, w, dims, e0, de, ne)
    ff = f.astype(np.float64)
    for j in range(ne):
        E = e0 + j * de
        ref = 0.0
        near = False
        for i in range(na):
            a, b = ff[i], ff[(i + 1) % na]
            lo, hi = min(a, b), max(a, b)
            near |= min(abs(E - a), abs(E - b)) < 1e-9
            if lo < E < hi:
                ref += 1.0 / (na * (hi - lo))
        if not near:
            assert got[j, 0] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_periodic_translation_invariance(oracle_lib):
    rng = np.random.default_rng(5)
    grid = (4, 5, 3)
    eps, w = _random_inputs(rng, grid, 2, 3)
    e0, de, ne = -1.1, 0.04, 60
    ref, cref = oracle_lib.dos(eps, w, grid, e0, de, ne)
    shift = (1, 3, 2)
    eps_r = np.roll(eps.reshape(2, *grid), shift, axis=(1, 2, 3)).reshape(eps.shape)
    w_r = np.roll(w.reshape(2, 3, *grid), shift, axis=(2, 3, 4)).reshape(w.shape)
    got, cnt = oracle_lib.dos(eps_r, w_r, grid, e0, de, ne)
    assert cnt == cref
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_energy_reflection(oracle_lib):
    """eps -> -eps maps DOS(E) to DOS(-E) on the reversed grid."""
    rng = np.random.default_rng(6)
    grid = (3, 4, 4)
    eps, w = _random_inputs(rng, grid, 2, 2)
    e0, de, ne = -1.05, 0.03, 71
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    e0r = -(e0 + (ne - 1) * de)
    got, _ = oracle_lib.dos(-eps, w, grid, e0r, de, ne)
    np.testing.assert_allclose(got[::-1], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_energy_scaling(oracle_lib):
    """eps -> 2 eps with the grid scaled alike divides the DOS by 2 (exact in binary)."""
    rng = np.random.default_rng(7)
    grid = (3, 3, 3)
    eps, w = _random_inputs(rng, grid, 2, 2)
    e0, de, ne = -1.05, 0.03, 71
    ref, _ = oracle_lib.dos(eps, w, grid, e0, de, ne)
    got, _ = oracle_lib.dos(2 * eps, w, grid, 2 * e0, 2 * de, ne)
    np.testing.assert_allclose(got, ref / 2, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_linearity_in_weights_and_orbital_sum(oracle_lib):
    eps, w = synth.band_structure(4, 3, (6, 5, 4))
    e0, de = synth.energy_grid(eps, 90)
    dos, _ = oracle_lib.dos(eps, w, (6, 5, 4), e0, de, 90)
    tot, _ = oracle_lib.dos(eps, np.ones((4, 1, eps.shape[1]), np.float32), (6, 5, 4), e0, de, 90)
    # sum_m b_mn = 1 up to FP32 rounding of the weights
    np.testing.assert_allclose(dos.sum(axis=1), tot[:, 0], rtol=2e-6, atol=1e-7 * tot.max())
    # exact linearity: DOS(b + b') = DOS(b) + DOS(b') for weights whose sum is exact in FP32
    w2 = (w * 0.5).astype(np.float32)
    d2, _ = oracle_lib.dos(eps, w2, (6, 5, 4), e0, de, 90)
    np.testing.assert_allclose(2 * d2, dos, rtol=1e-13, atol=1e-15)


def test_sum_rule(oracle_lib):
    """Integrated weights above every band give the mean orbital weight (= 1 by unitarity); the
    trapezoid integral of the point-sampled DOS is 1 up to quadrature error."""
    grid = (16, 16, 16)
    eps, w = synth.band_structure(8, 0, grid)
    e0, de = synth.energy_grid(eps, 200)
    top = float(np.max(eps)) + 0.5
    n, = oracle_lib.nos(eps, w, grid, top, 1.0, 1)
    mean_b = w.astype(np.float64).sum(axis=(0, 2)) / eps.shape[1]
    np.testing.assert_allclose(n, mean_b, rtol=1e-12)
    np.testing.assert_allclose(mean_b, 1.0, atol=1e-6)
    dos, _ = oracle_lib.dos(eps, w, grid, e0, de, 200)
    integral = np.trapezoid(dos, dx=de, axis=0)
    np.testing.assert_allclose(integral, 1.0, atol=5e-3)
    assert abs(integral.sum() - 8.0) < 2e-2


def test_nos_differences_integrate_dos(oracle_lib):
    """N(E_j+1) - N(E_j) is the integral of the point DOS over [E_j, E_j+1]: the DOS is continuous
    and piecewise cubic, so a trapezoid rule on a 512x refined grid reproduces it closely."""
    grid = (4, 4, 3)
    eps, w = synth.band_structure(3, 5, grid)
    e0, de = synth.energy_grid(eps, 12)
    nos = oracle_lib.nos(eps, w, grid, e0, de, 12)
    sub = 512
    dfine, _ = oracle_lib.dos(eps, w, grid, e0, de / sub, 11 * sub + 1)
    diffs = np.diff(nos, axis=0)
    for j in range(11):
        seg = dfine[j * sub:(j + 1) * sub + 1]
        trap = de / sub * (seg.sum(axis=0) - 0.5 * (seg[0] + seg[-1]))
        np.testing.assert_allclose(diffs[j], trap, rtol=1e-4, atol=1e-4 * np.abs(diffs).max())


def test_histogram_convergence_cosine_band(oracle_lib):
    """Bin-averaged tetrahedron DOS of -2(cos k1 + cos k2 + cos k3) approaches a brute-force fine-grid
    histogram as the grid is refined."""
    edges = np.linspace(-6.2, 6.2, 32)
    width = edges[1] - edges[0]
    M = 240
    k = 2 * np.pi * (np.arange(M) + 0.5) / M
    c = np.cos(k)
    fine = -2 * (c[:, None, None] + c[None, :, None] + c[None, None, :])
    hist = np.histogram(fine.ravel(), bins=edges)[0] / (fine.size * width)
    errs = []
    for N in (6, 12, 24):
        eps, w = synth.cosine_band((N, N, N))
        nos = oracle_lib.nos(eps, w, (N, N, N), edges[0], width, len(edges))
        binned = oracle_lib.dos_binned(eps, w, (N, N, N), edges[0] + 0.5 * width, width, len(edges) - 1)[:, 0]
        np.testing.assert_allclose(binned, np.diff(nos[:, 0]) / width, rtol=1e-12, atol=1e-12)
        errs.append(np.abs(binned - hist).sum() * width)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_bench_window_count_matches_oracle(oracle_lib):
    """The benchmark's in-window update count (the unit of its roofline) equals the oracle's count."""
    import bench

    for grid, norb, ne in (((16, 16, 16), 8, 200), ((5, 3, 7), 3, 333)):
        eps, w = synth.band_structure(norb, 1, grid)
        e0, de = synth.energy_grid(eps, ne)
        _, cnt = oracle_lib.dos(eps, w, grid, e0, de, ne)
        assert bench.count_window_updates(eps, grid, e0, de, ne) == cnt


def test_bench_step_count_brute_force():
    """The benchmark's number-of-states update count (the unit of its roofline): per tetrahedron-band,
    the grid indices from the first E_j > E1 to the first E_j >= E4, clipped to the grid with
    everything below it at index 0; brute force over the tetrahedra of a small grid."""
    import bench

    grid, ne = (5, 3, 4), 37
    eps, _ = synth.band_structure(3, 2, grid)
    n1, n2, n3 = grid
    lo, hi = float(eps.min()), float(eps.max())
    for origin_frac, joff in ((0.3, 0.0), (-0.2, -0.5), (0.9, 0.0)):
        e0 = float(np.float32(lo + origin_frac * (hi - lo)))
        de = float(np.float32(0.6 * (hi - lo) / ne))
        E = e0 + (np.arange(ne) + joff) * de
        want = 0
        for n in range(eps.shape[0]):
            for i1 in range(n1):
                for i2 in range(n2):
                    for i3 in range(n3):
                        for tet in bench.table1_offsets():
                            c = [eps[n, ((i1 + o[0]) % n1 * n2 + (i2 + o[1]) % n2) * n3 + (i3 + o[2]) % n3] for o in tet]
                            e1, e4 = float(min(c)), float(max(c))
                            above = np.nonzero(E > e1)[0]
                            ja = above[0] if len(above) else ne
                            reach = np.nonzero(E >= e4)[0]
                            js = reach[0] if len(reach) else ne
                            if ja < ne or js < ne:
                                want += min(js, ne - 1) - min(ja, js) + 1
        assert bench.count_step_updates(eps, grid, e0, de, ne, joff) == want
