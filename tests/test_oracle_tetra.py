"""Pins of the oracle's single-tetrahedron corner weights (Sec. II.C) against facts that do not come
from the oracle itself: geometry of plane sections, Bloechl's total-DOS closed form, derivative and
normalisation identities, symmetries and degenerate limits. CPU only."""
import os

import numpy as np
import pytest

from geometry import corner_dos, corner_nos, volume

HERE = os.path.dirname(os.path.abspath(__file__))
VOL = 0.37  # arbitrary V_T/V_G; every weight scales with it


def _sorted_sets(rng, n, spread=1.0):
    out = []
    for _ in range(n):
        e = np.sort(rng.uniform(-spread, spread, 4))
        if np.min(np.diff(e)) < 1e-3:
            continue
        out.append(e)
    return out


def _energies_inside(e, rng, per_interval=3):
    """Energies strictly inside each of the three sub-intervals, away from the corners."""
    Es = []
    for a, b in ((e[0], e[1]), (e[1], e[2]), (e[2], e[3])):
        for u in rng.uniform(0.02, 0.98, per_interval):
            Es.append(a + u * (b - a))
    return Es


def test_table1_matches_paper(oracle_lib):
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_tetrahedra.txt"), dtype=int)
    assert rows.shape == (6, 5)
    assert np.array_equal(rows[:, 0], np.arange(1, 7))
    assert np.array_equal(oracle_lib.table() + 1, rows[:, 1:])


def _slot_xyz(slot):
    # reading: label = 1 + o1 + 2*o2 + 4*o3
    return np.array([slot & 1, (slot >> 1) & 1, (slot >> 2) & 1], dtype=float)


def test_table1_tiles_the_cube(oracle_lib):
    """Six tetrahedra of volume 1/6 each, covering every interior point of the cube exactly once."""
    tab = oracle_lib.table()
    tets = [np.array([_slot_xyz(s) for s in row]) for row in tab]
    for X in tets:
        assert volume(X) == pytest.approx(1.0 / 6.0, abs=1e-14)
    rng = np.random.default_rng(11)
    pts = rng.uniform(0, 1, (4000, 3))
    count = np.zeros(len(pts), dtype=int)
    for X in tets:
        M = np.vstack([X.T, np.ones((1, 4))])
        lam = np.linalg.solve(M, np.vstack([pts.T, np.ones((1, len(pts)))]))
        count += np.all(lam > -1e-12, axis=0)
    assert np.all(count == 1)
    inc = np.bincount(tab.ravel(), minlength=8)
    assert inc.sum() == 24 and sorted(inc.tolist()) == [2, 2, 2, 2, 2, 2, 6, 6]


@pytest.mark.parametrize("seed", range(4))
def test_corner_dos_equals_section_geometry(oracle_lib, seed):
    """dw_l/dE of every corner equals the section integral of its barycentric coordinate."""
    rng = np.random.default_rng(seed)
    for e in _sorted_sets(rng, 6):
        X = rng.normal(size=(4, 3))
        if volume(X) < 0.05:
            continue
        for E in _energies_inside(e, rng):
            _, g = oracle_lib.corner_weights(e, E, VOL)
            ref = corner_dos(X, e, E, VOL)
            np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12 * VOL)


@pytest.mark.parametrize("seed", range(3))
def test_corner_nos_equals_clipped_volume_geometry(oracle_lib, seed):
    """w_l(E) equals the clipped-volume integral of each barycentric coordinate."""
    rng = np.random.default_rng(100 + seed)
    for e in _sorted_sets(rng, 5):
        X = rng.normal(size=(4, 3))
        if volume(X) < 0.05:
            continue
        for E in list(_energies_inside(e, rng, 2)) + [e[0] - 0.5, e[3] + 0.5]:
            w, _ = oracle_lib.corner_weights(e, E, VOL)
            ref = corner_nos(X, e, E, VOL)
            np.testing.assert_allclose(w, ref, rtol=1e-9, atol=1e-12 * VOL)


def _bloechl_total(e, E, vol):
    """Total DOS of one tetrahedron (Bloechl 1994), piecewise quadratic."""
    E1, E2, E3, E4 = e
    E21, E31, E41, E32, E42, E43 = E2 - E1, E3 - E1, E4 - E1, E3 - E2, E4 - E2, E4 - E3
    if E <= E1 or E >= E4:
        return 0.0
    if E <= E2:
        return 3 * vol * (E - E1) ** 2 / (E21 * E31 * E41)
    if E <= E3:
        return vol / (E31 * E41) * (3 * E21 + 6 * (E - E2) - 3 * (E31 + E42) * (E - E2) ** 2 / (E32 * E42))
    return 3 * vol * (E4 - E) ** 2 / (E41 * E42 * E43)


@pytest.mark.parametrize("seed", range(4))
def test_sum_of_corners_is_bloechl_total_dos(oracle_lib, seed):
    rng = np.random.default_rng(20 + seed)
    for e in _sorted_sets(rng, 50, spread=3.0):
        for E in _energies_inside(e, rng) + list(e):
            _, g = oracle_lib.corner_weights(e, E, VOL)
            assert g.sum() == pytest.approx(_bloechl_total(e, E, VOL), rel=1e-12, abs=1e-14)


def test_integrated_weights_sum_to_occupied_volume(oracle_lib):
    """sum_l w_l(E) = vol * (volume fraction of the tetrahedron below E)."""
    from scipy.integrate import quad

    rng = np.random.default_rng(5)
    for e in _sorted_sets(rng, 40):
        E1, E2, E3, E4 = e
        for E in _energies_inside(e, rng):
            w, _ = oracle_lib.corner_weights(e, E, VOL)
            if E <= E2:  # a small corner tetrahedron
                frac = (E - E1) ** 3 / ((E2 - E1) * (E3 - E1) * (E4 - E1))
            elif E <= E3:  # antiderivative of the total DOS closed form
                frac = quad(lambda x: _bloechl_total(e, x, 1.0), E1, E, points=[E2], epsabs=1e-14)[0]
            else:  # everything but a small corner tetrahedron at the top
                frac = 1 - (E4 - E) ** 3 / ((E4 - E1) * (E4 - E2) * (E4 - E3))
            assert w.sum() == pytest.approx(VOL * frac, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_density_weights_are_energy_derivatives(oracle_lib, seed):
    """The printed dw_l/dE agree with central differences of the printed w_l (catches the middle-case typo)."""
    rng = np.random.default_rng(30 + seed)
    h = 1e-6
    for e in _sorted_sets(rng, 30):
        for E in _energies_inside(e, rng):
            if np.min(np.abs(E - e)) < 10 * h:
                continue
            wp, _ = oracle_lib.corner_weights(e, E + h, VOL)
            wm, _ = oracle_lib.corner_weights(e, E - h, VOL)
            _, g = oracle_lib.corner_weights(e, E, VOL)
            np.testing.assert_allclose(g, (wp - wm) / (2 * h), rtol=1e-6, atol=1e-8 * VOL)


def test_each_corner_integrates_to_a_quarter(oracle_lib):
    """Each g_l is a cubic on every sub-interval, so Simpson per sub-interval integrates it exactly."""
    rng = np.random.default_rng(6)
    for e in _sorted_sets(rng, 40):
        total = np.zeros(4)
        for a, b in ((e[0], e[1]), (e[1], e[2]), (e[2], e[3])):
            # interior nodes only touch one case; endpoints are approached from inside
            d = (b - a) * 1e-13
            ga = oracle_lib.corner_weights(e, a + d, VOL)[1]
            gm = oracle_lib.corner_weights(e, 0.5 * (a + b), VOL)[1]
            gb = oracle_lib.corner_weights(e, b - d, VOL)[1]
            total += (b - a) / 6.0 * (ga + 4 * gm + gb)
        np.testing.assert_allclose(total, VOL / 4.0, rtol=1e-9)


def test_continuity_and_vanishing_ends(oracle_lib):
    rng = np.random.default_rng(7)
    for e in _sorted_sets(rng, 40):
        span = e[3] - e[0]
        d = 1e-9 * span
        for Ec in (e[1], e[2]):
            wl, gl = oracle_lib.corner_weights(e, Ec - d, VOL)
            wr, gr = oracle_lib.corner_weights(e, Ec + d, VOL)
            np.testing.assert_allclose(gl, gr, rtol=1e-6, atol=1e-9 * VOL / span)
            np.testing.assert_allclose(wl, wr, rtol=1e-6, atol=1e-9 * VOL)
        g1 = oracle_lib.corner_weights(e, e[0] + d, VOL)[1]
        g4 = oracle_lib.corner_weights(e, e[3] - d, VOL)[1]
        assert np.max(np.abs(g1)) < 1e-6 * VOL / span
        assert np.max(np.abs(g4)) < 1e-6 * VOL / span
        assert np.all(oracle_lib.corner_weights(e, e[0], VOL)[1] == 0)
        assert np.all(oracle_lib.corner_weights(e, e[3], VOL)[1] == 0)
        np.testing.assert_allclose(oracle_lib.corner_weights(e, e[3] + 1, VOL)[0], VOL / 4)


def test_reflection_symmetry(oracle_lib):
    """g_l(E; E1..E4) = g_{5-l}(-E; -E4..-E1): the first and third cases mirror each other."""
    rng = np.random.default_rng(8)
    for e in _sorted_sets(rng, 40):
        r = -e[::-1]
        for E in _energies_inside(e, rng):
            g = oracle_lib.corner_weights(e, E, VOL)[1]
            gr = oracle_lib.corner_weights(r, -E, VOL)[1]
            np.testing.assert_allclose(g, gr[::-1], rtol=1e-11, atol=1e-14)


def test_linear_exactness(oracle_lib):
    """sum_l E_l g_l(E) = E sum_l g_l(E): a linear function of energy is integrated exactly."""
    rng = np.random.default_rng(9)
    for e in _sorted_sets(rng, 40):
        for E in _energies_inside(e, rng):
            g = oracle_lib.corner_weights(e, E, VOL)[1]
            assert np.dot(e, g) == pytest.approx(E * g.sum(), rel=1e-11, abs=1e-14)


def test_corner_permutation_invariance(oracle_lib):
    rng = np.random.default_rng(10)
    import itertools

    for _ in range(20):
        e = rng.uniform(-1, 1, 4)
        b = rng.uniform(0, 1, 4)
        for E in np.linspace(e.min(), e.max(), 9)[1:-1]:
            ref = oracle_lib.tet_dos(e, b, E, VOL)
            for p in itertools.permutations(range(4)):
                p = list(p)
                assert oracle_lib.tet_dos(e[p], b[p], E, VOL) == pytest.approx(ref, rel=1e-13, abs=1e-16)


DEGENERATE = [
    [0.0, 0.0, 0.4, 1.0],
    [0.0, 0.3, 0.3, 1.0],
    [0.0, 0.3, 1.0, 1.0],
    [0.0, 0.0, 1.0, 1.0],
    [0.0, 0.0, 0.0, 1.0],
    [0.0, 1.0, 1.0, 1.0],
]


@pytest.mark.parametrize("e", DEGENERATE)
def test_degenerate_corners_are_finite_limits(oracle_lib, e):
    e = np.array(e)
    split = e + np.array([0.0, 1e-10, 2e-10, 3e-10])
    for E in np.linspace(-0.1, 1.1, 49):
        w, g = oracle_lib.corner_weights(e, E, VOL)
        ws, gs = oracle_lib.corner_weights(split, E, VOL)
        assert np.all(np.isfinite(g)) and np.all(np.isfinite(w))
        if np.min(np.abs(E - e)) > 1e-6:
            np.testing.assert_allclose(g, gs, rtol=1e-6, atol=1e-8)
            np.testing.assert_allclose(w, ws, rtol=1e-6, atol=1e-8)


def test_all_equal_corners_contribute_nothing(oracle_lib):
    e = np.full(4, 0.25)
    for E in (0.0, 0.25, 0.5):
        assert np.all(oracle_lib.corner_weights(e, E, VOL)[1] == 0)


def test_energy_on_a_corner_is_the_one_sided_limit(oracle_lib):
    rng = np.random.default_rng(12)
    for e in _sorted_sets(rng, 20):
        d = 1e-9 * (e[3] - e[0])
        for Ec in e[1:3]:
            g = oracle_lib.corner_weights(e, Ec, VOL)[1]
            gl = oracle_lib.corner_weights(e, Ec - d, VOL)[1]
            np.testing.assert_allclose(g, gl, rtol=1e-6, atol=1e-9)


def test_weight_derivatives_match_finite_differences(oracle_lib):
    """The dual-number partials d(dw_l/dE)/dE_i agree with central differences in FP64."""
    rng = np.random.default_rng(13)
    h = 1e-6
    for e in _sorted_sets(rng, 30):
        for E in _energies_inside(e, rng, 2):
            if np.min(np.abs(E - e)) < 1e-3:
                continue
            g, dg = oracle_lib.corner_weights_grad(e, E, VOL)
            for i in range(4):
                ep, em = e.copy(), e.copy()
                ep[i] += h
                em[i] -= h
                fd = (oracle_lib.corner_weights(ep, E, VOL)[1] - oracle_lib.corner_weights(em, E, VOL)[1]) / (2 * h)
                np.testing.assert_allclose(dg[:, i], fd, rtol=2e-5, atol=1e-7 * VOL)


@pytest.mark.parametrize("seed", range(3))
def test_tet_contributions_on_unsorted_corners_equal_geometry(oracle_lib, seed):
    """One tetrahedron's contributions with its corners in arbitrary order (Sec. II.C, summed with
    the corner values b as in eq. tetracontriborbitalresolved): sum_l b_l w_l(E) equals the
    clipped-volume integral and sum_l b_l dw_l/dE the section integral of the linear interpolant of b,
    both from plane geometry in the corners' own order. Distinct b per corner, so an unsorted b or a
    density weight in place of an integrated one fails."""
    rng = np.random.default_rng(300 + seed)
    done = 0
    while done < 6:
        e = rng.uniform(-1, 1, 4)
        if np.min(np.diff(np.sort(e))) < 1e-3:
            continue
        X = rng.normal(size=(4, 3))
        if volume(X) < 0.05:
            continue
        b = rng.uniform(0.1, 1.0, 4)
        es = np.sort(e)
        Es = list(_energies_inside(es, rng, 2)) + [es[0] - 0.3, es[3] + 0.3]
        for E in Es:
            ref_n = float(b @ corner_nos(X, e, E, VOL))
            ref_d = float(b @ corner_dos(X, e, E, VOL))
            assert oracle_lib.tet_nos(e, b, E, VOL) == pytest.approx(ref_n, rel=1e-9, abs=1e-12 * VOL)
            assert oracle_lib.tet_dos(e, b, E, VOL) == pytest.approx(ref_d, rel=1e-9, abs=1e-12 * VOL)
        done += 1


def test_tet_nos_permutation_invariance_and_limits(oracle_lib):
    """Permuting the (energy, b) corner pairs leaves sum_l b_l w_l unchanged; below E1 it is zero and
    above E4 it is V_T/(4 V_G) times the sum of the b values (Sec. II.C, fifth case)."""
    import itertools

    rng = np.random.default_rng(12)
    for _ in range(10):
        e = rng.uniform(-1, 1, 4)
        b = rng.uniform(0, 1, 4)
        assert oracle_lib.tet_nos(e, b, e.min() - 0.1, VOL) == 0.0
        assert oracle_lib.tet_nos(e, b, e.max() + 0.1, VOL) == pytest.approx(VOL / 4 * b.sum(), rel=1e-14)
        for E in np.linspace(e.min(), e.max(), 7)[1:-1]:
            ref = oracle_lib.tet_nos(e, b, E, VOL)
            for p in itertools.permutations(range(4)):
                p = list(p)
                assert oracle_lib.tet_nos(e[p], b[p], E, VOL) == pytest.approx(ref, rel=1e-13, abs=1e-16)
