"""Pins of the oracle's susceptibility spectral weight (the bare Lindhard susceptibility's imaginary
part at zero temperature, Im chi_0 = -pi S, by the linear tetrahedron method; the paper names
susceptibilities as the next application, Sec. I and Sec. V). CPU only.

S_m(q, w) = sum_{n,n'} (1/V_G) integral of W_m [theta(E_F - eps) theta(eps' - E_F)
            - theta(eps - E_F) theta(E_F - eps')] delta(w - (eps' - eps)) d^3k,
eps = eps_n(k), eps' = eps_n'(k + q), W_m = b_mn(k) b_mn'(k + q), all linear within each tetrahedron.

The oracle clips each tetrahedron by the two occupation half-spaces into sub-tetrahedra and applies
the corner weights of Sec. II.C to the difference energy. The pins below take other routes: the
plane section {eps' - eps = w} cut by the occupation half-planes (polygon geometry), the exact 1-D
integral of a band that is linear between grid points, the exact antisymmetry S(q, w) = -S(-q, -w)
of the method, and brute-force assembly."""
import itertools

import numpy as np
import pytest

import synth
from geometry import _affine, barycentric, volume


def _section_polygon(X, d, w):
    """Vertices of the plane section {d = w} of the tetrahedron, in cyclic order."""
    pts = []
    for i, j in itertools.combinations(range(4), 2):
        if (d[i] - w) * (d[j] - w) < 0:
            t = (w - d[i]) / (d[j] - d[i])
            pts.append(X[i] + t * (X[j] - X[i]))
    if len(pts) < 3:
        return np.zeros((0, 3))
    P = np.array(pts)
    a, _ = _affine(X, d)
    n = a / np.linalg.norm(a)
    c0 = P.mean(axis=0)
    u = P[0] - c0
    u -= n * (n @ u)
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    return P[np.argsort(np.arctan2((P - c0) @ v, (P - c0) @ u))]


def _clip_polygon(P, fun):
    """Sutherland-Hodgman: the part of the planar polygon P where the affine function fun <= 0."""
    if len(P) == 0:
        return P
    out = []
    f = [fun(p) for p in P]
    for i in range(len(P)):
        a, b = P[i], P[(i + 1) % len(P)]
        fa, fb = f[i], f[(i + 1) % len(P)]
        if fa <= 0:
            out.append(a)
        if (fa < 0 < fb) or (fb < 0 < fa):
            out.append(a + fa / (fa - fb) * (b - a))
    return np.array(out) if out else np.zeros((0, 3))


def _area_centroid(P):
    if len(P) < 3:
        return 0.0, None
    area, cen = 0.0, np.zeros(3)
    for i in range(1, len(P) - 1):
        tri = np.linalg.norm(np.cross(P[i] - P[0], P[i + 1] - P[0])) / 2.0
        area += tri
        cen += tri * (P[0] + P[i] + P[i + 1]) / 3.0
    return area, (cen / area if area > 0 else None)


def _geometry_chi(X, e, ep, W, ef, w, vol):
    """vol/V_T * (integral over the section {ep - e = w} of W times the occupation sign) / |grad(ep - e)|."""
    d = ep - e
    a, _ = _affine(X, d)
    sec = _section_polygon(X, d, w)
    ae, ce = _affine(X, e)
    ap, cp = _affine(X, ep)
    eps_at = lambda x: ae @ x + ce  # noqa: E731
    epp_at = lambda x: ap @ x + cp  # noqa: E731
    total = 0.0
    for sign, f1, f2 in ((1.0, lambda x: eps_at(x) - ef, lambda x: ef - epp_at(x)),
                         (-1.0, lambda x: ef - eps_at(x), lambda x: epp_at(x) - ef)):
        P = _clip_polygon(_clip_polygon(sec, f1), f2)
        area, cen = _area_centroid(P)
        if area > 0:
            total += sign * area * (barycentric(X, cen) @ W)
    return vol / volume(X) * total / np.linalg.norm(a)


def test_single_tetrahedron_matches_section_geometry(oracle_lib):
    rng = np.random.default_rng(17)
    checked = 0
    for _ in range(400):
        X = rng.normal(size=(4, 3))
        if volume(X) < 0.05:
            continue
        e = rng.uniform(-1, 1, 4)
        ep = rng.uniform(-1, 1, 4)
        W = rng.uniform(0.1, 1, 4)
        ef = rng.uniform(-0.5, 0.5)
        d = ep - e
        w = rng.uniform(d.min(), d.max())
        vol = rng.uniform(0.5, 2.0)
        ref = _geometry_chi(X, e, ep, W, ef, w, vol)
        got = oracle_lib.tet_chi(e, ep, W, ef, w, vol)
        assert abs(got - ref) <= 1e-9 * max(abs(ref), vol / np.ptp(d)), (got, ref)
        checked += ref != 0.0
    assert checked > 150  # most cases cut the section with at least one occupation boundary


def test_single_tetrahedron_corner_order_and_limits(oracle_lib):
    rng = np.random.default_rng(5)
    e = np.array([-0.4, 0.1, 0.3, -0.2])
    ep = np.array([0.5, -0.1, 0.9, 0.2])
    W = np.array([0.3, 0.7, 0.2, 0.9])
    for w in np.linspace(-1.5, 1.5, 31):
        ref = oracle_lib.tet_chi(e, ep, W, 0.05, w, 1.0)
        p = rng.permutation(4)
        assert oracle_lib.tet_chi(e[p], ep[p], W[p], 0.05, w, 1.0) == pytest.approx(ref, rel=1e-12, abs=1e-15)
    # everything occupied in both bands, or empty in both: no transitions
    assert oracle_lib.tet_chi(e, ep, W, 5.0, 0.3, 1.0) == 0.0
    assert oracle_lib.tet_chi(e, ep, W, -5.0, 0.3, 1.0) == 0.0
    # n fully occupied, n' fully empty: the plain DOS of the difference energy (region 1 only)
    e_low, ep_high = e - 3.0, ep + 3.0
    for w in (5.8, 6.0, 6.3):
        assert oracle_lib.tet_chi(e_low, ep_high, W, 0.0, w, 1.0) == pytest.approx(
            oracle_lib.tet_dos(ep_high - e_low, W, w, 1.0), rel=1e-12)


def _piecewise_linear_closed_form(f, b, q, ef, omegas):
    """Exact S for bands eps_n(i1) linear between grid points along axis 1 (constant along 2, 3), weights
    b_n(i1) interpolated the same way: (1/n1) sum over cells of the root contributions."""
    nb, n1 = f.shape
    out = np.zeros(len(omegas))
    for n in range(nb):
        for npr in range(nb):
            for i in range(n1):
                i2 = (i + 1) % n1
                e0_, e1_ = f[n, i], f[n, i2]
                p0, p1 = f[npr, (i + q) % n1], f[npr, (i2 + q) % n1]
                W0, W1 = b[n, i] * b[npr, (i + q) % n1], b[n, i2] * b[npr, (i2 + q) % n1]
                d0, s = p0 - e0_, (p1 - e1_) - (p0 - e0_)
                if s == 0.0:
                    continue
                for k, w in enumerate(omegas):
                    u = (w - d0) / s
                    if not 0.0 < u < 1.0:
                        continue
                    ev, epv = e0_ + u * (e1_ - e0_), p0 + u * (p1 - p0)
                    sign = 1.0 if ev <= ef <= epv else (-1.0 if epv <= ef <= ev else 0.0)
                    out[k] += sign * (W0 + u * (W1 - W0)) / abs(s) / n1
    return out


@pytest.mark.parametrize("q1", [1, 3, -2])
def test_grid_closed_form_for_bands_linear_between_grid_points(oracle_lib, q1):
    rng = np.random.default_rng(40 + q1)
    n1, n2, n3, nb = 11, 2, 3, 2
    f = rng.uniform(-1, 1, (nb, n1)).astype(np.float32).astype(np.float64)
    b = rng.uniform(0.2, 1, (nb, n1)).astype(np.float32).astype(np.float64)
    eps = np.repeat(f[:, :, None], n2 * n3, axis=2).reshape(nb, -1).astype(np.float32)
    w = np.repeat(b[:, None, :, None], n2 * n3, axis=3).reshape(nb, 1, -1).astype(np.float32)
    ef = 0.0625
    w0, dw, nw = -1.5, 0.0390625, 77
    got, _ = oracle_lib.chi(eps, w, (n1, n2, n3), (q1, 0, 0), ef, w0, dw, nw)
    omegas = w0 + dw * np.arange(nw)
    ref = _piecewise_linear_closed_form(f, b, q1, ef, omegas)
    # kinks (a root at a cell edge or on an occupation boundary) have measure zero; keep away from them
    np.testing.assert_allclose(got[:, 0], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert np.abs(ref).max() > 0.1


def test_antisymmetry_under_q_and_w_reversal(oracle_lib):
    eps, w = synth.band_structure(3, 4, (4, 3, 5))
    eps = eps.astype(np.float32)
    ef = float(np.float32(np.median(eps)))
    nw, dw = 61, 0.125
    w0 = -(nw - 1) // 2 * dw  # symmetric grid: w_j = -w_{nw-1-j} exactly
    q = (1, 2, -1)
    a, _ = oracle_lib.chi(eps, w, (4, 3, 5), q, ef, w0, dw, nw)
    b, _ = oracle_lib.chi(eps, w, (4, 3, 5), tuple(-x for x in q), ef, w0, dw, nw)
    np.testing.assert_allclose(a, -b[::-1], rtol=1e-10, atol=1e-12 * np.abs(a).max())
    assert np.abs(a).max() > 0 and np.abs(a[: nw // 2]).max() > 0  # both signs of w are exercised


def test_single_band_without_transfer_is_zero(oracle_lib):
    eps, w = synth.band_structure(1, 2, (5, 4, 3))
    got, _ = oracle_lib.chi(eps, w, (5, 4, 3), (0, 0, 0), float(np.median(eps)), -0.5, 0.01, 101)
    assert np.all(got == 0.0)


def test_grid_equals_brute_force_assembly(oracle_lib):
    rng = np.random.default_rng(8)
    grid = (3, 2, 2)
    n1, n2, n3 = grid
    nk, nb, norb = n1 * n2 * n3, 2, 2
    eps = rng.uniform(-1, 1, (nb, nk)).astype(np.float32)
    w = rng.uniform(0, 1, (nb, norb, nk)).astype(np.float32)
    q, ef = (1, 1, 0), 0.1
    w0, dw, nw = -2.0, 0.2, 21
    got, _ = oracle_lib.chi(eps, w, grid, q, ef, w0, dw, nw)
    tab = oracle_lib.table()
    vol = 1.0 / (6 * nk)
    ref = np.zeros((nw, norb))
    for i1, i2, i3 in itertools.product(range(n1), range(n2), range(n3)):
        for row in tab:
            offs = [(s & 1, (s >> 1) & 1, (s >> 2) & 1) for s in row]
            ks = [((i1 + a) % n1 * n2 + (i2 + b_) % n2) * n3 + (i3 + c) % n3 for a, b_, c in offs]
            kq = [((i1 + a + q[0]) % n1 * n2 + (i2 + b_ + q[1]) % n2) * n3 + (i3 + c + q[2]) % n3
                  for a, b_, c in offs]
            for n in range(nb):
                for npr in range(nb):
                    e, ep = eps[n, ks].astype(np.float64), eps[npr, kq].astype(np.float64)
                    for m in range(norb):
                        W = w[n, m, ks].astype(np.float64) * w[npr, m, kq].astype(np.float64)
                        for j in range(nw):
                            ref[j, m] += oracle_lib.tet_chi(e, ep, W, ef, w0 + j * dw, vol)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
