"""Independent geometry for pinning the oracle's corner weights.

For a tetrahedron with vertices X_l, energies e_l interpolated linearly (eps(x) = a.x + c) and
barycentric coordinates lambda_l(x), the linear tetrahedron method assigns corner l the integrated
weight and the density weight

    w_l(E)  = (vol / V_T) * integral over {x in T : eps(x) < E} of lambda_l(x) dV
    g_l(E)  = dw_l/dE = (vol / V_T) * integral over {x in T : eps(x) = E} of lambda_l(x) dS / |a|

with vol = V_T/V_G. Both integrands are linear, so each integral equals the measure of the clipped
region times lambda_l at its centroid. This module computes those regions directly (plane clipping,
triangle fans, a Delaunay split of the clipped polytope); it shares nothing with the paper's case
formulas.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import Delaunay


def _affine(X, e):
    A = np.hstack([X, np.ones((4, 1))])
    coef = np.linalg.solve(A, e)
    return coef[:3], coef[3]


def barycentric(X, x):
    M = np.vstack([X.T, np.ones((1, 4))])
    return np.linalg.solve(M, np.append(x, 1.0))


def volume(X):
    return abs(np.linalg.det(X[1:] - X[0])) / 6.0


def _edge_points(X, e, E):
    pts = []
    for i, j in itertools.combinations(range(4), 2):
        if (e[i] - E) * (e[j] - E) < 0:
            t = (E - e[i]) / (e[j] - e[i])
            pts.append(X[i] + t * (X[j] - X[i]))
    return np.array(pts)


def section(X, e, E):
    """(area, centroid) of the plane section {eps = E} of the tetrahedron."""
    a, _ = _affine(X, e)
    P = _edge_points(X, e, E)
    if len(P) < 3:
        return 0.0, None
    n = a / np.linalg.norm(a)
    c0 = P.mean(axis=0)
    u = P[0] - c0
    u -= n * (n @ u)
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    ang = np.arctan2((P - c0) @ v, (P - c0) @ u)
    P = P[np.argsort(ang)]
    area = 0.0
    cen = np.zeros(3)
    for i in range(1, len(P) - 1):
        tri = np.linalg.norm(np.cross(P[i] - P[0], P[i + 1] - P[0])) / 2.0
        area += tri
        cen += tri * (P[0] + P[i] + P[i + 1]) / 3.0
    return area, cen / area


def lower_region(X, e, E):
    """(volume, centroid) of {x in T : eps(x) < E}."""
    below = [X[i] for i in range(4) if e[i] < E]
    if not below:
        return 0.0, None
    P = np.vstack([np.array(below)] + ([_edge_points(X, e, E)] if len(below) < 4 else []))
    if len(P) < 4:
        return 0.0, None
    tri = Delaunay(P)
    vtot = 0.0
    cen = np.zeros(3)
    for s in tri.simplices:
        Q = P[s]
        vol = volume(Q)
        vtot += vol
        cen += vol * Q.mean(axis=0)
    return vtot, cen / vtot


def corner_dos(X, e, E, vol):
    """g_l(E), l = 0..3, from the section geometry (corner order of X/e, not sorted)."""
    a, _ = _affine(X, e)
    area, cen = section(X, e, E)
    if area == 0.0:
        return np.zeros(4)
    lam = barycentric(X, cen)
    return vol / volume(X) * area * lam / np.linalg.norm(a)


def corner_nos(X, e, E, vol):
    """w_l(E), l = 0..3, from the clipped-volume geometry (corner order of X/e)."""
    if E >= max(e):
        return np.full(4, vol / 4.0)
    v, cen = lower_region(X, e, E)
    if v == 0.0:
        return np.zeros(4)
    lam = barycentric(X, cen)
    return vol / volume(X) * v * lam
