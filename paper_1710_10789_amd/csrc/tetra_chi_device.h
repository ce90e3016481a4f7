// Device-side building blocks of the susceptibility kernel (gfx950). Internal header; also built for
// the host by the test harness.
//
// The orbital-resolved imaginary part of the bare (Lindhard) susceptibility at zero temperature, as
// the spectral weight
//   S_m(q, w) = sum_{n,n'} (1/V_G) int W_m [theta(E_F - eps) theta(eps' - E_F) - theta(eps - E_F) theta(E_F - eps')]
//               delta(w - (eps' - eps)) d^3k,     eps = eps_n(k), eps' = eps_n'(k + q), W_m = b_mn(k) b_mn'(k + q)
// (Im chi_0 = -pi S), by the linear tetrahedron method of Guterding & Jeschke (arXiv:1710.10789,
// Sec. II) applied to the difference energy eps' - eps: energies and W linear inside each tetrahedron
// of Table I, the two step functions applied exactly by clipping the tetrahedron at eps = E_F and
// eps' = E_F. Each piece of the clipped region is a sub-tetrahedron on which eps' - eps is linear, so
// its contribution is the tetrahedron DOS of Sec. II.C (corner weights dw/dE) with eps' - eps as the
// energy and the piece's share of V_T.
//
// Sub-tetrahedra are held as the barycentric coordinates of their four vertices with respect to the
// parent tetrahedron (row i = vertex i). Clipping a tetrahedron at a plane leaves one tetrahedron (one
// vertex inside) or a triangular prism (two or three inside) whose end triangles lie on the parent's
// faces and the plane; the prism (p0 p1 p2 | q0 q1 q2, with edges p_i q_i) is split into the three
// tetrahedra (p0 p1 p2 q2), (p0 p1 q1 q2), (p0 q0 q1 q2).
#pragma once

#include "tetra_device.h"

namespace tetra {

// Rows of v (and the values f at them) reordered so that the rows with f <= 0 come first (a
// five-comparator network on the key f > 0). Returns the number of rows with f <= 0.
__host__ __device__ __forceinline__ int inside_first(float v[4][4], float f[4]) {
  auto cx = [&](int a, int b) {
    const bool sw = (f[a] > 0.0f) && !(f[b] > 0.0f);
    const float fa = f[a], fb = f[b];
    f[a] = sw ? fb : fa;
    f[b] = sw ? fa : fb;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float x = v[a][c], y = v[b][c];
      v[a][c] = sw ? y : x;
      v[b][c] = sw ? x : y;
    }
  };
  cx(0, 1);
  cx(2, 3);
  cx(0, 2);
  cx(1, 3);
  cx(1, 2);
  return (f[0] <= 0.0f) + (f[1] <= 0.0f) + (f[2] <= 0.0f) + (f[3] <= 0.0f);
}

// The corners of a tetrahedron reordered (the same network) so that those with f <= 0 come first,
// carrying two per-corner values x, y and the corner's point index q along. Relabelling the corners
// of a tetrahedron changes nothing in its contribution, so the first clipping can then start from the
// identity (unit barycentric rows) instead of a permuted one.
__host__ __device__ __forceinline__ void inside_first_corners(float f[4], float x[4], float y[4], int q[4]) {
  auto cx = [&](int a, int b) {
    const bool sw = (f[a] > 0.0f) && !(f[b] > 0.0f);
    const float fa = f[a], fb = f[b], xa = x[a], xb = x[b], ya = y[a], yb = y[b];
    const int qa = q[a], qb = q[b];
    f[a] = sw ? fb : fa;
    f[b] = sw ? fa : fb;
    x[a] = sw ? xb : xa;
    x[b] = sw ? xa : xb;
    y[a] = sw ? yb : ya;
    y[b] = sw ? ya : yb;
    q[a] = sw ? qb : qa;
    q[b] = sw ? qa : qb;
  };
  cx(0, 1);
  cx(2, 3);
  cx(0, 2);
  cx(1, 3);
  cx(1, 2);
}

// Number of tetrahedra the part {f <= 0} splits into, for ni vertices inside.
__host__ __device__ __forceinline__ int clip_pieces(int ni) { return ni == 0 ? 0 : (ni == 1 || ni == 4) ? 1 : 3; }

// The piece idx (< clip_pieces(ni)) of {f <= 0} of the tetrahedron v, whose rows are ordered inside
// first (inside_first) with f the values at them.
__host__ __device__ __forceinline__ void clip_piece(const float v[4][4], const float f[4], int ni, int idx,
                                                    float out[4][4]) {
  // point on the edge from inside vertex a to outside vertex b where f = 0
  auto cut = [&](int a, int b, float p[4]) {
    const float t = f[a] / (f[a] - f[b]);
#pragma unroll
    for (int c = 0; c < 4; ++c) p[c] = __builtin_fmaf(t, v[b][c] - v[a][c], v[a][c]);
  };
  float p1[4], p2[4], q0[4], q1[4], q2[4];
  if (ni == 4) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      p1[c] = v[1][c];
      p2[c] = v[2][c];
      q2[c] = v[3][c];
      q0[c] = q1[c] = 0.0f;
    }
  } else if (ni == 1) {  // the corner tetrahedron (a, a->b, a->c, a->d)
    cut(0, 1, p1);
    cut(0, 2, p2);
    cut(0, 3, q2);
#pragma unroll
    for (int c = 0; c < 4; ++c) q0[c] = q1[c] = 0.0f;
  } else if (ni == 2) {  // prism (a, a->c, a->d | b, b->c, b->d)
    cut(0, 2, p1);
    cut(0, 3, p2);
    cut(1, 2, q1);
    cut(1, 3, q2);
#pragma unroll
    for (int c = 0; c < 4; ++c) q0[c] = v[1][c];
  } else {  // ni == 3: prism (a, b, c | a->d, b->d, c->d)
    cut(0, 3, q0);
    cut(1, 3, q1);
    cut(2, 3, q2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      p1[c] = v[1][c];
      p2[c] = v[2][c];
    }
  }
  // piece 0: (p0 p1 p2 q2), 1: (p0 p1 q1 q2), 2: (p0 q0 q1 q2); p0 is row 0 in every case
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    out[0][c] = v[0][c];
    out[1][c] = idx < 2 ? p1[c] : q0[c];
    out[2][c] = idx == 0 ? p2[c] : q1[c];
    out[3][c] = q2[c];
  }
}

// Volume of a sub-tetrahedron as a fraction of its parent's: |det| of its edge vectors in the
// coordinates (lambda_1, lambda_2, lambda_3).
__host__ __device__ __forceinline__ float sub_volume(const float s[4][4]) {
  float a[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) a[i][c] = s[i + 1][c + 1] - s[0][c + 1];
  const float det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                    a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                    a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  return fabsf(det);
}

// Occupation half-spaces of region r of one tetrahedron (corner energies e of band n at k, ep of band
// n' at k + q): r = 0 is {eps <= E_F, eps' >= E_F} (sign +1), r = 1 is {eps >= E_F, eps' <= E_F}
// (sign -1); f1, f2 <= 0 inside.
__host__ __device__ __forceinline__ void region_planes(int r, const float e[4], const float ep[4], float ef,
                                                       float f1[4], float f2[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    f1[c] = r == 0 ? e[c] - ef : ef - e[c];
    f2[c] = r == 0 ? ef - ep[c] : ep[c] - ef;
  }
}

// Whether region r can be non-empty: some corner on the occupied (r = 0) or empty (r = 1) side of E_F
// in band n and some on the other side in band n'.
__host__ __device__ __forceinline__ bool region_possible(int r, float emin, float emax, float epmin, float epmax,
                                                         float ef) {
  return r == 0 ? (emin <= ef && epmax >= ef) : (emax >= ef && epmin <= ef);
}

// Vertices of a sub-tetrahedron (rows of s, barycentric in the parent) sorted with their values d into
// ascending d, by the five-comparator network of sort4 (equal values may end in either order; the
// contribution does not depend on it).
__host__ __device__ __forceinline__ void sort4_rows(float d[4], float s[4][4]) {
  auto cx = [&](int a, int b) {
    const bool sw = d[b] < d[a];
    const float lo = sw ? d[b] : d[a], hi = sw ? d[a] : d[b];
    d[a] = lo;
    d[b] = hi;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float x = s[a][c], y = s[b][c];
      s[a][c] = sw ? y : x;
      s[b][c] = sw ? x : y;
    }
  };
  cx(0, 1);
  cx(2, 3);
  cx(0, 2);
  cx(1, 3);
  cx(1, 2);
}

}  // namespace tetra
