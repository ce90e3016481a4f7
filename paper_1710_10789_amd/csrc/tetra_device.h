// Device-side building blocks of the tetrahedron DOS kernels (gfx950). Internal header.
//
// The corner weights implement the five energy cases of Sec. II.C of Guterding & Jeschke
// (arXiv:1710.10789). The kernels use algebraically simplified forms of the printed formulas:
//
//   first case (E1 < E <= E2), x = E - E1, K = V / (E21 E31 E41), S = 1/E21 + 1/E31 + 1/E41:
//       g1 = 4 K x^2 (3 - x S),   g_l = 4 K x^3 / E_l1  (l = 2, 3, 4)
//   third case (E3 < E < E4), y = E4 - E, K' = V / (E41 E42 E43), S' = 1/E41 + 1/E42 + 1/E43:
//       g_l = 4 K' y^3 / E_4l  (l = 1, 2, 3),   g4 = 4 K' y^2 (3 - y S')
//   middle case (E2 < E <= E3), z = E - E2: the printed C1, C2, C3 and their derivatives, with the
//       last term of dw3/dE taken as (C2 + C3)/E32 (the energy derivative of the printed w3),
//       expanded as cubics in z (coefficients at corner_dos_B_coeffs).
//
// with V = V_T / (4 V_G). Energies are handled in local frames: x = E_j - E1 (z = E_j - E2 in the
// middle case, y = E4 - E_j in the third) is formed per (tetrahedron, band, j) from e0 - E1 (e0 - E2,
// e0 - E4) split into a head and an exact tail, so that the absolute magnitude of the energies does
// not cost resolution.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tetra {

// Table I: the six tetrahedra of an elemental cube by corner label L = 1 + o1 + 2*o2 + 4*o3, with
// (o1, o2, o3) the corner's offsets along grid axes (1, 2, 3):
//   {1,2,3,6} {2,3,4,6} {1,3,5,6} {3,4,6,8} {3,5,6,7} {3,6,7,8}
// Returned as corner slots s = L - 1 in 4-bit fields (slot of the l-th corner at bits 4l..4l+2).
// t is uniform across a wavefront, so the switch is a scalar branch.
__host__ __device__ __forceinline__ uint32_t tet_slots(int t) {
  switch (t) {
    case 0: return 0x5210u;
    case 1: return 0x5321u;
    case 2: return 0x5420u;
    case 3: return 0x7532u;
    case 4: return 0x6542u;
    default: return 0x7652u;
  }
}

__host__ __device__ __forceinline__ bool finite4(float a, float b, float c, float d) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c) && __builtin_isfinite(d);
}

// Compare-exchange carrying an integer tag (here the corner's LDS point index) with the energy;
// returns whether the pair was swapped.
__host__ __device__ __forceinline__ bool cswap(float& ea, int& pa, float& eb, int& pb) {
  const bool sw = eb < ea;
  const float lo = sw ? eb : ea;
  const float hi = sw ? ea : eb;
  const int plo = sw ? pb : pa;
  const int phi = sw ? pa : pb;
  ea = lo;
  eb = hi;
  pa = plo;
  pb = phi;
  return sw;
}

// Five-comparator network: ascending energies e[0..3] with their tags. Equal energies may end in
// either order; the weights of corners with equal energies are equal, so the result does not depend
// on it. sw[] records the exchanges, so that unsort_rows can map per-corner results back.
__host__ __device__ __forceinline__ void sort4(float e[4], int p[4], bool sw[5]) {
  sw[0] = cswap(e[0], p[0], e[1], p[1]);
  sw[1] = cswap(e[2], p[2], e[3], p[3]);
  sw[2] = cswap(e[0], p[0], e[2], p[2]);
  sw[3] = cswap(e[1], p[1], e[3], p[3]);
  sw[4] = cswap(e[1], p[1], e[2], p[2]);
}

__host__ __device__ __forceinline__ void sort4(float e[4], int p[4]) {
  bool sw[5];
  sort4(e, p, sw);
}

// Inverse of the permutation sort4 applied: rows r[0..3] (K values each, in sorted-corner order) are
// put back into the order of the corners before the sort, by the recorded exchanges in reverse.
template <int K>
__host__ __device__ __forceinline__ void unsort_rows(const bool sw[5], float (&r)[4][K]) {
  constexpr int A[5] = {0, 2, 0, 1, 1}, B[5] = {1, 3, 2, 3, 2};
#pragma unroll
  for (int k = 4; k >= 0; --k) {
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const float a = r[A[k]][v], b = r[B[k]][v];
      r[A[k]][v] = sw[k] ? b : a;
      r[B[k]][v] = sw[k] ? a : b;
    }
  }
}

// 1/x by the hardware reciprocal (within 1 ulp; +inf for +0) on the device, a division on the host.
__host__ __device__ __forceinline__ float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// a + b = hi + lo exactly (Knuth's two-sum).
__host__ __device__ __forceinline__ void two_sum(float a, float b, float& hi, float& lo) {
  hi = a + b;
  const float bb = hi - a;
  lo = (a - (hi - bb)) + (b - bb);
}

// Per (tetrahedron, band) constants of the corner-weight evaluation.
struct TetSetup {
  float d_hi, d_lo;            // e0 - E1 = d_hi + d_lo exactly
  float f_hi, f_lo;            // e0 - E4 = f_hi + f_lo exactly
  float h_hi, h_lo;            // e0 - E2 = h_hi + h_lo exactly
  float e21, e31, e41;         // E2 - E1, E3 - E1, E4 - E1
  float e32, e42;              // E3 - E2, E4 - E2 (each rounded once, exact when the two are close)
  float kA, sA;                // first case: K, S
  float kC, sC;                // third case: K', S'
  float r21, r31, r41, r32, r42, r43;
  float k1, k2, k3;            // middle case: V/(E31 E41), V/(E31 E32 E41), V/(E32 E41 E42)
};

__host__ __device__ __forceinline__ TetSetup tet_setup(const float e[4], float e0, float V) {
  TetSetup c;
  two_sum(e0, -e[0], c.d_hi, c.d_lo);
  two_sum(e0, -e[3], c.f_hi, c.f_lo);
  two_sum(e0, -e[1], c.h_hi, c.h_lo);
  c.e21 = e[1] - e[0];
  c.e31 = e[2] - e[0];
  c.e41 = e[3] - e[0];
  c.e32 = e[2] - e[1];
  c.e42 = e[3] - e[1];
  const float e32 = c.e32, e42 = c.e42, e43 = e[3] - e[2];
  // Reciprocals of zero differences are infinite; the case that would use them is never selected.
  c.r21 = rcp(c.e21);
  c.r31 = rcp(c.e31);
  c.r41 = rcp(c.e41);
  c.r32 = rcp(e32);
  c.r42 = rcp(e42);
  c.r43 = rcp(e43);
  c.kA = V * c.r21 * c.r31 * c.r41;
  c.sA = c.r21 + c.r31 + c.r41;
  c.kC = V * c.r41 * c.r42 * c.r43;
  c.sC = c.r41 + c.r42 + c.r43;
  c.k1 = V * c.r31 * c.r41;
  c.k2 = c.k1 * c.r32;
  c.k3 = V * c.r32 * c.r41 * c.r42;
  return c;
}

// x = E_j - E1 for E_j = e0 + j*de.
__host__ __device__ __forceinline__ float local_x(const TetSetup& c, int j, float de) {
  return __builtin_fmaf((float)j, de, c.d_hi) + c.d_lo;
}

// z = E_j - E2 (the middle case's variable).
__host__ __device__ __forceinline__ float local_z(const TetSetup& c, int j, float de) {
  return __builtin_fmaf((float)j, de, c.h_hi) + c.h_lo;
}

// y = E4 - E_j, accurate near E4 (the third case's variable).
__host__ __device__ __forceinline__ float local_y(const TetSetup& c, int j, float de) {
  return -(__builtin_fmaf((float)j, de, c.f_hi) + c.f_lo);
}

// dw_l/dE in sorted-corner order, one function per energy case: A at x = E - E1 with 0 < x <= E21
// (E1 < E <= E2), B at z = E - E2 with 0 < z <= E32 (E2 < E <= E3), C at y = E4 - E with 0 < y < E43
// (E3 < E < E4).
__host__ __device__ __forceinline__ void corner_dos_A(const TetSetup& c, float x, float g[4]) {
  const float t = 4.0f * c.kA * x * x;
  const float u = t * x;
  g[0] = t * (3.0f - x * c.sA);
  g[1] = u * c.r21;
  g[2] = u * c.r31;
  g[3] = u * c.r41;
}

// Middle case. On (E2, E3] every corner weight is a cubic in z = E - E2, g_l(z) = sum_k c_lk z^k, with
// coefficients in a = E21, b = E32, c = E42 and k1 = V/(E31 E41) (the expansion of the printed formulas):
//   g1: 4 a k1 (ab + ac + 2bc) / (E31 E41),  -12 k1 (a^2 - bc) / (E31 E41),  -12 k1 (2a + b + c) / (E31 E41),
//       4 k1 (a^2 + 2ab + 2ac + b^2 + bc + c^2) / (b c E31 E41)
//   g2: 4 a k1,  12 k1,  -12 k1 (a + b + c) / (b c),  4 k1 (ab + ac + b^2 + bc + c^2) / (b^2 c^2)
//   g3: 4 a^2 k1 / E31,  12 a k1 / E31,  12 k1 / E31,  -4 k1 (a^2 + 2ab + ac + b^2 + 2bc) / (b^2 c E31)
//   g4: 4 a^2 k1 / E41,  12 a k1 / E41,  12 k1 / E41,  -4 k1 (a^2 + ab + 2ac + 2bc + c^2) / (b c^2 E41)
// coef[l][k] is the z^k coefficient of g_{l+1}.
__host__ __device__ __forceinline__ void corner_dos_B_coeffs(const TetSetup& c, float V, float coef[4][4]) {
  const float a = c.e21, b = c.e32, cc = c.e42;
  const float rb = c.r32, rc = c.r42, rbc = rb * rc;
  const float k1 = V * c.r31 * c.r41, k31 = k1 * c.r31, k41 = k1 * c.r41, k3141 = k31 * c.r41;
  const float ab = a * b, ac = a * cc, bc = b * cc, aa = a * a, bb = b * b, c2 = cc * cc;
  coef[0][0] = 4.0f * a * (ab + ac + 2.0f * bc) * k3141;
  coef[0][1] = -12.0f * (aa - bc) * k3141;
  coef[0][2] = -12.0f * (2.0f * a + b + cc) * k3141;
  coef[0][3] = 4.0f * (aa + 2.0f * ab + 2.0f * ac + bb + bc + c2) * rbc * k3141;
  coef[1][0] = 4.0f * a * k1;
  coef[1][1] = 12.0f * k1;
  coef[1][2] = -12.0f * (a + b + cc) * rbc * k1;
  coef[1][3] = 4.0f * (ab + ac + bb + bc + c2) * rbc * rbc * k1;
  coef[2][0] = 4.0f * aa * k31;
  coef[2][1] = 12.0f * a * k31;
  coef[2][2] = 12.0f * k31;
  coef[2][3] = -4.0f * (aa + 2.0f * ab + ac + bb + 2.0f * bc) * rb * rbc * k31;
  coef[3][0] = 4.0f * aa * k41;
  coef[3][1] = 12.0f * a * k41;
  coef[3][2] = 12.0f * k41;
  coef[3][3] = -4.0f * (aa + ab + 2.0f * ac + 2.0f * bc + c2) * rc * rbc * k41;
}

__host__ __device__ __forceinline__ void corner_dos_B_poly(const float coef[4][4], float z, float g[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l)
    g[l] = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(coef[l][3], z, coef[l][2]), z, coef[l][1]), z, coef[l][0]);
}

__host__ __device__ __forceinline__ void corner_dos_C(const TetSetup& c, float y, float g[4]) {
  const float t = 4.0f * c.kC * y * y;
  const float u = t * y;
  g[0] = u * c.r41;
  g[1] = u * c.r42;
  g[2] = u * c.r43;
  g[3] = t * (3.0f - y * c.sC);
}

// Adjoint of the corner weights by moments. For multipliers s_l (one per sorted corner), summed over the
// energies of one case range, F = sum_j sum_l s_l g_l(E_j) is a combination of the moments
// sum_j s_l t_j^k of the range's local variable t (x = E - E1 in the first case, z = E - E2 in the
// middle one, y = E4 - E in the third), because every corner weight is a cubic in t on its range.
// The *_finish functions take the derivative of F with respect to the four sorted corner energies at
// fixed E_j from the moments, in reverse through the per-tetrahedron constants.

// First case: g1 = 4K x^2 (3 - x S), g_l = 4K x^3 r_l1 (l = 2, 3, 4), K = V r21 r31 r41, S = r21 + r31 + r41.
// Moments m[9] (sums over the range): s1 x, s1 x^2, s1 x^3, s_l x^2 (l = 2, 3, 4), s_l x^3 (l = 2, 3, 4).
__host__ __device__ __forceinline__ void corner_dos_moments_finish_A(const TetSetup& c, float V, const float m[9], float Eb[4]) {
  // F = 4K T, T = 3 sum s1 x^2 - S sum s1 x^3 + sum_l r_l1 sum s_l x^3
  const float T = 3.0f * m[1] - c.sA * m[2] + c.r21 * m[6] + c.r31 * m[7] + c.r41 * m[8];
  const float K4 = 4.0f * c.kA, V4T = 4.0f * V * T;
  const float F21 = V4T * c.r31 * c.r41 + K4 * (m[6] - m[2]);
  const float F31 = V4T * c.r21 * c.r41 + K4 * (m[7] - m[2]);
  const float F41 = V4T * c.r21 * c.r31 + K4 * (m[8] - m[2]);
  // dF/dx summed over the range (x = E - E1 moves with E1)
  const float Fx = K4 * (6.0f * m[0] - 3.0f * c.sA * m[1] + 3.0f * (c.r21 * m[3] + c.r31 * m[4] + c.r41 * m[5]));
  const float e21b = -F21 * c.r21 * c.r21, e31b = -F31 * c.r31 * c.r31, e41b = -F41 * c.r41 * c.r41;
  Eb[0] = -(e21b + e31b + e41b) - Fx;
  Eb[1] = e21b;
  Eb[2] = e31b;
  Eb[3] = e41b;
}

// Third case (mirror of the first, y = E4 - E): g_l = 4K' y^3 r_4l (l = 1, 2, 3), g4 = 4K' y^2 (3 - y S'),
// K' = V r41 r42 r43, S' = r41 + r42 + r43. Moments m[9]: s4 y, s4 y^2, s4 y^3, s_l y^2 (l = 1, 2, 3),
// s_l y^3 (l = 1, 2, 3).
__host__ __device__ __forceinline__ void corner_dos_moments_finish_C(const TetSetup& c, float V, const float m[9], float Eb[4]) {
  const float T = 3.0f * m[1] - c.sC * m[2] + c.r41 * m[6] + c.r42 * m[7] + c.r43 * m[8];
  const float K4 = 4.0f * c.kC, V4T = 4.0f * V * T;
  const float F41 = V4T * c.r42 * c.r43 + K4 * (m[6] - m[2]);
  const float F42 = V4T * c.r41 * c.r43 + K4 * (m[7] - m[2]);
  const float F43 = V4T * c.r41 * c.r42 + K4 * (m[8] - m[2]);
  // dF/dy summed over the range (y = E4 - E moves with E4)
  const float Fy = K4 * (6.0f * m[0] - 3.0f * c.sC * m[1] + 3.0f * (c.r41 * m[3] + c.r42 * m[4] + c.r43 * m[5]));
  const float e41b = -F41 * c.r41 * c.r41, e42b = -F42 * c.r42 * c.r42, e43b = -F43 * c.r43 * c.r43;
  Eb[0] = -e41b;
  Eb[1] = -e42b;
  Eb[2] = -e43b;
  Eb[3] = e41b + e42b + e43b + Fy;
}

// Middle case: the 16 moments M_lk = sum_j s_l z_j^k (k = 0..3) give F = sum_lk c_lk M_lk.
__host__ __device__ __forceinline__ void corner_dos_moments_finish_B(const TetSetup& c, float V, const float M[4][4],
                                                                     float Eb[4]) {
  const float a = c.e21, b = c.e32, cc = c.e42;
  const float r31 = c.r31, r41 = c.r41, rb = c.r32, rc = c.r42;
  const float k1 = V * r31 * r41;
  const float ab = a * b, ac = a * cc, bc = b * cc, aa = a * a, bb = b * b, ccc = cc * cc;
  const float P1 = aa + 2.0f * ab + 2.0f * ac + bb + bc + ccc;
  const float P2 = ab + ac + bb + bc + ccc;
  const float P3 = aa + 2.0f * ab + ac + bb + 2.0f * bc;
  const float P4 = aa + ab + 2.0f * ac + 2.0f * bc + ccc;
  const float Q0 = ab + ac + 2.0f * bc;
  const float rbc = rb * rc;
  const float S = a + b + cc;
  // coefficients / k1, for the derivative through z (z = E - E2 moves with E2)
  const float u0 = 4.0f * a * Q0, u1 = -12.0f * (aa - bc), u2 = -12.0f * (2.0f * a + b + cc);
  const float w13 = 4.0f * P1 * rbc;
  const float w22 = -12.0f * S * rbc, w23 = 4.0f * P2 * rbc * rbc;
  const float w33 = -4.0f * P3 * rb * rbc, w43 = -4.0f * P4 * rc * rbc;
  // F / k1 = T = T1 + T2 + T3 + T4
  const float X1 = u0 * M[0][0] + u1 * M[0][1] + u2 * M[0][2] + w13 * M[0][3];
  const float T2 = 4.0f * a * M[1][0] + 12.0f * M[1][1] + w22 * M[1][2] + w23 * M[1][3];
  const float W3 = 4.0f * aa * M[2][0] + 12.0f * a * M[2][1] + 12.0f * M[2][2];
  const float X3 = W3 + w33 * M[2][3];
  const float W4 = 4.0f * aa * M[3][0] + 12.0f * a * M[3][1] + 12.0f * M[3][2];
  const float X4 = W4 + w43 * M[3][3];
  const float T = r31 * r41 * X1 + T2 + r31 * X3 + r41 * X4;
  // dF/dz summed over the range: sum_{l, k >= 1} k c_lk M_l,k-1
  const float dz1 = r31 * r41 * (u1 * M[0][0] + 2.0f * u2 * M[0][1] + 3.0f * w13 * M[0][2]);
  const float dz2 = 12.0f * M[1][0] + 2.0f * w22 * M[1][1] + 3.0f * w23 * M[1][2];
  const float dz3 = r31 * (12.0f * a * M[2][0] + 24.0f * M[2][1] + 3.0f * w33 * M[2][2]);
  const float dz4 = r41 * (12.0f * a * M[3][0] + 24.0f * M[3][1] + 3.0f * w43 * M[3][2]);
  const float Fz = k1 * (dz1 + dz2 + dz3 + dz4);
  // reverse sweep of F = k1 T with respect to a, b, c and the reciprocals
  const float Tb = k1;
  float r31b = V * r41 * T, r41b = V * r31 * T, rbb = 0.0f, rcb = 0.0f;
  float ab_ = 0.0f, bb_ = 0.0f, cb_ = 0.0f;
  // T1 = r31 r41 X1
  r31b += r41 * X1 * Tb;
  r41b += r31 * X1 * Tb;
  const float X1b = r31 * r41 * Tb;
  ab_ += X1b * (M[0][0] * (4.0f * Q0 + 4.0f * a * (b + cc)) - 24.0f * a * M[0][1] - 24.0f * M[0][2]);
  bb_ += X1b * (4.0f * a * (a + 2.0f * cc) * M[0][0] + 12.0f * cc * M[0][1] - 12.0f * M[0][2]);
  cb_ += X1b * (4.0f * a * (a + 2.0f * b) * M[0][0] + 12.0f * b * M[0][1] - 12.0f * M[0][2]);
  const float P1b = 4.0f * rbc * M[0][3] * X1b;
  rbb += 4.0f * P1 * rc * M[0][3] * X1b;
  rcb += 4.0f * P1 * rb * M[0][3] * X1b;
  // T2
  ab_ += Tb * (4.0f * M[1][0] - 12.0f * rbc * M[1][2]);
  bb_ += Tb * (-12.0f * rbc * M[1][2]);
  cb_ += Tb * (-12.0f * rbc * M[1][2]);
  rbb += Tb * (-12.0f * S * rc * M[1][2] + 8.0f * P2 * rb * rc * rc * M[1][3]);
  rcb += Tb * (-12.0f * S * rb * M[1][2] + 8.0f * P2 * rb * rb * rc * M[1][3]);
  const float P2b = 4.0f * rbc * rbc * M[1][3] * Tb;
  // T3 = r31 X3
  r31b += X3 * Tb;
  const float X3b = r31 * Tb;
  ab_ += X3b * (8.0f * a * M[2][0] + 12.0f * M[2][1]);
  const float P3b = -4.0f * rb * rbc * M[2][3] * X3b;
  rbb += -8.0f * P3 * rbc * M[2][3] * X3b;
  rcb += -4.0f * P3 * rb * rb * M[2][3] * X3b;
  // T4 = r41 X4
  r41b += X4 * Tb;
  const float X4b = r41 * Tb;
  ab_ += X4b * (8.0f * a * M[3][0] + 12.0f * M[3][1]);
  const float P4b = -4.0f * rc * rbc * M[3][3] * X4b;
  rbb += -4.0f * P4 * rc * rc * M[3][3] * X4b;
  rcb += -8.0f * P4 * rbc * M[3][3] * X4b;
  // the polynomials P1..P4
  ab_ += P1b * (2.0f * S) + P2b * (b + cc) + P3b * (2.0f * a + 2.0f * b + cc) + P4b * (2.0f * a + b + 2.0f * cc);
  bb_ += P1b * (2.0f * a + 2.0f * b + cc) + P2b * (a + 2.0f * b + cc) + P3b * (2.0f * S) + P4b * (a + 2.0f * cc);
  cb_ += P1b * (2.0f * a + b + 2.0f * cc) + P2b * (a + b + 2.0f * cc) + P3b * (a + 2.0f * b) + P4b * (2.0f * S);
  // reciprocals: r31 = 1/(a + b), r41 = 1/(a + c), rb = 1/b, rc = 1/c
  const float d31 = -r31b * r31 * r31, d41 = -r41b * r41 * r41;
  ab_ += d31 + d41;
  bb_ += d31 - rbb * rb * rb;
  cb_ += d41 - rcb * rc * rc;
  // a = E2 - E1, b = E3 - E2, c = E4 - E2, z = E - E2
  Eb[0] = -ab_;
  Eb[1] = ab_ - bb_ - cb_ - Fz;
  Eb[2] = bb_;
  Eb[3] = cb_;
}

// Range ends of the adjoint. Over the energies of one case range with local variable t, the loop
// accumulates only the power sums H_k[m] = sum_j G[j][m] t_j^k of the loss gradient G. Then, with
// b[l] the orbital weights of sorted corner l and g_l(t) = sum_k c_lk t^k,
//   dL/db_l[m] += sum_k c_lk H_k[m]                      (the weight gradient)
//   moments    sum_j s_l(t_j) t_j^k = sum_m b_l[m] H_k[m] (s_l = sum_m G b_l, for the energy gradient)
// and Eb gets the range's derivative with respect to the four sorted corner energies.
template <int NORB>
__host__ __device__ __forceinline__ float dot_row(const float* b, const float h[NORB]) {
  float acc = 0.0f;
#pragma unroll
  for (int m = 0; m < NORB; ++m) acc = __builtin_fmaf(b[m], h[m], acc);
  return acc;
}

// First case, t = x = E - E1, H[0..2] = powers 1..3.
template <int NORB>
__host__ __device__ __forceinline__ void adjoint_range_A(const TetSetup& c, float V, const float* const b[4],
                                                         const float H[3][NORB], float gb[4][NORB], float Eb[4]) {
  const float mo[9] = {dot_row<NORB>(b[0], H[0]), dot_row<NORB>(b[0], H[1]), dot_row<NORB>(b[0], H[2]),
                       dot_row<NORB>(b[1], H[1]), dot_row<NORB>(b[2], H[1]), dot_row<NORB>(b[3], H[1]),
                       dot_row<NORB>(b[1], H[2]), dot_row<NORB>(b[2], H[2]), dot_row<NORB>(b[3], H[2])};
  corner_dos_moments_finish_A(c, V, mo, Eb);
  // g1 = 12 K x^2 - 4 K S x^3, g_l = 4 K r_l1 x^3
  const float c12 = 12.0f * c.kA, c13 = -4.0f * c.kA * c.sA, k4 = 4.0f * c.kA;
  const float c3[3] = {k4 * c.r21, k4 * c.r31, k4 * c.r41};
#pragma unroll
  for (int m = 0; m < NORB; ++m) {
    gb[0][m] = __builtin_fmaf(c12, H[1][m], __builtin_fmaf(c13, H[2][m], gb[0][m]));
#pragma unroll
    for (int l = 1; l < 4; ++l) gb[l][m] = __builtin_fmaf(c3[l - 1], H[2][m], gb[l][m]);
  }
}

// Middle case, t = z = E - E2, H[0..3] = powers 0..3.
template <int NORB>
__host__ __device__ __forceinline__ void adjoint_range_B(const TetSetup& c, float V, const float* const b[4],
                                                         const float H[4][NORB], float gb[4][NORB], float Eb[4]) {
  float M[4][4];
#pragma unroll
  for (int l = 0; l < 4; ++l)
#pragma unroll
    for (int k = 0; k < 4; ++k) M[l][k] = dot_row<NORB>(b[l], H[k]);
  corner_dos_moments_finish_B(c, V, M, Eb);
  float coef[4][4];
  corner_dos_B_coeffs(c, V, coef);
#pragma unroll
  for (int l = 0; l < 4; ++l)
#pragma unroll
    for (int m = 0; m < NORB; ++m)
      gb[l][m] += __builtin_fmaf(coef[l][3], H[3][m],
                                 __builtin_fmaf(coef[l][2], H[2][m], __builtin_fmaf(coef[l][1], H[1][m], coef[l][0] * H[0][m])));
}

// Third case, t = y = E4 - E, H[0..2] = powers 1..3.
template <int NORB>
__host__ __device__ __forceinline__ void adjoint_range_C(const TetSetup& c, float V, const float* const b[4],
                                                         const float H[3][NORB], float gb[4][NORB], float Eb[4]) {
  const float mo[9] = {dot_row<NORB>(b[3], H[0]), dot_row<NORB>(b[3], H[1]), dot_row<NORB>(b[3], H[2]),
                       dot_row<NORB>(b[0], H[1]), dot_row<NORB>(b[1], H[1]), dot_row<NORB>(b[2], H[1]),
                       dot_row<NORB>(b[0], H[2]), dot_row<NORB>(b[1], H[2]), dot_row<NORB>(b[2], H[2])};
  corner_dos_moments_finish_C(c, V, mo, Eb);
  // g_l = 4 K' r_4l y^3 (l = 1, 2, 3), g4 = 12 K' y^2 - 4 K' S' y^3
  const float c42 = 12.0f * c.kC, c43 = -4.0f * c.kC * c.sC, k4 = 4.0f * c.kC;
  const float c3[3] = {k4 * c.r41, k4 * c.r42, k4 * c.r43};
#pragma unroll
  for (int m = 0; m < NORB; ++m) {
    gb[3][m] = __builtin_fmaf(c42, H[1][m], __builtin_fmaf(c43, H[2][m], gb[3][m]));
#pragma unroll
    for (int l = 0; l < 3; ++l) gb[l][m] = __builtin_fmaf(c3[l], H[2][m], gb[l][m]);
  }
}

// Estimate of the window of grid indices j with E1 < E_j < E4, clipped to [lo, hi] (empty when
// jlo > jhi). Computed in FP32 from absolute energies, so either end can be off by one index; use
// tet_window to make it exact for one tetrahedron-band.
__host__ __device__ __forceinline__ void energy_window(float e1, float e4, float e0, float inv_de, int lo, int hi,
                                                       int& jlo, int& jhi) {
  const float big = 3.0e7f;  // beyond any supported grid length
  float t1 = (e1 - e0) * inv_de;
  float t4 = (e4 - e0) * inv_de;
  t1 = fminf(fmaxf(t1, -2.0f), big);
  t4 = fminf(fmaxf(t4, -2.0f), big);
  const int a = (int)floorf(t1) + 1, b = (int)ceilf(t4) - 1;
  jlo = a > lo ? a : lo;
  jhi = b < hi ? b : hi;
}

// Exact window {j in [lo, hi] : 0 < x_j < E41} of one tetrahedron-band, from the estimate (off by at
// most one index at either end for ne <= 2^22) and the accurate local-frame x, which is
// non-decreasing in j. A boundary index matters for the gradient: the derivative of the corner
// weights with respect to E1 (or E4) vanishes only linearly in x (or E4 - E_j), with a prefactor
// 1/(E21 E31 E41) that is large for narrow tetrahedra.
__host__ __device__ __forceinline__ void tet_window(const TetSetup& c, float de, int lo, int hi, int& jlo, int& jhi) {
  if (jlo <= hi && !(local_x(c, jlo, de) > 0.0f)) ++jlo;
  else if (jlo > lo && local_x(c, jlo - 1, de) > 0.0f) --jlo;
  if (jhi >= lo && !(local_x(c, jhi, de) < c.e41)) --jhi;
  else if (jhi < hi && local_x(c, jhi + 1, de) < c.e41) ++jhi;
}

// Last j in [jlo, jhi] with x_j <= thr (jlo - 1 if none), for x_j non-decreasing in j.
__host__ __device__ __forceinline__ int last_at_or_below(const TetSetup& c, float de, float inv_de, int jlo, int jhi,
                                                         float thr) {
  const float x0 = local_x(c, jlo, de);
  float t = (thr - x0) * inv_de;
  t = fminf(fmaxf(t, -1.0f), (float)(jhi - jlo));
  int j = jlo + (int)floorf(t);
  if (j >= jlo && local_x(c, j, de) > thr) --j;
  else if (j < jhi && local_x(c, j + 1, de) <= thr) ++j;
  return j;
}

// Case boundaries inside the window: [jlo, jA] first case, (jA, jB] middle case, (jB, jhi] third case.
__host__ __device__ __forceinline__ void case_split(const TetSetup& c, float de, float inv_de, int jlo, int jhi,
                                                    int& jA, int& jB) {
  jA = last_at_or_below(c, de, inv_de, jlo, jhi, c.e21);
  jB = last_at_or_below(c, de, inv_de, jlo, jhi, c.e31);
  if (jB < jA) jB = jA;
}

// Estimate of the energy range of a set of grid points, one index wider on each side than
// energy_window so that it contains every exact tetrahedron window of the set.
__host__ __device__ __forceinline__ void range_window(float emin, float emax, float e0, float inv_de, int ne, int& J0,
                                                      int& J1) {
  energy_window(emin, emax, e0, inv_de, 0, ne - 1, J0, J1);
  J0 = J0 > 0 ? J0 - 1 : 0;
  J1 = J1 < ne - 1 ? J1 + 1 : ne - 1;
}

}  // namespace tetra
