// Device-side building blocks of the number-of-states kernel (gfx950). Internal header.
//
// Integrated corner weights w_l of the five energy cases of Sec. II.C of Guterding & Jeschke
// (arXiv:1710.10789), in the notation of tetra_device.h, and the grid indices at which a
// tetrahedron-band's number of states changes.
#pragma once

#include "tetra_device.h"

namespace tetra {

// Integrated corner weights w_l (Sec. II.C), for the number of states, in the local variables of
// tetra_device.h:
//   first case   w1 = K x^3 (4 - x S),  w_l = K x^4 r_l1 (l = 2, 3, 4)
//   third case   w_l = V - K' y^4 r_4l (l = 1, 2, 3),  w4 = V - K' y^3 (4 - y S')
//   middle case  w_l(z) = w_l(E2) + sum_k c_lk z^(k+1) / (k+1): the integral from E2 of the cubic
//                dw_l/dE (the expansion written out at corner_dos_B_coeffs), with w_l(E2) the first
//                case's value at x = E21.
// Two precisions. The kernel adds increments w_l(E_j) - w_l(E_{j-1}); with bins much narrower than
// the tetrahedron they are small differences of values up to V = V_T/(4 V_G), and FP32 evaluation
// leaves them a relative error of about 1e-7 E41/de, FP64 about 1e-16 E41/de. The FP32 forms take
// the float TetSetup, the FP64 ones a NosSetup.

__host__ __device__ __forceinline__ void corner_nos_A(const TetSetup& c, float x, float w[4]) {
  const float t = c.kA * x * x * x;
  const float u = t * x;
  w[0] = t * (4.0f - x * c.sA);
  w[1] = u * c.r21;
  w[2] = u * c.r31;
  w[3] = u * c.r41;
}

// coef[l][k] is the z^k coefficient of w_{l+1} on the middle case (k = 0..4).
__host__ __device__ __forceinline__ void corner_nos_B_coeffs(const TetSetup& c, float V, float coef[4][5]) {
  float g[4][4];
  corner_dos_B_coeffs(c, V, g);
  // first-case values at x = a = E21, written with a * r21 = 1 so that a = 0 gives zeros
  const float a = c.e21, ka2 = V * c.r31 * c.r41 * a * a;
  coef[0][0] = ka2 * (3.0f - a * c.r31 - a * c.r41);
  coef[1][0] = ka2;
  coef[2][0] = ka2 * a * c.r31;
  coef[3][0] = ka2 * a * c.r41;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    coef[l][1] = g[l][0];
    coef[l][2] = 0.5f * g[l][1];
    coef[l][3] = (1.0f / 3.0f) * g[l][2];
    coef[l][4] = 0.25f * g[l][3];
  }
}

__host__ __device__ __forceinline__ void corner_nos_B_poly(const float coef[4][5], float z, float w[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l)
    w[l] = __builtin_fmaf(
        __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(coef[l][4], z, coef[l][3]), z, coef[l][2]), z, coef[l][1]), z,
        coef[l][0]);
}

__host__ __device__ __forceinline__ void corner_nos_C(const TetSetup& c, float V, float y, float w[4]) {
  const float t = c.kC * y * y * y;
  const float u = t * y;
  w[0] = V - u * c.r41;
  w[1] = V - u * c.r42;
  w[2] = V - u * c.r43;
  w[3] = V - t * (4.0f - y * c.sC);
}

// FP64 constants of one tetrahedron-band.
struct NosSetup {
  double x0, z0, y0;  // grid index 0 in the local frames: E_0 - E1, E_0 - E2, E4 - E_0
  double e21, e31, e41, e32, e42;
  double r21, r31, r41, r32, r42, r43;
  double kA, sA, kC, sC;
};

// e sorted ascending; grid E_j = e0 + (j + joff) de. Differences of FP32 values are exact in FP64.
__host__ __device__ __forceinline__ NosSetup nos_setup(const float e[4], float e0, float joff, float de, double V) {
  NosSetup c;
  const double E0 = (double)e0 + (double)joff * (double)de;
  c.x0 = E0 - (double)e[0];
  c.z0 = E0 - (double)e[1];
  c.y0 = (double)e[3] - E0;
  c.e21 = (double)e[1] - (double)e[0];
  c.e31 = (double)e[2] - (double)e[0];
  c.e41 = (double)e[3] - (double)e[0];
  c.e32 = (double)e[2] - (double)e[1];
  c.e42 = (double)e[3] - (double)e[1];
  // Reciprocals of zero differences are infinite; the case that would use them is never selected.
  c.r21 = 1.0 / c.e21;
  c.r31 = 1.0 / c.e31;
  c.r41 = 1.0 / c.e41;
  c.r32 = 1.0 / c.e32;
  c.r42 = 1.0 / c.e42;
  c.r43 = 1.0 / ((double)e[3] - (double)e[2]);
  c.kA = V * c.r21 * c.r31 * c.r41;
  c.sA = c.r21 + c.r31 + c.r41;
  c.kC = V * c.r41 * c.r42 * c.r43;
  c.sC = c.r41 + c.r42 + c.r43;
  return c;
}

__host__ __device__ __forceinline__ void corner_nos_A(const NosSetup& c, double x, double w[4]) {
  const double t = c.kA * x * x * x;
  const double u = t * x;
  w[0] = t * (4.0 - x * c.sA);
  w[1] = u * c.r21;
  w[2] = u * c.r31;
  w[3] = u * c.r41;
}

// coef[l][k] is the z^k coefficient of w_{l+1} on the middle case (k = 0..4).
__host__ __device__ __forceinline__ void corner_nos_B_coeffs(const NosSetup& c, double V, double coef[4][5]) {
  const double a = c.e21, b = c.e32, cc = c.e42;
  const double rb = c.r32, rc = c.r42, rbc = rb * rc;
  const double k1 = V * c.r31 * c.r41, k31 = k1 * c.r31, k41 = k1 * c.r41, k3141 = k31 * c.r41;
  const double ab = a * b, ac = a * cc, bc = b * cc, aa = a * a, bb = b * b, c2 = cc * cc;
  // the cubic dw_l/dE = sum_k g_lk z^k (same expansion as corner_dos_B_coeffs)
  const double g[4][4] = {
      {4.0 * a * (ab + ac + 2.0 * bc) * k3141, -12.0 * (aa - bc) * k3141, -12.0 * (2.0 * a + b + cc) * k3141,
       4.0 * (aa + 2.0 * ab + 2.0 * ac + bb + bc + c2) * rbc * k3141},
      {4.0 * a * k1, 12.0 * k1, -12.0 * (a + b + cc) * rbc * k1, 4.0 * (ab + ac + bb + bc + c2) * rbc * rbc * k1},
      {4.0 * aa * k31, 12.0 * a * k31, 12.0 * k31, -4.0 * (aa + 2.0 * ab + ac + bb + 2.0 * bc) * rb * rbc * k31},
      {4.0 * aa * k41, 12.0 * a * k41, 12.0 * k41, -4.0 * (aa + ab + 2.0 * ac + 2.0 * bc + c2) * rc * rbc * k41}};
  // first-case values at x = a = E21, written with a * r21 = 1 so that a = 0 gives zeros
  const double ka2 = k1 * a * a;
  coef[0][0] = ka2 * (3.0 - a * c.r31 - a * c.r41);
  coef[1][0] = ka2;
  coef[2][0] = ka2 * a * c.r31;
  coef[3][0] = ka2 * a * c.r41;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    coef[l][1] = g[l][0];
    coef[l][2] = 0.5 * g[l][1];
    coef[l][3] = (1.0 / 3.0) * g[l][2];
    coef[l][4] = 0.25 * g[l][3];
  }
}

__host__ __device__ __forceinline__ void corner_nos_B_poly(const double coef[4][5], double z, double w[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) w[l] = (((coef[l][4] * z + coef[l][3]) * z + coef[l][2]) * z + coef[l][1]) * z + coef[l][0];
}

__host__ __device__ __forceinline__ void corner_nos_C(const NosSetup& c, double V, double y, double w[4]) {
  const double t = c.kC * y * y * y;
  const double u = t * y;
  w[0] = V - u * c.r41;
  w[1] = V - u * c.r42;
  w[2] = V - u * c.r43;
  w[3] = V - t * (4.0 - y * c.sC);
}

// Moves the energy origin of the local frames by s (the energies become E_j = e0 + s + j*de); s = -de/2
// gives the midpoints between grid energies. Each head absorbs s exactly, the rounding goes to the tail.
__host__ __device__ __forceinline__ void shift_frames(TetSetup& c, float s) {
  float hi, lo;
  two_sum(c.d_hi, s, hi, lo);
  c.d_hi = hi;
  c.d_lo += lo;
  two_sum(c.f_hi, s, hi, lo);
  c.f_hi = hi;
  c.f_lo += lo;
  two_sum(c.h_hi, s, hi, lo);
  c.h_hi = hi;
  c.h_lo += lo;
}

// Steps of one tetrahedron-band's number of states on the grid E_j = e0 + (j + joff) de, with the
// frames of c shifted by joff*de: ja = first j with x_j > 0 (E_j > E1), js = first j with x_j >= E41
// (E_j >= E4), exact from estimates and the local frame. Indices below 0 or beyond the grid are only
// determined as such (the estimates are clamped to [-2, 3e7]).
__host__ __device__ __forceinline__ void step_window(const TetSetup& c, float e1, float e4, float e0, float joff,
                                                     float de, float inv_de, int& ja, int& js) {
  const float big = 3.0e7f;
  const float t1 = fminf(fmaxf((e1 - e0) * inv_de - joff, -2.0f), big);
  const float t4 = fminf(fmaxf((e4 - e0) * inv_de - joff, -2.0f), big);
  ja = (int)floorf(t1) + 1;
  js = (int)ceilf(t4);
  if (!(local_x(c, ja, de) > 0.0f)) ++ja;
  else if (local_x(c, ja - 1, de) > 0.0f) --ja;
  if (!(local_x(c, js, de) >= c.e41)) ++js;
  else if (local_x(c, js - 1, de) >= c.e41) --js;
}

}  // namespace tetra
