// Device-side building blocks of the tetrahedron DOS kernels (gfx950). Internal header.
//
// The corner weights implement the five energy cases of Sec. II.C of Guterding & Jeschke
// (arXiv:1710.10789). The kernels use algebraically simplified forms of the printed formulas:
//
//   first case (E1 < E <= E2), x = E - E1, K = V / (E21 E31 E41), S = 1/E21 + 1/E31 + 1/E41:
//       g1 = 4 K x^2 (3 - x S),   g_l = 4 K x^3 / E_l1  (l = 2, 3, 4)
//   third case (E3 < E < E4), y = E4 - E, K' = V / (E41 E42 E43), S' = 1/E41 + 1/E42 + 1/E43:
//       g_l = 4 K' y^3 / E_4l  (l = 1, 2, 3),   g4 = 4 K' y^2 (3 - y S')
//   middle case (E2 < E <= E3): the printed C1, C2, C3 and their derivatives with z = E - E2,
//       q = E3 - E, p = E4 - E, and the last term of dw3/dE taken as (C2 + C3)/E32, the form
//       that is the energy derivative of the printed w3.
//
// with V = V_T / (4 V_G). Energies are handled in a local frame: x = E_j - E1 is formed once per
// (tetrahedron, band, j) from e0 - E1 split into a head and an exact tail, so that the absolute
// magnitude of the energies does not cost resolution.
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
  float e21, e31, e41;         // E2 - E1, E3 - E1, E4 - E1
  float kA, sA;                // first case: K, S
  float kC, sC;                // third case: K', S'
  float r21, r31, r41, r32, r42, r43;
  float k1, k2, k3;            // middle case: V/(E31 E41), V/(E31 E32 E41), V/(E32 E41 E42)
};

__host__ __device__ __forceinline__ TetSetup tet_setup(const float e[4], float e0, float V) {
  TetSetup c;
  two_sum(e0, -e[0], c.d_hi, c.d_lo);
  c.e21 = e[1] - e[0];
  c.e31 = e[2] - e[0];
  c.e41 = e[3] - e[0];
  const float e32 = e[2] - e[1], e42 = e[3] - e[1], e43 = e[3] - e[2];
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

// dw_l/dE at local energy x, sorted-corner order, one function per energy case:
// A: 0 < x <= E21 (E1 < E <= E2), B: E21 < x <= E31 (E2 < E <= E3), C: E31 < x < E41 (E3 < E < E4).
__host__ __device__ __forceinline__ void corner_dos_A(const TetSetup& c, float x, float g[4]) {
  const float t = 4.0f * c.kA * x * x;
  const float u = t * x;
  g[0] = t * (3.0f - x * c.sA);
  g[1] = u * c.r21;
  g[2] = u * c.r31;
  g[3] = u * c.r41;
}

__host__ __device__ __forceinline__ void corner_dos_B(const TetSetup& c, float x, float g[4]) {
  const float z = x - c.e21, q = c.e31 - x, p = c.e41 - x;
  const float C1 = c.k1 * x * x, dC1 = 2.0f * c.k1 * x;
  const float C2 = c.k2 * x * z * q, dC2 = c.k2 * (x * q + z * q - x * z);
  const float C3 = c.k3 * z * z * p, dC3 = c.k3 * z * (2.0f * p - z);
  const float S12 = C1 + C2, D12 = dC1 + dC2, S23 = C2 + C3, D23 = dC2 + dC3;
  const float S123 = S12 + C3, D123 = D12 + dC3;
  g[0] = dC1 + (D12 * q - S12) * c.r31 + (D123 * p - S123) * c.r41;
  g[1] = D123 + (D23 * q - S23) * c.r32 + (dC3 * p - C3) * c.r42;
  g[2] = (D12 * x + S12) * c.r31 + (D23 * z + S23) * c.r32;
  g[3] = (D123 * x + S123) * c.r41 + (dC3 * z + C3) * c.r42;
}

__host__ __device__ __forceinline__ void corner_dos_C(const TetSetup& c, float x, float g[4]) {
  const float y = c.e41 - x;
  const float t = 4.0f * c.kC * y * y;
  const float u = t * y;
  g[0] = u * c.r41;
  g[1] = u * c.r42;
  g[2] = u * c.r43;
  g[3] = t * (3.0f - y * c.sC);
}

// dw_l/dE at local energy x (0 < x < E41 assumed by the caller).
__host__ __device__ __forceinline__ void corner_dos(const TetSetup& c, float x, float g[4]) {
  if (x <= c.e21) corner_dos_A(c, x, g);
  else if (x <= c.e31) corner_dos_B(c, x, g);
  else corner_dos_C(c, x, g);
}

// Adjoint of the corner weights for the gradient with respect to the corner energies. For multipliers
// s[4] (one per sorted corner) the quantity sum_l s_l g_l(E) depends on the sorted energies E_1..E_4
// through the local variables (x = E - E1, ...) and through the per-tetrahedron constants (reciprocal
// differences and the K factors). Reverse accumulation per energy gives adjoints that are linear in s,
// so over the energies of one case range they are summed first (the *_acc functions, which also
// return g for the weight gradient) and pushed through the constants once (the *_finish functions),
// which yields Eb[i] = sum over the range of d(sum_l s_l g_l)/dE_i at fixed E.

struct AdjA {  // first and third case: adjoint sums of the local variable, the reciprocals, K
  float vb, ra, rb, rc, kb;
};

__host__ __device__ __forceinline__ void adj_zero(AdjA& a) { a.vb = a.ra = a.rb = a.rc = a.kb = 0.0f; }

// First case: g1 = 4K x^2 (3 - x S), g_l = 4K x^3 r_l1 (l = 2, 3, 4), S = r21 + r31 + r41.
__host__ __device__ __forceinline__ void corner_dos_adjoint_acc_A(const TetSetup& c, float x, const float s[4], float g[4],
                                                                  AdjA& a) {
  const float t = 4.0f * c.kA * x * x;
  const float u = t * x;
  const float w = 3.0f - x * c.sA;
  g[0] = t * w;
  g[1] = u * c.r21;
  g[2] = u * c.r31;
  g[3] = u * c.r41;
  const float s0t = s[0] * t;
  const float sA_b = -s0t * x;
  const float u_b = s[1] * c.r21 + s[2] * c.r31 + s[3] * c.r41;
  a.ra += s[1] * u + sA_b;
  a.rb += s[2] * u + sA_b;
  a.rc += s[3] * u + sA_b;
  const float t_b = s[0] * w + u_b * x;
  a.kb += t_b * x * x;  // dt/dK = 4 x^2: the 4 is applied in the finish
  a.vb += u_b * t - s0t * c.sA + t_b * 8.0f * c.kA * x;
}

__host__ __device__ __forceinline__ void corner_dos_adjoint_finish_A(const TetSetup& c, float V, const AdjA& a, float Eb[4]) {
  const float kA_b = 4.0f * a.kb * V;  // K = V r21 r31 r41
  const float r21_b = a.ra + kA_b * c.r31 * c.r41;
  const float r31_b = a.rb + kA_b * c.r21 * c.r41;
  const float r41_b = a.rc + kA_b * c.r21 * c.r31;
  const float e21_b = -r21_b * c.r21 * c.r21, e31_b = -r31_b * c.r31 * c.r31, e41_b = -r41_b * c.r41 * c.r41;
  Eb[0] = -(e21_b + e31_b + e41_b + a.vb);
  Eb[1] = e21_b;
  Eb[2] = e31_b;
  Eb[3] = e41_b;
}

// Third case (mirror of the first with y = E4 - E): g_l = 4K' y^3 r_4l (l = 1, 2, 3),
// g4 = 4K' y^2 (3 - y S'), S' = r41 + r42 + r43.
__host__ __device__ __forceinline__ void corner_dos_adjoint_acc_C(const TetSetup& c, float x, const float s[4], float g[4],
                                                                  AdjA& a) {
  const float y = c.e41 - x;
  const float t = 4.0f * c.kC * y * y;
  const float u = t * y;
  const float w = 3.0f - y * c.sC;
  g[0] = u * c.r41;
  g[1] = u * c.r42;
  g[2] = u * c.r43;
  g[3] = t * w;
  const float s3t = s[3] * t;
  const float sC_b = -s3t * y;
  const float u_b = s[0] * c.r41 + s[1] * c.r42 + s[2] * c.r43;
  a.ra += s[0] * u + sC_b;
  a.rb += s[1] * u + sC_b;
  a.rc += s[2] * u + sC_b;
  const float t_b = s[3] * w + u_b * y;
  a.kb += t_b * y * y;
  a.vb += u_b * t - s3t * c.sC + t_b * 8.0f * c.kC * y;
}

__host__ __device__ __forceinline__ void corner_dos_adjoint_finish_C(const TetSetup& c, float V, const AdjA& a, float Eb[4]) {
  const float kC_b = 4.0f * a.kb * V;  // K' = V r41 r42 r43
  const float r41_b = a.ra + kC_b * c.r42 * c.r43;
  const float r42_b = a.rb + kC_b * c.r41 * c.r43;
  const float r43_b = a.rc + kC_b * c.r41 * c.r42;
  const float e41_b = -r41_b * c.r41 * c.r41, e42_b = -r42_b * c.r42 * c.r42, e43_b = -r43_b * c.r43 * c.r43;
  // y = E4 - E depends on E4 only
  Eb[0] = -e41_b;
  Eb[1] = -e42_b;
  Eb[2] = -e43_b;
  Eb[3] = e41_b + e42_b + e43_b + a.vb;
}

struct AdjB {  // middle case: adjoint sums of x, z, q, p, the reciprocals and k1, k2, k3
  float xb, zb, qb, pb, r31b, r41b, r32b, r42b, k1b, k2b, k3b;
};

__host__ __device__ __forceinline__ void adj_zero(AdjB& a) {
  a.xb = a.zb = a.qb = a.pb = a.r31b = a.r41b = a.r32b = a.r42b = a.k1b = a.k2b = a.k3b = 0.0f;
}

// Middle case: the printed C1, C2, C3 and their energy derivatives (with the corrected last term of
// dw3/dE), differentiated in reverse through the same expressions as corner_dos_B.
__host__ __device__ __forceinline__ void corner_dos_adjoint_acc_B(const TetSetup& c, float x, const float s[4], float g[4],
                                                                  AdjB& a) {
  const float z = x - c.e21, q = c.e31 - x, p = c.e41 - x;
  const float C1 = c.k1 * x * x, dC1 = 2.0f * c.k1 * x;
  const float C2 = c.k2 * x * z * q, dC2 = c.k2 * (x * q + z * q - x * z);
  const float C3 = c.k3 * z * z * p, dC3 = c.k3 * z * (2.0f * p - z);
  const float S12 = C1 + C2, D12 = dC1 + dC2, S23 = C2 + C3, D23 = dC2 + dC3;
  const float S123 = S12 + C3, D123 = D12 + dC3;
  g[0] = dC1 + (D12 * q - S12) * c.r31 + (D123 * p - S123) * c.r41;
  g[1] = D123 + (D23 * q - S23) * c.r32 + (dC3 * p - C3) * c.r42;
  g[2] = (D12 * x + S12) * c.r31 + (D23 * z + S23) * c.r32;
  g[3] = (D123 * x + S123) * c.r41 + (dC3 * z + C3) * c.r42;
  // adjoints of the quantities the four outputs read
  float dC1_b = s[0];
  float D12_b = (s[0] * q + s[2] * x) * c.r31;
  float S12_b = (s[2] - s[0]) * c.r31;
  const float D123_b = s[0] * p * c.r41 + s[1] + s[3] * x * c.r41;
  const float S123_b = (s[3] - s[0]) * c.r41;
  const float D23_b = (s[1] * q + s[2] * z) * c.r32;
  const float S23_b = (s[2] - s[1]) * c.r32;
  float dC3_b = (s[1] * p + s[3] * z) * c.r42;
  float C3_b = (s[3] - s[1]) * c.r42;
  float q_b = s[0] * D12 * c.r31 + s[1] * D23 * c.r32;
  float p_b = s[0] * D123 * c.r41 + s[1] * dC3 * c.r42;
  float x_b = s[2] * D12 * c.r31 + s[3] * D123 * c.r41;
  float z_b = s[2] * D23 * c.r32 + s[3] * dC3 * c.r42;
  a.r31b += s[0] * (D12 * q - S12) + s[2] * (D12 * x + S12);
  a.r41b += s[0] * (D123 * p - S123) + s[3] * (D123 * x + S123);
  a.r32b += s[1] * (D23 * q - S23) + s[2] * (D23 * z + S23);
  a.r42b += s[1] * (dC3 * p - C3) + s[3] * (dC3 * z + C3);
  // partial sums
  S12_b += S123_b;
  C3_b += S123_b + S23_b;
  D12_b += D123_b;
  dC3_b += D123_b + D23_b;
  const float C2_b = S23_b + S12_b;
  const float dC2_b = D23_b + D12_b;
  const float C1_b = S12_b;
  dC1_b += D12_b;
  // C3, dC3
  a.k3b += dC3_b * z * (2.0f * p - z) + C3_b * z * z * p;
  z_b += dC3_b * c.k3 * (2.0f * p - 2.0f * z) + C3_b * 2.0f * c.k3 * z * p;
  p_b += dC3_b * 2.0f * c.k3 * z + C3_b * c.k3 * z * z;
  // C2, dC2
  a.k2b += dC2_b * (x * q + z * q - x * z) + C2_b * x * z * q;
  x_b += dC2_b * c.k2 * (q - z) + C2_b * c.k2 * z * q;
  q_b += dC2_b * c.k2 * (x + z) + C2_b * c.k2 * x * z;
  z_b += dC2_b * c.k2 * (q - x) + C2_b * c.k2 * x * q;
  // C1, dC1
  a.k1b += dC1_b * 2.0f * x + C1_b * x * x;
  x_b += dC1_b * 2.0f * c.k1 + C1_b * 2.0f * c.k1 * x;
  a.xb += x_b;
  a.zb += z_b;
  a.qb += q_b;
  a.pb += p_b;
}

__host__ __device__ __forceinline__ void corner_dos_adjoint_finish_B(const TetSetup& c, float V, const AdjB& a, float Eb[4]) {
  // k1 = V r31 r41, k2 = k1 r32, k3 = V r32 r41 r42
  const float k1_b = a.k1b + a.k2b * c.r32;
  const float r32_b = a.r32b + a.k2b * c.k1 + a.k3b * V * c.r41 * c.r42;
  const float r41_b = a.r41b + a.k3b * V * c.r32 * c.r42 + k1_b * V * c.r31;
  const float r42_b = a.r42b + a.k3b * V * c.r32 * c.r41;
  const float r31_b = a.r31b + k1_b * V * c.r41;
  const float e31_b = -r31_b * c.r31 * c.r31, e41_b = -r41_b * c.r41 * c.r41;
  const float e32_b = -r32_b * c.r32 * c.r32, e42_b = -r42_b * c.r42 * c.r42;
  // x = E - E1, z = E - E2, q = E3 - E, p = E4 - E
  Eb[0] = -a.xb - e31_b - e41_b;
  Eb[1] = -a.zb - e32_b - e42_b;
  Eb[2] = a.qb + e31_b + e32_b;
  Eb[3] = a.pb + e41_b + e42_b;
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
