// Susceptibility kernel: orbital-resolved imaginary part of the bare (Lindhard) susceptibility at zero
// temperature for a transfer q on the k-grid, as the spectral weight S_m(q, w) of tetra_chi_device.h
// (Im chi_0 = -pi S), by the linear tetrahedron method of Guterding & Jeschke (arXiv:1710.10789,
// Sec. II) with the difference energy eps_n'(k + q) - eps_n(k) in the role of the band energy.
//
// Work decomposition, as the DOS forward: one workgroup per (tile of TX x TY x TZ cubes, band pair
// (n, n')), units tile-major, and each XCD takes a contiguous range of them. The tile's grid points
// are staged in LDS with eps_n at the point, eps_n' at the point shifted by q (periodic), and the
// product weights W_m = b_mn(k) b_mn'(k + q). Each energy pass runs two sweeps:
//  * one lane per cube over the six tetrahedra of Table I: an occupation region that is the whole
//    tetrahedron (band n occupied and n' empty at every corner, or the reverse; most of them) is the
//    DOS of eps' - eps formed as in the forward kernel (sort, exact window, case split, corner weights
//    of Sec. II.C); the other regions that may be non-empty go to a queue in LDS;
//  * every lane over the queued regions' sub-tetrahedra: a region is clipped at eps = E_F and
//    eps' = E_F into at most nine of them (held as barycentric rows in the parent); each takes the
//    same DOS treatment with W formed at its vertices and its share of the volume. The regions that
//    need clipping lie where a band crosses E_F, in a few cubes of a tile: shared out piece by piece
//    they no longer hold one wavefront, and the workgroup behind its barrier, for the whole pass.
// The LDS histograms hold fixed point with a power-of-two scale from a bound: the part of a
// tetrahedron on either side of an occupation boundary has a section no larger than the whole
// tetrahedron's, so a tetrahedron adds at most 12 V max|W| / (max - min of eps' - eps) to any bin
// (V = V_T/(4 V_G)). With non-negative weights each region's terms are non-negative: one histogram per
// region, two orbitals per 64-bit word; otherwise one signed 64-bit histogram. The sums are exact
// integers, so the order in which the queue is filled and worked off does not change them. One global
// float atomic per touched (energy, orbital) bin at the end.

#include <type_traits>

#include "tetra_chi_device.h"
#include "tetra_device.h"
#include "tetra_internal.h"
#include "tetra_weights.h"

namespace tetra {

namespace {

constexpr int NT = kTileCubes;
constexpr int NPMAX = kTilePointsMax;
constexpr int HCAP = 2048;  // LDS histogram capacity in 64-bit words
constexpr int NXCD = 8;

struct ChiArgs {
  const float* eps;
  const void* w;
  const float* w_scale;
  float* out;
  int n1, n2, n3, nb, ne;
  int q1, q2, q3;  // transfer in grid steps, reduced to [0, n)
  float ef, e0, de, inv_de, V;
  int TX, TY, TZ;
  int t1, t2, t3, ntiles, nunits, per_xcd;
  // Energy range (smallest, largest finite value) of every (tile, band): rows [0, nb) at the tile's
  // points, rows [nb, 2 nb) at the points shifted by q; NULL where not computed.
  const float2* ranges;
};

__device__ __forceinline__ int wrap_index(int v, int n) {
  if (v >= n) v -= n;
  if (v >= n) v %= n;
  return v;
}

__device__ __forceinline__ float wave_min_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// First pass of the workspace variant: one workgroup per (tile, band) writes the band's energy range
// over the tile's grid points (the points a unit stages) and over the same points shifted by q.
__global__ __launch_bounds__(NT) void chi_ranges_kernel(ChiArgs a) {
  __shared__ float s_r[4 * (NT / 64)];
  const int tile = blockIdx.x % a.ntiles, band = blockIdx.x / a.ntiles;
  const int PY = a.TY + 1, PZ = a.TZ + 1, NP = (a.TX + 1) * PY * PZ;
  const int tz = tile % a.t3, ty = (tile / a.t3) % a.t2, tx = tile / (a.t3 * a.t2);
  const int x0 = tx * a.TX, y0 = ty * a.TY, z0 = tz * a.TZ;
  const int64_t nk = (int64_t)a.n1 * a.n2 * a.n3;
  const float* e_b = a.eps + (int64_t)band * nk;
  float kmin = __builtin_huge_valf(), kmax = -__builtin_huge_valf(), qmin = kmin, qmax = kmax;
  for (int p = threadIdx.x; p < NP; p += NT) {
    const int pz = p % PZ, py = (p / PZ) % PY, px = p / (PZ * PY);
    const int i1 = wrap_index(x0 + px, a.n1), i2 = wrap_index(y0 + py, a.n2), i3 = wrap_index(z0 + pz, a.n3);
    const float e = e_b[((int64_t)i1 * a.n2 + i2) * a.n3 + i3];
    const float eq = e_b[((int64_t)wrap_index(i1 + a.q1, a.n1) * a.n2 + wrap_index(i2 + a.q2, a.n2)) * a.n3 +
                         wrap_index(i3 + a.q3, a.n3)];
    if (__builtin_isfinite(e)) {
      kmin = fminf(kmin, e);
      kmax = fmaxf(kmax, e);
    }
    if (__builtin_isfinite(eq)) {
      qmin = fminf(qmin, eq);
      qmax = fmaxf(qmax, eq);
    }
  }
  kmin = wave_min_f(kmin);
  kmax = wave_max_f(kmax);
  qmin = wave_min_f(qmin);
  qmax = wave_max_f(qmax);
  if ((threadIdx.x & 63) == 0) {
    const int wv = threadIdx.x >> 6;
    s_r[wv] = kmin;
    s_r[(NT / 64) + wv] = kmax;
    s_r[2 * (NT / 64) + wv] = qmin;
    s_r[3 * (NT / 64) + wv] = qmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int wv = 1; wv < NT / 64; ++wv) {
      kmin = fminf(kmin, s_r[wv]);
      kmax = fmaxf(kmax, s_r[(NT / 64) + wv]);
      qmin = fminf(qmin, s_r[2 * (NT / 64) + wv]);
      qmax = fmaxf(qmax, s_r[3 * (NT / 64) + wv]);
    }
    float2* r = const_cast<float2*>(a.ranges);
    r[(int64_t)band * a.ntiles + tile] = make_float2(kmin, kmax);
    r[(int64_t)(a.nb + band) * a.ntiles + tile] = make_float2(qmin, qmax);
  }
}

// Waves per SIMD the kernel is held to. With nothing of the clipping live over a sub-tetrahedron's
// energy loop it needs 100-140 VGPRs up to 8 orbitals (139 at 8: held to 4 waves it keeps 8 values in
// scratch, 2.00 against 2.27 ms at 3 waves for the 64^3 x 8 x 8 x 500 workload) and up to 196 at 16
// (held to 3 waves it keeps 30 values in scratch and still beats 2 waves: 4.68 against 5.18 ms for
// 48^3 x 16 x 16 x 500).
constexpr int chi_waves(int norb) { return norb <= 8 ? 4 : 3; }

template <int NORB, typename WT>
__global__ __launch_bounds__(NT, chi_waves(NORB)) void chi_kernel(ChiArgs a) {
  constexpr int RS = (HCAP / NORB - 1) | 1;  // histogram row stride (one row per orbital), odd
  __shared__ float s_e[NPMAX];
  __shared__ float s_ep[NPMAX];
  __shared__ float s_W[NPMAX * NORB];
  __shared__ unsigned long long s_hist[HCAP];
  __shared__ float s_red[8 * (NT / 64)];
  // regions to clip, queued by the first sweep of a pass and shared out over every lane by the second:
  // lane of the cube << 4 | tetrahedron << 1 | region (at most 6 x 2 per cube)
  __shared__ unsigned short s_q[NT * 12];
  __shared__ int s_qn;

  const int b = blockIdx.x;
  const int unit = (b % NXCD) * a.per_xcd + b / NXCD;
  if (unit >= a.nunits) return;
  // Tile-major units: the band pairs of one tile follow each other, so the tile's points (every band)
  // stay in the XCD's L2 while its pairs run.
  const int npairs = a.nb * a.nb;
  const int tile = unit / npairs;
  const int pair = unit - tile * npairs;
  const int n = pair / a.nb, np = pair - n * a.nb;
  const int TX = a.TX, TY = a.TY, TZ = a.TZ;
  const int PY = TY + 1, PZ = TZ + 1;
  const int NP = (TX + 1) * PY * PZ;
  const int tz = tile % a.t3;
  const int ty = (tile / a.t3) % a.t2;
  const int tx = tile / (a.t3 * a.t2);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int tid = threadIdx.x;
  const int64_t nk = (int64_t)a.n1 * a.n2 * a.n3;
  const float* eps_n = a.eps + (int64_t)n * nk;
  const float* eps_p = a.eps + (int64_t)np * nk;
  const WT* w_n = static_cast<const WT*>(a.w) + (int64_t)n * NORB * nk;
  const WT* w_p = static_cast<const WT*>(a.w) + (int64_t)np * NORB * nk;
  const float sc_n = a.w_scale ? a.w_scale[n] : 1.0f, sc_p = a.w_scale ? a.w_scale[np] : 1.0f;

  // With the first pass's ranges a unit that cannot contribute leaves before loading anything: the
  // tables bound the staged values (their ranges include points where only one band is finite), so
  // these tests only ever let through units that the exact ones below then drop.
  if (a.ranges) {
    const float2 rk = a.ranges[(int64_t)n * a.ntiles + tile];
    const float2 rq = a.ranges[(int64_t)(a.nb + np) * a.ntiles + tile];
    if (!(rk.x <= rk.y) || !(rq.x <= rq.y)) return;  // no finite energy in one of the bands
    if (!region_possible(0, rk.x, rk.y, rq.x, rq.y, a.ef) && !region_possible(1, rk.x, rk.y, rq.x, rq.y, a.ef))
      return;
    int K0, K1;
    range_window(rq.x - rk.y, rq.y - rk.x, a.e0, a.inv_de, a.ne, K0, K1);
    if (K0 > K1) return;
  }
  // Stage the tile's energies: eps_n at the point, eps_n' at the point + q; reduce the ranges of eps,
  // eps' and eps' - eps. Most (tile, band pair) units end here: no region can be occupied on one side
  // and empty on the other, or eps' - eps stays outside the energy grid; their weights are never read.
  auto point_k = [&](int p, int64_t& k, int64_t& kq) {
    const int pz = p % PZ, py = (p / PZ) % PY, px = p / (PZ * PY);
    const int i1 = wrap_index(x0 + px, a.n1), i2 = wrap_index(y0 + py, a.n2), i3 = wrap_index(z0 + pz, a.n3);
    k = ((int64_t)i1 * a.n2 + i2) * a.n3 + i3;
    kq = ((int64_t)wrap_index(i1 + a.q1, a.n1) * a.n2 + wrap_index(i2 + a.q2, a.n2)) * a.n3 +
         wrap_index(i3 + a.q3, a.n3);
  };
  float r_emin = __builtin_huge_valf(), r_emax = -__builtin_huge_valf();
  float r_pmin = __builtin_huge_valf(), r_pmax = -__builtin_huge_valf();
  float r_dmin = __builtin_huge_valf(), r_dmax = -__builtin_huge_valf();
  for (int p = tid; p < NP; p += NT) {
    int64_t k, kq;
    point_k(p, k, kq);
    const float e = eps_n[k], ep = eps_p[kq];
    s_e[p] = e;
    s_ep[p] = ep;
    if (__builtin_isfinite(e) && __builtin_isfinite(ep)) {
      r_emin = fminf(r_emin, e);
      r_emax = fmaxf(r_emax, e);
      r_pmin = fminf(r_pmin, ep);
      r_pmax = fmaxf(r_pmax, ep);
      r_dmin = fminf(r_dmin, ep - e);
      r_dmax = fmaxf(r_dmax, ep - e);
    }
  }
  float red[8] = {wave_min_f(r_emin), wave_max_f(r_emax), wave_min_f(r_pmin), wave_max_f(r_pmax),
                  wave_min_f(r_dmin), wave_max_f(r_dmax), 0.0f, 0.0f};
  if ((tid & 63) == 0)
#pragma unroll
    for (int i = 0; i < 6; ++i) s_red[i * (NT / 64) + (tid >> 6)] = red[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float v = s_red[i * (NT / 64)];
#pragma unroll
    for (int wv = 1; wv < NT / 64; ++wv) {
      const float x = s_red[i * (NT / 64) + wv];
      v = (i == 0 || i == 2 || i == 4) ? fminf(v, x) : fmaxf(v, x);
    }
    red[i] = v;
  }
  const float ef = a.ef;
  if (!(red[4] <= red[5])) return;  // no finite pair in this tile (uniform across the block)
  if (!region_possible(0, red[0], red[1], red[2], red[3], ef) && !region_possible(1, red[0], red[1], red[2], red[3], ef))
    return;
  int J0, J1;
  range_window(red[4], red[5], a.e0, a.inv_de, a.ne, J0, J1);
  if (J0 > J1) return;

  // The weights W = b_n(k) b_n'(k + q), with the largest |W| and the smallest W.
  float r_wmax = 0.0f, r_wmin = 0.0f;
  for (int p = tid; p < NP; p += NT) {
    int64_t k, kq;
    point_k(p, k, kq);
#pragma unroll
    for (int m = 0; m < NORB; ++m) {
      const float W = weight_value(w_n[(int64_t)m * nk + k], sc_n) * weight_value(w_p[(int64_t)m * nk + kq], sc_p);
      s_W[p * NORB + m] = W;
      r_wmax = fmaxf(r_wmax, fabsf(W));
      r_wmin = fminf(r_wmin, W);
    }
  }
  r_wmax = wave_max_f(r_wmax);
  r_wmin = wave_min_f(r_wmin);
  if ((tid & 63) == 0) {
    s_red[6 * (NT / 64) + (tid >> 6)] = r_wmax;
    s_red[7 * (NT / 64) + (tid >> 6)] = r_wmin;
  }
  __syncthreads();
  red[6] = s_red[6 * (NT / 64)];
  red[7] = s_red[7 * (NT / 64)];
#pragma unroll
  for (int wv = 1; wv < NT / 64; ++wv) {
    red[6] = fmaxf(red[6], s_red[6 * (NT / 64) + wv]);
    red[7] = fminf(red[7], s_red[7 * (NT / 64) + wv]);
  }
  const float wmax = red[6], wmin = red[7];

  const int cz = tid % TZ, cy = (tid / TZ) % TY, cx = tid / (TZ * TY);
  const bool valid = (x0 + cx < a.n1) && (y0 + cy < a.n2) && (z0 + cz < a.n3);
  const int pbase = (cx * PY + cy) * PZ + cz;
  auto point_offset = [PY, PZ](int s) { return (s & 1) * (PY * PZ) + ((s >> 1) & 1) * PZ + (s >> 2); };

  // Corner data of tetrahedron t of this lane's cube; false when it cannot contribute to [lo, hi].
  // whole: the region that is the whole tetrahedron (n occupied and n' empty at every corner for region
  // 0, the reverse for region 1), or -1.
  auto corners = [&](int t, int lo, int hi, int pt[4], float e[4], float ep[4], bool reg[2], int& whole) {
    const uint32_t slots = tet_slots(t);
    float emin = __builtin_huge_valf(), emax = -emin, pmin = emin, pmax = -emin, dmin = emin, dmax = -emin;
    bool fin = true;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      pt[l] = pbase + point_offset((slots >> (4 * l)) & 7);
      e[l] = s_e[pt[l]];
      ep[l] = s_ep[pt[l]];
      fin = fin && __builtin_isfinite(e[l]) && __builtin_isfinite(ep[l]);
      emin = fminf(emin, e[l]);
      emax = fmaxf(emax, e[l]);
      pmin = fminf(pmin, ep[l]);
      pmax = fmaxf(pmax, ep[l]);
      dmin = fminf(dmin, ep[l] - e[l]);
      dmax = fmaxf(dmax, ep[l] - e[l]);
    }
    if (!fin || !(dmax > dmin)) return false;
    whole = (emax <= ef && pmin >= ef) ? 0 : (emin >= ef && pmax <= ef) ? 1 : -1;
    reg[0] = region_possible(0, emin, emax, pmin, pmax, ef);
    reg[1] = region_possible(1, emin, emax, pmin, pmax, ef);
    if (!reg[0] && !reg[1]) return false;
    int jlo, jhi;
    energy_window(dmin, dmax, a.e0, a.inv_de, lo, hi, jlo, jhi);
    return jlo <= jhi + 2;
  };

  // Bound on any bin's |sum|: sum over tetrahedra that may contribute of 12 V max|W| / (dmax - dmin).
  // Narrow tetrahedra (a range of eps' - eps below 2 de) give spikes that make B loose.
  float bound = 0.0f, narrow = 0.0f;
  if (valid) {
#pragma unroll 1
    for (int t = 0; t < 6; ++t) {
      int pt[4];
      float e[4], ep[4];
      bool reg[2];
      int whole;
      if (!corners(t, J0, J1, pt, e, ep, reg, whole)) continue;
      float dmin = ep[0] - e[0], dmax = dmin;
#pragma unroll
      for (int l = 1; l < 4; ++l) {
        dmin = fminf(dmin, ep[l] - e[l]);
        dmax = fmaxf(dmax, ep[l] - e[l]);
      }
      const float term = 12.0f * a.V * wmax * rcp(dmax - dmin);
      bound += term;
      if (dmax - dmin < 2.0f * a.de) narrow += term;
    }
  }
  bound = wave_sum_f(fminf(bound, 1.0e37f));
  narrow = wave_sum_f(fminf(narrow, 1.0e37f));
  __syncthreads();  // every lane has read s_red
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = bound;
    s_red[(NT / 64) + (tid >> 6)] = narrow;
  }
  __syncthreads();
  float B = 0.0f, Bn = 0.0f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    B += s_red[i];
    Bn += s_red[NT / 64 + i];
  }
  if (!(B > 0.0f)) return;  // nothing to add (uniform across the block)
  // Packed: within one region every contribution is non-negative when the weights are (corner weights
  // and barycentric coordinates are), so each region gets a histogram of its own with two orbitals per
  // 64-bit word as 32-bit fields (B S <= 2^30, no carry between fields) and the result is their
  // difference. Otherwise one signed 64-bit histogram (B S <= 2^62).
  const bool packed = wmin >= 0.0f && Bn <= 0.5f * B;  // uniform across the block
  int bexp;
  frexpf(fminf(B, 3.0e38f), &bexp);  // B <= 2^bexp
  const int sexp = min((packed ? 30 : 62) - bexp, 126);
  const float VS = a.V * ldexpf(1.0f, sexp);  // V_T/(4 V_G) in units of the fixed point
  const double inv_S = ldexp(1.0, -sexp);

  auto passes = [&](auto packed_tag) {
    constexpr bool PACKED = decltype(packed_tag)::value;
    constexpr int NPAIR = (NORB + 1) / 2;
    // rows: packed, one per orbital pair in each region's half of the histogram; wide, one per orbital
    constexpr int RSP = (HCAP / 2 / NPAIR - 1) | 1;
    constexpr int RSX = PACKED ? RSP : RS;
    unsigned long long* hist_m = s_hist + (PACKED ? HCAP / 2 : 0);  // region -1 (packed only)
    // Corner weights dw/dE of a (sub-)tetrahedron's sorted vertices at grid energy j.
    auto corner_g = [&](const TetSetup& cs, const float (&coef)[4][4], int j, int jA, int jB, float g[4]) {
      if (j <= jA) {
        corner_dos_A(cs, local_x(cs, j, a.de), g);
        g[0] = fmaxf(g[0], 0.0f);
      } else if (j <= jB) {
        corner_dos_B_poly(coef, local_z(cs, j, a.de), g);
#pragma unroll
        for (int l = 0; l < 4; ++l) g[l] = fmaxf(g[l], 0.0f);
      } else {
        corner_dos_C(cs, local_y(cs, j, a.de), g);
        g[3] = fmaxf(g[3], 0.0f);
      }
    };
    // One energy's terms sum_l G_l Wr[l][m] into the region's histogram row h.
    auto deposit = [&](unsigned long long* h, float G[4], const float (&Wr)[4][NORB], float sign) {
      if (PACKED) {
        // non-negative terms: the truncating conversion of 1/2 + v rounds (halves up)
#pragma unroll
        for (int pr = 0; pr < NPAIR; ++pr) {
          const int m0 = 2 * pr, m1 = 2 * pr + 1;
          const float v0 = __builtin_fmaf(G[0], Wr[0][m0], __builtin_fmaf(G[1], Wr[1][m0],
                           __builtin_fmaf(G[2], Wr[2][m0], __builtin_fmaf(G[3], Wr[3][m0], 0.5f))));
          unsigned long long word = (unsigned long long)(unsigned)v0;
          if (m1 < NORB) {
            const float v1 = __builtin_fmaf(G[0], Wr[0][m1], __builtin_fmaf(G[1], Wr[1][m1],
                             __builtin_fmaf(G[2], Wr[2][m1], __builtin_fmaf(G[3], Wr[3][m1], 0.5f))));
            word |= (unsigned long long)(unsigned)v1 << 32;
          }
          atomicAdd(&h[pr * RSX], word);
        }
      } else {
#pragma unroll
        for (int l = 0; l < 4; ++l) G[l] *= sign;
#pragma unroll
        for (int m = 0; m < NORB; ++m) {
          const float v = __builtin_fmaf(G[0], Wr[0][m], __builtin_fmaf(G[1], Wr[1][m],
                                         __builtin_fmaf(G[2], Wr[2][m], G[3] * Wr[3][m])));
          atomicAdd(&h[m * RSX], (unsigned long long)__float2ll_rn(v));
        }
      }
    };
    for (int c0 = J0; c0 <= J1; c0 += RSX) {
      const int c1 = min(c0 + RSX - 1, J1);
      const int L = c1 - c0 + 1;
      const int rows = PACKED ? NPAIR : NORB;
      for (int q = tid; q < rows * L; q += NT) {
        const int m = q / L;
        s_hist[m * RSX + (q - m * L)] = 0ull;
        if (PACKED) hist_m[m * RSX + (q - m * L)] = 0ull;
      }
      if (tid == 0) s_qn = 0;
      __syncthreads();
      // First sweep, every lane on its own cube: the regions that are the whole tetrahedron, most of
      // them, as the forward kernel forms a DOS (the corners sorted with their points, the weights read
      // in sorted order, no clipping), and the other regions queued. The regions that need clipping lie where a band crosses E_F, in a
      // few cubes of the tile; sharing them out over all lanes keeps them from holding one wavefront,
      // and the workgroup behind its barrier, for the whole pass.
      if (valid) {
#pragma unroll 1
        for (int t = 0; t < 6; ++t) {
          int pt[4];
          float e[4], ep[4];
          bool reg[2];
          int whole;
          if (!corners(t, c0, c1, pt, e, ep, reg, whole)) continue;
#pragma unroll
          for (int r = 0; r < 2; ++r)
            if (reg[r] && r != whole) s_q[atomicAdd(&s_qn, 1)] = (unsigned short)((tid << 4) | (t << 1) | r);
          if (whole < 0) continue;
          float d[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) d[c] = ep[c] - e[c];
          sort4(d, pt);
          int jlo, jhi;
          energy_window(d[0], d[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
          if (jlo > jhi + 2) continue;
          const TetSetup cs = tet_setup(d, a.e0, VS);
          tet_window(cs, a.de, c0, c1, jlo, jhi);
          if (jlo > jhi) continue;
          float ws[4][NORB];
#pragma unroll
          for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int m = 0; m < NORB; ++m) ws[l][m] = s_W[pt[l] * NORB + m];
          int jA, jB;
          case_split(cs, a.de, a.inv_de, jlo, jhi, jA, jB);
          float coef[4][4];
          if (jB > jA) corner_dos_B_coeffs(cs, VS, coef);
          const float sign = whole == 0 ? 1.0f : -1.0f;
          unsigned long long* hreg = (PACKED && whole == 1) ? hist_m : s_hist;
          for (int j = jlo; j <= jhi; ++j) {
            float g[4];
            corner_g(cs, coef, j, jA, jB, g);
            deposit(&hreg[j - c0], g, ws, sign);
          }
        }
      }
      __syncthreads();
      // Second sweep: the queued regions, clipped at the two occupation boundaries into at most 3 x 3
      // sub-tetrahedra. The lanes take (first piece, second piece, region) slots, piece-major: a
      // region's first slot holds a piece unless the region is empty, the others only for some
      // regions, so the slots with work stay together and a wavefront whose slots hold no piece
      // leaves early. Each slot redoes its region's
      // planes and first clipping from LDS (nothing of the clipping stays live over a piece's energy
      // loop) and leaves early if its piece does not exist.
      const int nq = s_qn;
      constexpr float I[4][4] = {{1.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 1.0f, 0.0f, 0.0f},
                                 {0.0f, 0.0f, 1.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 1.0f}};
#pragma unroll 1
      for (int ip = tid; ip < 9 * nq; ip += NT) {
        const int piece = ip / nq, iq = ip - piece * nq;
        const int ia = piece / 3, ib = piece - 3 * ia;
        const int item = s_q[iq];
        const int it = item >> 4, t = (item >> 1) & 7, r = item & 1;
        const int qz = it % TZ, qy = (it / TZ) % TY, qx = it / (TZ * TY);
        const int qbase = (qx * PY + qy) * PZ + qz;
        // Occupation planes at the corners (f1, f2c <= 0 inside), the difference energies dd and the
        // corners' points, reordered so that the corners inside the first plane come first: the first
        // clipping then starts from the identity, whose unit rows fold into constants.
        float f1[4], f2c[4], dd[4];
        int q[4];
        {
          const uint32_t slots = tet_slots(t);
          float er[4], epr[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            q[c] = qbase + point_offset((slots >> (4 * c)) & 7);
            er[c] = s_e[q[c]];
            epr[c] = s_ep[q[c]];
          }
          region_planes(r, er, epr, ef, f1, f2c);
#pragma unroll
          for (int c = 0; c < 4; ++c) dd[c] = epr[c] - er[c];
        }
        const int ni1 = (f1[0] <= 0.0f) + (f1[1] <= 0.0f) + (f1[2] <= 0.0f) + (f1[3] <= 0.0f);
        if (ia >= clip_pieces(ni1)) continue;
        if (ni1 > 0 && ni1 < 4) inside_first_corners(f1, f2c, dd, q);
        float A[4][4], f2[4];
        if (ni1 == 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) A[i][c] = I[i][c];
        } else {
          clip_piece(I, f1, ni1, ia, A);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          f2[i] = __builtin_fmaf(A[i][0], f2c[0], __builtin_fmaf(A[i][1], f2c[1],
                                 __builtin_fmaf(A[i][2], f2c[2], A[i][3] * f2c[3])));
        const int ni2 = (f2[0] <= 0.0f) + (f2[1] <= 0.0f) + (f2[2] <= 0.0f) + (f2[3] <= 0.0f);
        if (ib >= clip_pieces(ni2)) continue;
        if (ni2 > 0 && ni2 < 4) inside_first(A, f2);
        float S[4][4];
        float frac;
        if (ni2 == 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) S[i][c] = A[i][c];
          frac = ni1 == 4 ? 1.0f : sub_volume(S);
        } else {
          clip_piece(A, f2, ni2, ib, S);
          frac = sub_volume(S);
        }
        if (!(frac > 0.0f)) continue;
        float d[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          d[i] = __builtin_fmaf(S[i][0], dd[0], __builtin_fmaf(S[i][1], dd[1],
                                __builtin_fmaf(S[i][2], dd[2], S[i][3] * dd[3])));
        sort4_rows(d, S);
        int jlo, jhi;
        energy_window(d[0], d[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
        if (jlo > jhi + 2) continue;
        const float Vs = VS * frac;
        const TetSetup cs = tet_setup(d, a.e0, Vs);
        tet_window(cs, a.de, c0, c1, jlo, jhi);
        if (jlo > jhi) continue;
        // W at the sorted vertices (linear on the parent): Wv[l] = sum_c S[l][c] W_c
        float wv[4][NORB];
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
          for (int m = 0; m < NORB; ++m) wv[l][m] = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int m = 0; m < NORB; ++m) {
            const float wc = s_W[q[c] * NORB + m];
#pragma unroll
            for (int l = 0; l < 4; ++l) wv[l][m] = __builtin_fmaf(S[l][c], wc, wv[l][m]);
          }
        int jA, jB;
        case_split(cs, a.de, a.inv_de, jlo, jhi, jA, jB);
        float coef[4][4];
        if (jB > jA) corner_dos_B_coeffs(cs, Vs, coef);
        const float sign = r == 0 ? 1.0f : -1.0f;
        unsigned long long* hreg = (PACKED && r == 1) ? hist_m : s_hist;
        for (int j = jlo; j <= jhi; ++j) {
          float g[4];
          corner_g(cs, coef, j, jA, jB, g);
          deposit(&hreg[j - c0], g, wv, sign);
        }
      }
      __syncthreads();
      for (int q = tid; q < L * NORB; q += NT) {
        const int rr = q / NORB, m = q - rr * NORB;
        double v;
        if (PACKED) {
          const unsigned long long wp = s_hist[(m >> 1) * RSX + rr], wm = hist_m[(m >> 1) * RSX + rr];
          const unsigned fp = (m & 1) ? (unsigned)(wp >> 32) : (unsigned)(wp & 0xffffffffull);
          const unsigned fm = (m & 1) ? (unsigned)(wm >> 32) : (unsigned)(wm & 0xffffffffull);
          v = (double)fp - (double)fm;
        } else {
          v = (double)(long long)s_hist[m * RSX + rr];
        }
        if (v != 0.0) unsafeAtomicAdd(&a.out[(int64_t)(c0 + rr) * NORB + m], (float)(v * inv_S));
      }
      __syncthreads();
    }
  };
  if (packed)
    passes(std::true_type{});
  else
    passes(std::false_type{});
}

template <int NORB>
hipError_t launch_chi(const ChiArgs& a, int wtype, int grid, hipStream_t s) {
  if (wtype == TETRA_W_F16)
    hipLaunchKernelGGL((chi_kernel<NORB, _Float16>), dim3(grid), dim3(NT), 0, s, a);
  else if (wtype == TETRA_W_C32)
    hipLaunchKernelGGL((chi_kernel<NORB, float2>), dim3(grid), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((chi_kernel<NORB, float>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int64_t chi_units(const tetra_desc& d, int shape) {
  const TileShape sh = tile_shape(shape);
  const int64_t ntiles = (int64_t)((d.n1 + sh.x - 1) / sh.x) * ((d.n2 + sh.y - 1) / sh.y) * ((d.n3 + sh.z - 1) / sh.z);
  return ntiles * d.nb * d.nb;
}

int64_t chi_range_entries(const tetra_desc& d, int shape) {
  const TileShape sh = tile_shape(shape);
  return 2 * (int64_t)d.nb * ((d.n1 + sh.x - 1) / sh.x) * ((d.n2 + sh.y - 1) / sh.y) * ((d.n3 + sh.z - 1) / sh.z);
}

hipError_t chi(const tetra_desc& d, int q1, int q2, int q3, float e_fermi, const float* eps, const void* w, int wtype,
               const float* w_scale, float* out, int shape, void* ranges_ws, hipStream_t s) {
  ChiArgs a;
  a.eps = eps;
  a.w = w;
  a.w_scale = w_scale;
  a.out = out;
  a.n1 = d.n1;
  a.n2 = d.n2;
  a.n3 = d.n3;
  a.nb = d.nb;
  a.ne = d.ne;
  a.q1 = ((q1 % d.n1) + d.n1) % d.n1;
  a.q2 = ((q2 % d.n2) + d.n2) % d.n2;
  a.q3 = ((q3 % d.n3) + d.n3) % d.n3;
  a.ef = e_fermi;
  a.e0 = d.e0;
  a.de = d.de;
  a.inv_de = 1.0f / d.de;
  a.V = (float)(1.0 / (24.0 * (double)d.n1 * d.n2 * d.n3));
  const TileShape sh = tile_shape(shape);
  a.TX = sh.x;
  a.TY = sh.y;
  a.TZ = sh.z;
  a.t1 = (d.n1 + sh.x - 1) / sh.x;
  a.t2 = (d.n2 + sh.y - 1) / sh.y;
  a.t3 = (d.n3 + sh.z - 1) / sh.z;
  a.ntiles = a.t1 * a.t2 * a.t3;
  a.nunits = (int)chi_units(d, shape);
  a.per_xcd = (a.nunits + NXCD - 1) / NXCD;
  const int grid = a.per_xcd * NXCD;
  a.ranges = static_cast<const float2*>(ranges_ws);
  hipError_t e = fill_zero(out, (int64_t)d.ne * d.norb, s);
  if (e != hipSuccess) return e;
  if (ranges_ws) {
    hipLaunchKernelGGL(chi_ranges_kernel, dim3(a.ntiles * d.nb), dim3(NT), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (d.norb) {
#define TETRA_CASE(N) \
  case N:             \
    return launch_chi<N>(a, wtype, grid, s);
    TETRA_CASE(1) TETRA_CASE(2) TETRA_CASE(3) TETRA_CASE(4) TETRA_CASE(5) TETRA_CASE(6) TETRA_CASE(7)
    TETRA_CASE(8) TETRA_CASE(9) TETRA_CASE(10) TETRA_CASE(11) TETRA_CASE(12) TETRA_CASE(13)
    TETRA_CASE(14) TETRA_CASE(15) TETRA_CASE(16)
#undef TETRA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace tetra
