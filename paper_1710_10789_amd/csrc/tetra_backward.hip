// Backward (adjoint) kernel of the orbital-resolved tetrahedron DOS on gfx950.
//
// For a scalar loss L with G[j][m] = dL/dDOS[j][m], the forward sum
//   DOS[j][m] = sum_{tetrahedra, n, l} b[n][m][k_l] g_l(E_j; E_1..E_4)
// (eq. tetmethoorbitalresolved with the corner weights of Sec. II.C, arXiv:1710.10789) gives
//   dL/db[n][m][k] = sum over the incidences (tetrahedron, corner l) of k of sum_j G[j][m] g_l(E_j)
//   dL/deps[n][k]  = sum over the incidences of sum_j sum_l s_l(E_j) dg_l(E_j)/dE_{corner of k},
//                    s_l(E_j) = sum_m G[j][m] b[n][m][k_l].
// The derivative through the sort is the identity on the corner each sorted energy came from.
//
// Work decomposition: output-stationary. One workgroup owns a tile of OX x OY x OZ k-points of one
// band and processes every cube that has one of them as a corner (the tile's cubes plus a one-cube
// halo below it, recomputed by the neighbouring workgroups too). Gradients of owned points are
// written once with plain coalesced stores: no global atomics and no zero-fill pass.
// Inside the workgroup there are no atomics either (LDS float atomics are slow on gfx950): all lanes
// work on the same tetrahedron index t at a time, one cube per lane, so for each of t's four corners
// the map cube -> corner point is injective across lanes. After a tetrahedron, four barrier-separated
// rounds add each lane's per-corner sums into LDS point totals with plain read-modify-writes.

#include "tetra_device.h"
#include "tetra_internal.h"

namespace tetra {

namespace {

constexpr int OX = 4, OY = 4, OZ = 16;         // owned k-points per tile along axes 1, 2, 3
constexpr int NT = 256;                        // threads per workgroup
constexpr int NOWN = OX * OY * OZ;             // owned points
constexpr int SX = OX + 2, SY = OY + 2, SZ = OZ + 2;  // staged points (halo cube layer + top corners)
constexpr int NSP = SX * SY * SZ;
constexpr int HCAP = 4096;  // LDS capacity for the rows of G, in floats
constexpr int NXCD = 8;

struct BwdArgs {
  const float* eps;
  const float* w;
  const float* G;
  float* grad_eps;
  float* grad_w;
  int n1, n2, n3, ne;
  float e0, de, inv_de, V;
  int t1, t2, t3;
  int ntiles, nunits, per_xcd;
};

__device__ __forceinline__ int wrap_pos(int v, int n) {  // v >= 0
  while (v >= n) v -= n;
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Per axis: owned points [x0, x0 + own) and the cubes touching them, cube origins start + i for
// i in [0, cnt) (mod n). When one tile owns the whole axis every cube of that axis is processed once.
struct AxisPlan {
  int x0, own, start, cnt;
};

__device__ __forceinline__ AxisPlan axis_plan(int tile_index, int O, int n) {
  AxisPlan p;
  p.x0 = tile_index * O;
  p.own = min(O, n - p.x0);
  if (p.own == n) {
    p.start = 0;
    p.cnt = n;
  } else {
    p.start = p.x0 - 1 + n;  // kept non-negative; reduced mod n where used
    p.cnt = p.own + 1;
  }
  return p;
}

template <int NORB>
__global__ __launch_bounds__(NT) void dos_backward_kernel(BwdArgs a) {
  constexpr int LC = HCAP / NORB;
  __shared__ float s_eps[NSP];
  __shared__ float s_w[NSP * NORB];
  __shared__ short s_own[NSP];     // owned-point index of a staged point, or -1
  __shared__ float s_pt[NSP * (NORB + 1)];  // per staged point: dL/deps, then dL/db[0..NORB)
  __shared__ float s_G[HCAP];
  __shared__ float s_red[2 * (NT / 64)];

  const int b = blockIdx.x;
  const int unit = (b % NXCD) * a.per_xcd + b / NXCD;
  if (unit >= a.nunits) return;
  const int band = unit / a.ntiles;
  const int tile = unit - band * a.ntiles;
  const AxisPlan P3 = axis_plan(tile % a.t3, OZ, a.n3);
  const AxisPlan P2 = axis_plan((tile / a.t3) % a.t2, OY, a.n2);
  const AxisPlan P1 = axis_plan(tile / (a.t3 * a.t2), OX, a.n1);
  const int tid = threadIdx.x;
  const int64_t nk = (int64_t)a.n1 * a.n2 * a.n3;
  const float* eps_n = a.eps + (int64_t)band * nk;
  const float* w_n = a.w + (int64_t)band * NORB * nk;

  for (int q = tid; q < NSP * (NORB + 1); q += NT) s_pt[q] = 0.0f;

  // Stage the corner points of the processed cubes; mark the owned ones.
  float lmin = __builtin_huge_valf(), lmax = -__builtin_huge_valf();
  for (int p = tid; p < NSP; p += NT) {
    const int i3 = p % SZ, i2 = (p / SZ) % SY, i1 = p / (SZ * SY);
    if (i1 > P1.cnt || i2 > P2.cnt || i3 > P3.cnt) {
      s_own[p] = -1;
      continue;
    }
    const int g1 = wrap_pos(P1.start + i1, a.n1), g2 = wrap_pos(P2.start + i2, a.n2),
              g3 = wrap_pos(P3.start + i3, a.n3);
    const int64_t k = ((int64_t)g1 * a.n2 + g2) * a.n3 + g3;
    const float e = eps_n[k];
    s_eps[p] = e;
    if (__builtin_isfinite(e)) {
      lmin = fminf(lmin, e);
      lmax = fmaxf(lmax, e);
    }
#pragma unroll
    for (int m = 0; m < NORB; ++m) s_w[p * NORB + m] = w_n[(int64_t)m * nk + k];
    const int d1 = g1 - P1.x0, d2 = g2 - P2.x0, d3 = g3 - P3.x0;
    const bool owned = d1 >= 0 && d1 < P1.own && d2 >= 0 && d2 < P2.own && d3 >= 0 && d3 < P3.own;
    s_own[p] = owned ? (short)((d1 * OY + d2) * OZ + d3) : (short)-1;
  }
  lmin = wave_min(lmin);
  lmax = wave_max(lmax);
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = lmin;
    s_red[(NT / 64) + (tid >> 6)] = lmax;
  }
  __syncthreads();
  float emin = s_red[0], emax = s_red[NT / 64];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    emin = fminf(emin, s_red[i]);
    emax = fmaxf(emax, s_red[NT / 64 + i]);
  }
  int J0 = 0, J1 = -1;
  if (emin <= emax) range_window(emin, emax, a.e0, a.inv_de, a.ne, J0, J1);

  const int ncubes = P1.cnt * P2.cnt * P3.cnt;
  auto point_offset = [](int s) { return (s & 1) * (SY * SZ) + ((s >> 1) & 1) * SZ + (s >> 2); };

  for (int c0 = J0; c0 <= J1; c0 += LC) {
    const int c1 = min(c0 + LC - 1, J1);
    const int L = c1 - c0 + 1;
    for (int q = tid; q < L * NORB; q += NT) s_G[q] = a.G[(int64_t)c0 * NORB + q];
    __syncthreads();
    for (int cr = 0; cr < ncubes; cr += NT) {  // rounds of one cube per lane
      const int c = cr + tid;
      const bool active = c < ncubes;
      const int c3 = active ? c % P3.cnt : 0, c2 = active ? (c / P3.cnt) % P2.cnt : 0;
      const int c1i = active ? c / (P3.cnt * P2.cnt) : 0;
      const int pbase = (c1i * SY + c2) * SZ + c3;
#pragma unroll 1
      for (int t = 0; t < 6; ++t) {
        const uint32_t slots = tet_slots(t);
        float e[4];
        int s[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          s[l] = (slots >> (4 * l)) & 7;
          e[l] = s_eps[pbase + point_offset(s[l])];
        }
        float gb[4][NORB];
        float ge[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
          for (int m = 0; m < NORB; ++m) gb[l][m] = 0.0f;
        bool any = false;  // this lane has something to add for tetrahedron t
        if (active && finite4(e[0], e[1], e[2], e[3])) {
          sort4(e, s);
          int jlo, jhi;
          energy_window(e[0], e[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
          bool owned_corner = false;
#pragma unroll
          for (int l = 0; l < 4; ++l) owned_corner = owned_corner || (s_own[pbase + point_offset(s[l])] >= 0);
          if (jlo <= jhi + 2 && owned_corner) {
            const TetSetup cs = tet_setup(e, a.e0, a.V);
            tet_window(cs, a.de, c0, c1, jlo, jhi);
            if (jlo <= jhi) {
              any = true;
              float bb[4][NORB];
#pragma unroll
              for (int l = 0; l < 4; ++l) {
                const int p = pbase + point_offset(s[l]);
#pragma unroll
                for (int m = 0; m < NORB; ++m) bb[l][m] = s_w[p * NORB + m];
              }
              for (int j = jlo; j <= jhi; ++j) {
                const float x = local_x(cs, j, a.de);
                if (!(x > 0.0f && x < cs.e41)) continue;
                const float* Gj = &s_G[(j - c0) * NORB];
                float Gm[NORB];
#pragma unroll
                for (int m = 0; m < NORB; ++m) Gm[m] = Gj[m];
                float sl[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                  float acc = 0.0f;
#pragma unroll
                  for (int m = 0; m < NORB; ++m) acc += Gm[m] * bb[l][m];
                  sl[l] = acc;
                }
                float g[4], Eb[4];
                corner_dos_adjoint(cs, a.V, x, sl, g, Eb);
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                  ge[l] += Eb[l];
#pragma unroll
                  for (int m = 0; m < NORB; ++m) gb[l][m] += Gm[m] * g[l];
                }
              }
            }
          }
        }
        // Four rounds, one per static corner of tetrahedron t: for a fixed corner slot the target
        // points of different lanes are distinct, so plain read-modify-writes do not race.
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int slot = (slots >> (4 * q)) & 7;
          // sorted position of this corner
          const int i = (s[0] == slot) ? 0 : (s[1] == slot) ? 1 : (s[2] == slot) ? 2 : 3;
          __syncthreads();
          if (any) {
            float* dst = &s_pt[(pbase + point_offset(slot)) * (NORB + 1)];
            float v = (i == 0) ? ge[0] : (i == 1) ? ge[1] : (i == 2) ? ge[2] : ge[3];
            dst[0] += v;
#pragma unroll
            for (int m = 0; m < NORB; ++m) {
              v = (i == 0) ? gb[0][m] : (i == 1) ? gb[1][m] : (i == 2) ? gb[2][m] : gb[3][m];
              dst[1 + m] += v;
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // Write the owned points (coalesced along axis 3). With periodic wrap on a short axis one k-point
  // can appear at several staged positions; their partial sums are added here.
  for (int q = tid; q < NOWN; q += NT) {
    const int d3 = q % OZ, d2 = (q / OZ) % OY, d1 = q / (OZ * OY);
    if (d1 >= P1.own || d2 >= P2.own || d3 >= P3.own) continue;
    float ge = 0.0f;
    float gw[NORB];
#pragma unroll
    for (int m = 0; m < NORB; ++m) gw[m] = 0.0f;
    // staged copies of owned point (x0+d1, y0+d2, z0+d3): local index i_a with (start_a + i_a) % n_a
    // equal to its coordinate, i_a in [0, cnt_a]
    for (int i1 = 0; i1 <= P1.cnt; ++i1) {
      if (wrap_pos(P1.start + i1, a.n1) != P1.x0 + d1) continue;
      for (int i2 = 0; i2 <= P2.cnt; ++i2) {
        if (wrap_pos(P2.start + i2, a.n2) != P2.x0 + d2) continue;
        for (int i3 = 0; i3 <= P3.cnt; ++i3) {
          if (wrap_pos(P3.start + i3, a.n3) != P3.x0 + d3) continue;
          const float* src = &s_pt[((i1 * SY + i2) * SZ + i3) * (NORB + 1)];
          ge += src[0];
#pragma unroll
          for (int m = 0; m < NORB; ++m) gw[m] += src[1 + m];
        }
      }
    }
    const int64_t k = ((int64_t)(P1.x0 + d1) * a.n2 + (P2.x0 + d2)) * a.n3 + (P3.x0 + d3);
    if (a.grad_eps) a.grad_eps[(int64_t)band * nk + k] = ge;
    if (a.grad_w) {
#pragma unroll
      for (int m = 0; m < NORB; ++m) a.grad_w[((int64_t)band * NORB + m) * nk + k] = gw[m];
    }
  }
}

template <int NORB>
hipError_t launch_bwd(const BwdArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(dos_backward_kernel<NORB>, dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t backward_f32(const tetra_desc& d, const float* eps, const float* w, const float* G, float* grad_eps,
                        float* grad_w, hipStream_t s) {
  BwdArgs a;
  a.eps = eps;
  a.w = w;
  a.G = G;
  a.grad_eps = grad_eps;
  a.grad_w = grad_w;
  a.n1 = d.n1;
  a.n2 = d.n2;
  a.n3 = d.n3;
  a.ne = d.ne;
  a.e0 = d.e0;
  a.de = d.de;
  a.inv_de = 1.0f / d.de;
  a.V = (float)(1.0 / (24.0 * (double)d.n1 * d.n2 * d.n3));
  a.t1 = (d.n1 + OX - 1) / OX;
  a.t2 = (d.n2 + OY - 1) / OY;
  a.t3 = (d.n3 + OZ - 1) / OZ;
  a.ntiles = a.t1 * a.t2 * a.t3;
  a.nunits = a.ntiles * d.nb;
  a.per_xcd = (a.nunits + NXCD - 1) / NXCD;
  const int grid = a.per_xcd * NXCD;
  switch (d.norb) {
#define TETRA_CASE(N) \
  case N:             \
    return launch_bwd<N>(a, grid, s);
    TETRA_CASE(1) TETRA_CASE(2) TETRA_CASE(3) TETRA_CASE(4) TETRA_CASE(5) TETRA_CASE(6) TETRA_CASE(7)
    TETRA_CASE(8) TETRA_CASE(9) TETRA_CASE(10) TETRA_CASE(11) TETRA_CASE(12) TETRA_CASE(13)
    TETRA_CASE(14) TETRA_CASE(15) TETRA_CASE(16)
#undef TETRA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace tetra
