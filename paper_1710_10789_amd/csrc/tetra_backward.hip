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
// Work decomposition: one workgroup per (tile of TX x TY x TZ cubes, band), one lane per cube, every
// cube processed exactly once (as in the forward kernel). There are no LDS atomics (LDS float atomics
// are slow on gfx950): all lanes work on the same tetrahedron index t at a time, so for each of t's
// four corners the map cube -> corner point is injective across lanes, and four barrier-separated
// rounds add each lane's per-corner sums into LDS point totals with plain read-modify-writes.
// A grid point whose eight cubes all belong to the tile is complete in LDS and written with a plain
// store. A point on the tile's boundary gets its partial sums one of two ways:
//  * two-phase (a workspace, grid sides multiples of the tile's, more than one tile per axis): the
//    tile stores them in its face slots (tetra_faces.h) with plain stores, and a gather pass adds the
//    2 to 8 partials of every boundary grid point in a fixed order and writes the outputs. Nothing
//    is zero-filled, no atomics, and the result does not depend on the order workgroups run in;
//  * otherwise one global float atomic per value into zero-filled outputs. On an axis short enough
//    for the periodic wrap to repeat a point inside one tile, every point goes through the atomics,
//    which sums the repeats.

#include <algorithm>
#include <type_traits>

#include "tetra_device.h"
#include "tetra_faces.h"
#include "tetra_internal.h"
#include "tetra_weights.h"

namespace tetra {

namespace {

constexpr int NT = kTileCubes;      // one lane per cube of the tile
constexpr int NPMAX = kTilePointsMax;  // grid points (cube corners) of the largest tile shape
constexpr int HCAP = 4096;        // LDS capacity for the rows of G, in floats
constexpr int NXCD = 8;

struct BwdArgs {
  const float* eps;
  const void* w;        // float, _Float16 or float2 (complex amplitude) [nb][norb][nk]
  const float* w_scale;  // per-band scale of _Float16 weights
  const float* G;
  float* grad_eps;
  float* grad_w;  // [nb][norb][nk], or [nb][norb][nk][2] (re, im) for complex amplitudes
  float* part;    // two-phase output: [unit][nface][1 + norb] face partial sums, or null
  int nface;      // face points per tile
  int wtype;
  int n1, n2, n3, ne;
  float e0, de, inv_de, V;
  int TX, TY, TZ;  // cubes per tile along grid axes 1, 2, 3 (TX*TY*TZ = NT)
  int t1, t2, t3;
  int ntiles, nunits, per_xcd;
};

__device__ __forceinline__ int wrap(int v, int n) {
  if (v >= n) v -= n;
  if (v >= n) v %= n;
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

template <int NORB, typename WT>
__global__ __launch_bounds__(NT) void dos_backward_kernel(BwdArgs a) {
  constexpr int LC = HCAP / NORB;
  __shared__ float s_eps[NPMAX];
  __shared__ float s_w[NPMAX * NORB];
  __shared__ float s_pt[NPMAX * (NORB + 1)];  // per tile point: dL/deps, then dL/db[0..NORB)
  __shared__ float s_G[HCAP];
  __shared__ float s_red[2 * (NT / 64)];

  const int b = blockIdx.x;
  const int unit = (b % NXCD) * a.per_xcd + b / NXCD;
  if (unit >= a.nunits) return;
  const int TX = a.TX, TY = a.TY, TZ = a.TZ;
  const int PY = TY + 1, PZ = TZ + 1;
  const int NP = (TX + 1) * PY * PZ;
  const int band = unit / a.ntiles;
  const int tile = unit - band * a.ntiles;
  const int tz = tile % a.t3;
  const int ty = (tile / a.t3) % a.t2;
  const int tx = tile / (a.t3 * a.t2);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int tid = threadIdx.x;
  const int64_t nk = (int64_t)a.n1 * a.n2 * a.n3;
  const float* eps_n = a.eps + (int64_t)band * nk;
  const WT* w_n = static_cast<const WT*>(a.w) + (int64_t)band * NORB * nk;
  const float wscale = a.w_scale ? a.w_scale[band] : 1.0f;

  for (int q = tid; q < NP * (NORB + 1); q += NT) s_pt[q] = 0.0f;
  float lmin = __builtin_huge_valf(), lmax = -__builtin_huge_valf();
  for (int p = tid; p < NP; p += NT) {
    const int pz = p % PZ, py = (p / PZ) % PY, px = p / (PZ * PY);
    const int64_t k = ((int64_t)wrap(x0 + px, a.n1) * a.n2 + wrap(y0 + py, a.n2)) * a.n3 + wrap(z0 + pz, a.n3);
    const float e = eps_n[k];
    s_eps[p] = e;
    if (__builtin_isfinite(e)) {
      lmin = fminf(lmin, e);
      lmax = fmaxf(lmax, e);
    }
#pragma unroll
    for (int m = 0; m < NORB; ++m) s_w[p * NORB + m] = weight_value(w_n[(int64_t)m * nk + k], wscale);
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
  // No finite energy: nothing to add, but the zero sums are still written (the two-phase output
  // does not zero-fill).
  int J0 = 0, J1 = -1;
  if (emin <= emax) range_window(emin, emax, a.e0, a.inv_de, a.ne, J0, J1);

  const int cz = tid % TZ, cy = (tid / TZ) % TY, cx = tid / (TZ * TY);
  const bool active = (x0 + cx < a.n1) && (y0 + cy < a.n2) && (z0 + cz < a.n3);
  const int pbase = (cx * PY + cy) * PZ + cz;
  auto point_offset = [PY, PZ](int s) { return (s & 1) * (PY * PZ) + ((s >> 1) & 1) * PZ + (s >> 2); };

  // Corners 2 and 5 of the cube (its body diagonal) belong to all six tetrahedra of Table I: their sums
  // stay in registers over every tetrahedron and energy pass and go to LDS once at the end, so each
  // tetrahedron needs only two rounds (its other two corners): 2 % faster at norb = 8. It costs 2 to
  // 45 VGPRs; orbital counts where that would lower the waves per SIMD keep four rounds.
  constexpr bool DIAG = !(NORB == 2 || NORB == 5 || NORB == 9 || NORB == 10 || NORB == 16);
  float diag2[NORB + 1], diag5[NORB + 1];
#pragma unroll
  for (int v = 0; v <= NORB; ++v) diag2[v] = diag5[v] = 0.0f;
  for (int c0 = J0; c0 <= J1; c0 += LC) {
    const int c1 = min(c0 + LC - 1, J1);
    const int L = c1 - c0 + 1;
    for (int q = tid; q < L * NORB; q += NT) s_G[q] = a.G[(int64_t)c0 * NORB + q];
    __syncthreads();
    {
#pragma unroll 1
      for (int t = 0; t < 6; ++t) {
        const uint32_t slots = tet_slots(t);
        float e[4];
        int pt[4];  // LDS point of each corner, carried through the sort
        bool sw[5] = {false, false, false, false, false};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          pt[l] = pbase + point_offset((slots >> (4 * l)) & 7);
          e[l] = s_eps[pt[l]];
        }
        float gb[4][NORB];
        float ge[4][1] = {{0.0f}, {0.0f}, {0.0f}, {0.0f}};
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
          for (int m = 0; m < NORB; ++m) gb[l][m] = 0.0f;
        // Straight-line set-up for every lane (a lane without work gets an empty window), so that
        // the accumulators above have one definition and no copies on merging paths.
        const bool fin = active && finite4(e[0], e[1], e[2], e[3]);
        sort4(e, pt, sw);
        int jlo, jhi;
        energy_window(e[0], e[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
        const TetSetup cs = tet_setup(e, a.e0, a.V);
        tet_window(cs, a.de, c0, c1, jlo, jhi);
        if (!fin) {
          jlo = c0;
          jhi = c0 - 1;
        }
        const bool any = jlo <= jhi;  // this lane has something to add for tetrahedron t
        {
          {
            {
              // One loop per energy case (each case has its own polynomial variable and power sums).
              int jA, jB;
              case_split(cs, a.de, a.inv_de, jlo, jhi, jA, jB);
              if (!any) jA = jB = jhi;
              // Every corner weight is a cubic in the range's local variable t, g_l(t) = sum_k c_lk t^k,
              // so over a case range both the weight gradient sum_j G[j][m] g_l(t_j) and the moments
              // sum_j s_l(t_j) t_j^k of the energy gradient (s_l = sum_m G b_l) are contractions of the
              // power sums H_k[m] = sum_j G[j][m] t_j^k: the loop over energies accumulates only those.
              auto rowG = [&](int j, float Gm[NORB]) {
                const float* Gj = &s_G[(j - c0) * NORB];
#pragma unroll
                for (int m = 0; m < NORB; ++m) Gm[m] = Gj[m];
              };
              const float* const brow[4] = {&s_w[pt[0] * NORB], &s_w[pt[1] * NORB], &s_w[pt[2] * NORB],
                                            &s_w[pt[3] * NORB]};
              auto add_eb = [&](const float Eb[4]) {
#pragma unroll
                for (int l = 0; l < 4; ++l) ge[l][0] += Eb[l];
              };
              if (jA >= jlo) {  // first case, t = x: powers 1..3
                float H[3][NORB];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                  for (int m = 0; m < NORB; ++m) H[k][m] = 0.0f;
                for (int j = jlo; j <= jA; ++j) {
                  float Gm[NORB];
                  rowG(j, Gm);
                  const float x = local_x(cs, j, a.de), x2 = x * x, x3 = x2 * x;
#pragma unroll
                  for (int m = 0; m < NORB; ++m) {
                    H[0][m] = __builtin_fmaf(Gm[m], x, H[0][m]);
                    H[1][m] = __builtin_fmaf(Gm[m], x2, H[1][m]);
                    H[2][m] = __builtin_fmaf(Gm[m], x3, H[2][m]);
                  }
                }
                float Eb[4];
                adjoint_range_A<NORB>(cs, a.V, brow, H, gb, Eb);
                add_eb(Eb);
              }
              if (jB > jA) {  // middle case, t = z: powers 0..3
                float H[4][NORB];
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                  for (int m = 0; m < NORB; ++m) H[k][m] = 0.0f;
                for (int j = jA + 1; j <= jB; ++j) {
                  float Gm[NORB];
                  rowG(j, Gm);
                  const float z = local_z(cs, j, a.de), z2 = z * z, z3 = z2 * z;
#pragma unroll
                  for (int m = 0; m < NORB; ++m) {
                    H[0][m] += Gm[m];
                    H[1][m] = __builtin_fmaf(Gm[m], z, H[1][m]);
                    H[2][m] = __builtin_fmaf(Gm[m], z2, H[2][m]);
                    H[3][m] = __builtin_fmaf(Gm[m], z3, H[3][m]);
                  }
                }
                float Eb[4];
                adjoint_range_B<NORB>(cs, a.V, brow, H, gb, Eb);
                add_eb(Eb);
              }
              if (jhi > jB) {  // third case, t = y: powers 1..3
                float H[3][NORB];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                  for (int m = 0; m < NORB; ++m) H[k][m] = 0.0f;
                for (int j = jB + 1; j <= jhi; ++j) {
                  float Gm[NORB];
                  rowG(j, Gm);
                  const float y = local_y(cs, j, a.de), y2 = y * y, y3 = y2 * y;
#pragma unroll
                  for (int m = 0; m < NORB; ++m) {
                    H[0][m] = __builtin_fmaf(Gm[m], y, H[0][m]);
                    H[1][m] = __builtin_fmaf(Gm[m], y2, H[1][m]);
                    H[2][m] = __builtin_fmaf(Gm[m], y3, H[2][m]);
                  }
                }
                float Eb[4];
                adjoint_range_C<NORB>(cs, a.V, brow, H, gb, Eb);
                add_eb(Eb);
              }
            }
          }
        }
        // Back to the corner order of Table I, then four rounds, one per corner of tetrahedron t: for a
        // fixed corner slot the target points of different lanes are distinct, so plain
        // read-modify-writes do not race.
        unsort_rows(sw, ge);
        unsort_rows(sw, gb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int corner = (slots >> (4 * q)) & 7;  // uniform: t is the same for every lane
          if (DIAG && corner == 2) {
            diag2[0] += ge[q][0];
#pragma unroll
            for (int m = 0; m < NORB; ++m) diag2[1 + m] += gb[q][m];
            continue;
          }
          if (DIAG && corner == 5) {
            diag5[0] += ge[q][0];
#pragma unroll
            for (int m = 0; m < NORB; ++m) diag5[1 + m] += gb[q][m];
            continue;
          }
          __syncthreads();
          if (any) {
            float* dst = &s_pt[(pbase + point_offset(corner)) * (NORB + 1)];
            dst[0] += ge[q][0];
#pragma unroll
            for (int m = 0; m < NORB; ++m) dst[1 + m] += gb[q][m];
          }
        }
      }
    }
    __syncthreads();
  }
  if constexpr (DIAG) {
    // the two diagonal corners, one round each (a lane's sums are zero where it had nothing to add)
    __syncthreads();
    if (active) {
      float* dst = &s_pt[(pbase + point_offset(2)) * (NORB + 1)];
#pragma unroll
      for (int v = 0; v <= NORB; ++v) dst[v] += diag2[v];
    }
    __syncthreads();
    if (active) {
      float* dst = &s_pt[(pbase + point_offset(5)) * (NORB + 1)];
#pragma unroll
      for (int v = 0; v <= NORB; ++v) dst[v] += diag5[v];
    }
    __syncthreads();
  }

  // Interior points are complete: plain stores. Boundary points: face slots (two-phase), or one
  // global atomic per non-zero value.
  const bool no_repeat = a.n1 > TX && a.n2 > TY && a.n3 > TZ;
  for (int p = tid; p < NP; p += NT) {
    const int pz = p % PZ, py = (p / PZ) % PY, px = p / (PZ * PY);
    const bool interior = no_repeat && px >= 1 && px < TX && py >= 1 && py < TY && pz >= 1 && pz < TZ &&
                          x0 + px < a.n1 && y0 + py < a.n2 && z0 + pz < a.n3;
    if (a.part && !interior) {
      float* dst = a.part + ((int64_t)unit * a.nface + face_index(px, py, pz, TX, TY, TZ)) * (NORB + 1);
      const float* src = &s_pt[p * (NORB + 1)];
#pragma unroll
      for (int v = 0; v <= NORB; ++v) dst[v] = src[v];
      continue;
    }
    const int64_t k = ((int64_t)wrap(x0 + px, a.n1) * a.n2 + wrap(y0 + py, a.n2)) * a.n3 + wrap(z0 + pz, a.n3);
    const float* src = &s_pt[p * (NORB + 1)];
    if (a.grad_eps) {
      float* dst = &a.grad_eps[(int64_t)band * nk + k];
      if (interior) *dst = src[0];
      else if (src[0] != 0.0f) unsafeAtomicAdd(dst, src[0]);
    }
    if (a.grad_w) {
#pragma unroll
      for (int m = 0; m < NORB; ++m) {
        if constexpr (std::is_same<WT, float2>::value) {
          // b = re^2 + im^2: dL/d(re, im) = 2 (re, im) dL/db, linear in each partial sum
          const float2 amp = w_n[(int64_t)m * nk + k];
          const float g2 = 2.0f * src[1 + m];
          float* dst = &a.grad_w[2 * (((int64_t)band * NORB + m) * nk + k)];
          if (interior) {
            *reinterpret_cast<float2*>(dst) = make_float2(g2 * amp.x, g2 * amp.y);
          } else if (g2 != 0.0f) {
            unsafeAtomicAdd(dst, g2 * amp.x);
            unsafeAtomicAdd(dst + 1, g2 * amp.y);
          }
        } else {
          float* dst = &a.grad_w[((int64_t)band * NORB + m) * nk + k];
          if (interior) *dst = src[1 + m];
          else if (src[1 + m] != 0.0f) unsafeAtomicAdd(dst, src[1 + m]);
        }
      }
    }
  }
}

// Second phase of the two-phase output: every (band, grid point) not complete in its own tile adds the
// face partials of the tiles holding it (face_tiles on each axis, a fixed order) and writes the
// outputs.
struct GatherArgs {
  const void* w;  // complex amplitudes for the chain to (re, im); unused otherwise
  const float* part;
  float* grad_eps;
  float* grad_w;
  int n1, n2, n3, nb;
  int TX, TY, TZ;
  int t1, t2, t3, ntiles, nface;
};

template <int NORB, typename WT>
__global__ __launch_bounds__(256) void bwd_gather_kernel(GatherArgs g) {
  const int64_t nk = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t total = nk * g.nb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int band = (int)(i / nk);
    const int64_t k = i - (int64_t)band * nk;
    const int z = (int)(k % g.n3), y = (int)((k / g.n3) % g.n2), x = (int)(k / ((int64_t)g.n2 * g.n3));
    int ta[2], pa[2], tb[2], pb[2], tc[2], pc[2];
    const int na = face_tiles(x, g.TX, g.t1, ta, pa);
    const int nbt = face_tiles(y, g.TY, g.t2, tb, pb);
    const int nc = face_tiles(z, g.TZ, g.t3, tc, pc);
    if (pa[0] && pb[0] && pc[0]) continue;  // complete in its own tile, stored by the adjoint kernel
    float acc[NORB + 1];
#pragma unroll
    for (int v = 0; v <= NORB; ++v) acc[v] = 0.0f;
    for (int ia = 0; ia < na; ++ia)
      for (int ib = 0; ib < nbt; ++ib)
        for (int ic = 0; ic < nc; ++ic) {
          const int tile = (ta[ia] * g.t2 + tb[ib]) * g.t3 + tc[ic];
          const float* src = g.part + (((int64_t)band * g.ntiles + tile) * g.nface +
                                       face_index(pa[ia], pb[ib], pc[ic], g.TX, g.TY, g.TZ)) * (NORB + 1);
#pragma unroll
          for (int v = 0; v <= NORB; ++v) acc[v] += src[v];
        }
    if (g.grad_eps) g.grad_eps[(int64_t)band * nk + k] = acc[0];
    if (g.grad_w) {
#pragma unroll
      for (int m = 0; m < NORB; ++m) {
        const int64_t idx = ((int64_t)band * NORB + m) * nk + k;
        if constexpr (std::is_same<WT, float2>::value) {
          const float2 amp = static_cast<const float2*>(g.w)[idx];
          const float g2 = 2.0f * acc[1 + m];
          *reinterpret_cast<float2*>(&g.grad_w[2 * idx]) = make_float2(g2 * amp.x, g2 * amp.y);
        } else {
          g.grad_w[idx] = acc[1 + m];
        }
      }
    }
  }
}

template <int NORB>
hipError_t launch_gather(const GatherArgs& g, int wtype, hipStream_t s) {
  const int64_t total = (int64_t)g.n1 * g.n2 * g.n3 * g.nb;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  if (wtype == TETRA_W_C32)
    hipLaunchKernelGGL((bwd_gather_kernel<NORB, float2>), dim3(blocks), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((bwd_gather_kernel<NORB, float>), dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

template <int NORB>
hipError_t launch_bwd(const BwdArgs& a, int grid, hipStream_t s) {
  if (a.wtype == TETRA_W_F16)
    hipLaunchKernelGGL((dos_backward_kernel<NORB, _Float16>), dim3(grid), dim3(NT), 0, s, a);
  else if (a.wtype == TETRA_W_C32)
    hipLaunchKernelGGL((dos_backward_kernel<NORB, float2>), dim3(grid), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((dos_backward_kernel<NORB, float>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

size_t backward_workspace_bytes(const tetra_desc& d, int shape) {
  const TileShape sh = tile_shape(shape);
  if (d.n1 % sh.x || d.n2 % sh.y || d.n3 % sh.z || d.n1 <= sh.x || d.n2 <= sh.y || d.n3 <= sh.z) return 0;
  const size_t units = (size_t)(d.n1 / sh.x) * (d.n2 / sh.y) * (d.n3 / sh.z) * d.nb;
  return units * (size_t)(d.norb + 1) * face_count(sh.x, sh.y, sh.z) * sizeof(float);
}

hipError_t backward(const tetra_desc& d, const float* eps, const void* w, int wtype, const float* w_scale,
                    const float* G, float* grad_eps, float* grad_w, int shape, void* workspace, hipStream_t s) {
  BwdArgs a;
  a.wtype = wtype;
  a.eps = eps;
  a.w = w;
  a.w_scale = w_scale;
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
  const TileShape sh = tile_shape(shape);
  a.TX = sh.x;
  a.TY = sh.y;
  a.TZ = sh.z;
  a.t1 = (d.n1 + sh.x - 1) / sh.x;
  a.t2 = (d.n2 + sh.y - 1) / sh.y;
  a.t3 = (d.n3 + sh.z - 1) / sh.z;
  a.ntiles = a.t1 * a.t2 * a.t3;
  a.nunits = a.ntiles * d.nb;
  a.per_xcd = (a.nunits + NXCD - 1) / NXCD;
  const int grid = a.per_xcd * NXCD;
  const int64_t nk = (int64_t)d.n1 * d.n2 * d.n3;
  const bool two_phase = workspace && backward_workspace_bytes(d, shape) > 0;
  a.part = two_phase ? static_cast<float*>(workspace) : nullptr;
  a.nface = face_count(sh.x, sh.y, sh.z);
  GatherArgs g;
  g.w = w;
  g.part = a.part;
  g.grad_eps = grad_eps;
  g.grad_w = grad_w;
  g.n1 = d.n1;
  g.n2 = d.n2;
  g.n3 = d.n3;
  g.nb = d.nb;
  g.TX = sh.x;
  g.TY = sh.y;
  g.TZ = sh.z;
  g.t1 = a.t1;
  g.t2 = a.t2;
  g.t3 = a.t3;
  g.ntiles = a.ntiles;
  g.nface = a.nface;
  hipError_t e = hipSuccess;
  if (!two_phase) {
    if (grad_eps) e = fill_zero(grad_eps, nk * d.nb, s);
    if (e == hipSuccess && grad_w) e = fill_zero(grad_w, nk * d.nb * d.norb * (wtype == TETRA_W_C32 ? 2 : 1), s);
    if (e != hipSuccess) return e;
  }
  switch (d.norb) {
#define TETRA_CASE(N)                                \
  case N:                                            \
    e = launch_bwd<N>(a, grid, s);                   \
    if (e == hipSuccess && two_phase) e = launch_gather<N>(g, wtype, s); \
    return e;
    TETRA_CASE(1) TETRA_CASE(2) TETRA_CASE(3) TETRA_CASE(4) TETRA_CASE(5) TETRA_CASE(6) TETRA_CASE(7)
    TETRA_CASE(8) TETRA_CASE(9) TETRA_CASE(10) TETRA_CASE(11) TETRA_CASE(12) TETRA_CASE(13)
    TETRA_CASE(14) TETRA_CASE(15) TETRA_CASE(16)
#undef TETRA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace tetra
