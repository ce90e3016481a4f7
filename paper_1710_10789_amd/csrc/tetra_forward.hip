// Forward kernel: orbital-resolved tetrahedron DOS on gfx950.
//
// Sum of eq. (tetracontriborbitalresolved) over the tetrahedra and bands of a periodic k-grid
// (eq. tetmethoorbitalresolved, Guterding & Jeschke, arXiv:1710.10789, Sec. II.C), with the
// tetrahedra of Table I.
//
// Work decomposition (differs from the paper's Sec. III.B on purpose; see the design notes):
//  * one workgroup per (tile of TX x TY x TZ cubes, band); one lane per cube, looping over the six
//    tetrahedra of Table I. Cube corner indices are computed from the lane's coordinates (no index
//    table), and the (TX+1)(TY+1)(TZ+1) grid points of the tile are staged once in LDS (energies and
//    orbital weights), so each k-point is read from HBM about once per band;
//  * per (tetrahedron, band): a five-comparator sort of the corner energies, then a loop over only
//    the energy-grid indices inside (E1, E4) -- the paper's kernel visits every energy;
//  * per (tetrahedron, band, energy): the four corner weights (tetra_device.h) contracted with the
//    four corners' orbital weights, added to an LDS histogram that covers only the tile-band's
//    energy range;
//  * the LDS histogram holds 64-bit fixed-point integers: LDS float atomics are an order of
//    magnitude slower than integer ones on gfx950. Every contribution is non-negative (a corner
//    weight is the section integral of a barycentric coordinate) and a tetrahedron's point DOS never
//    exceeds 3 V_T/(V_G E41), so with bmax = max |b| of the tile, a per-workgroup bound
//    B = sum 12 V bmax / E41 over the tetrahedra with a non-empty window bounds every bin's |sum| and
//    fixes a power-of-two scale S with B*S <= 2^62 (two's complement, so signed weights work too).
//    The in-LDS sum is then exact and independent of the order of the atomics; the only rounding
//    left is that of each FP32 contribution;
//  * one global float atomic per touched (energy, orbital) bin when the workgroup finishes.
// Workgroups are assigned so that each XCD (eight per MI355X, each with its own L2) works through a
// contiguous range of tiles of the same band, keeping shared halo points in one L2.

#include "tetra_device.h"
#include "tetra_internal.h"

namespace tetra {

namespace {

constexpr int TX = 4, TY = 4, TZ = 16;  // cubes per tile along grid axes 1, 2, 3
constexpr int NT = TX * TY * TZ;        // one lane per cube
constexpr int PX = TX + 1, PY = TY + 1, PZ = TZ + 1;
constexpr int NP = PX * PY * PZ;  // staged grid points (cube corners of the tile)
constexpr int HCAP = 2048;        // LDS histogram capacity in 64-bit words
constexpr int NXCD = 8;

struct FwdArgs {
  const float* eps;
  const float* w;
  float* dos;
  int n1, n2, n3, ne;
  float e0, de, inv_de, V;
  int t1, t2, t3;  // tiles along each axis
  int ntiles, nunits, per_xcd;
};

// Global float add without a compare-and-swap loop (device memory from hipMalloc).
__device__ __forceinline__ void atomic_add_global(float* p, float v) { unsafeAtomicAdd(p, v); }

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
__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int NORB>
__global__ __launch_bounds__(NT) void dos_forward_kernel(FwdArgs a) {
  constexpr int LC = ((HCAP / NORB) - 1) & ~1;  // energies per histogram pass (even)
  __shared__ float s_eps[NP];
  __shared__ float s_w[NP * NORB];
  __shared__ unsigned long long s_hist[HCAP];
  __shared__ float s_red[3 * (NT / 64)];

  // XCD-aware mapping: hardware dispatches block b to XCD b % 8; give each XCD a contiguous range.
  const int b = blockIdx.x;
  const int unit = (b % NXCD) * a.per_xcd + b / NXCD;
  if (unit >= a.nunits) return;
  const int band = unit / a.ntiles;
  const int tile = unit - band * a.ntiles;
  const int tz = tile % a.t3;
  const int ty = (tile / a.t3) % a.t2;
  const int tx = tile / (a.t3 * a.t2);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int tid = threadIdx.x;
  const int64_t nk = (int64_t)a.n1 * a.n2 * a.n3;
  const float* eps_n = a.eps + (int64_t)band * nk;
  const float* w_n = a.w + (int64_t)band * NORB * nk;

  // Stage the tile's grid points (periodic wrap) and find their energy range.
  float lmin = __builtin_huge_valf(), lmax = -__builtin_huge_valf(), lbmax = 0.0f;
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
    for (int m = 0; m < NORB; ++m) {
      const float b = w_n[(int64_t)m * nk + k];
      s_w[p * NORB + m] = b;
      lbmax = fmaxf(lbmax, fabsf(b));
    }
  }
  lmin = wave_min(lmin);
  lmax = wave_max(lmax);
  lbmax = wave_max(lbmax);
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = lmin;
    s_red[(NT / 64) + (tid >> 6)] = lmax;
    s_red[2 * (NT / 64) + (tid >> 6)] = lbmax;
  }
  __syncthreads();
  float emin = s_red[0], emax = s_red[NT / 64], bmax = s_red[2 * (NT / 64)];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    emin = fminf(emin, s_red[i]);
    emax = fmaxf(emax, s_red[NT / 64 + i]);
    bmax = fmaxf(bmax, s_red[2 * (NT / 64) + i]);
  }
  if (!(emin <= emax)) return;  // no finite energy in this tile-band (uniform across the block)
  int J0, J1;
  range_window(emin, emax, a.e0, a.inv_de, a.ne, J0, J1);

  // This lane's cube; corner slot s sits at LDS point pbase + point_offset(s).
  const int cz = tid % TZ, cy = (tid / TZ) % TY, cx = tid / (TZ * TY);
  const bool valid = (x0 + cx < a.n1) && (y0 + cy < a.n2) && (z0 + cz < a.n3);
  const int pbase = (cx * PY + cy) * PZ + cz;
  auto point_offset = [](int s) { return (s & 1) * (PY * PZ) + ((s >> 1) & 1) * PZ + (s >> 2); };

  // Bound on any bin's sum: sum over tetrahedra with a possibly non-empty window of 12 V bmax / E41.
  float bound = 0.0f;
  if (valid) {
#pragma unroll 1
    for (int t = 0; t < 6; ++t) {
      const uint32_t slots = tet_slots(t);
      float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
      bool fin = true;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const float e = s_eps[pbase + point_offset((slots >> (4 * l)) & 7)];
        fin = fin && __builtin_isfinite(e);
        lo = fminf(lo, e);
        hi = fmaxf(hi, e);
      }
      if (!fin || !(hi > lo)) continue;
      int jlo, jhi;
      energy_window(lo, hi, a.e0, a.inv_de, J0, J1, jlo, jhi);
      if (jlo > jhi + 2) continue;
      bound += 12.0f * a.V * bmax / (hi - lo);
    }
  }
  bound = wave_sum(fminf(bound, 1.0e37f));
  __syncthreads();  // every lane has read s_red
  if ((tid & 63) == 0) s_red[tid >> 6] = bound;
  __syncthreads();
  float B = 0.0f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) B += s_red[i];
  if (!(B > 0.0f)) return;  // nothing to add (uniform across the block)
  int bexp;
  frexpf(fminf(B, 3.0e38f), &bexp);  // B <= 2^bexp
  const int sexp = min(62 - bexp, 126);
  const float S = ldexpf(1.0f, sexp);        // B * S <= 2^62
  const double inv_S = ldexp(1.0, -sexp);

  for (int c0 = J0; c0 <= J1; c0 += LC) {
    const int c1 = min(c0 + LC - 1, J1);
    const int L = c1 - c0 + 1;
    const int LP = L | 1;  // odd row pitch: the flush reads across orbitals without bank conflicts
    for (int q = tid; q < NORB * LP; q += NT) s_hist[q] = 0ull;
    __syncthreads();
    if (valid) {
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
        if (!finite4(e[0], e[1], e[2], e[3])) continue;
        sort4(e, s);
        int jlo, jhi;
        energy_window(e[0], e[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
        if (jlo > jhi + 2) continue;  // empty even after moving both ends by one
        const TetSetup cs = tet_setup(e, a.e0, a.V);
        tet_window(cs, a.de, c0, c1, jlo, jhi);
        if (jlo > jhi) continue;
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
          float g[4];
          corner_dos(cs, x, g);
          unsigned long long* h = &s_hist[j - c0];
#pragma unroll
          for (int m = 0; m < NORB; ++m) {
            const float v = g[0] * bb[0][m] + g[1] * bb[1][m] + g[2] * bb[2][m] + g[3] * bb[3][m];
            atomicAdd(&h[m * LP], (unsigned long long)__float2ll_rn(v * S));
          }
        }
      }
    }
    __syncthreads();
    for (int q = tid; q < L * NORB; q += NT) {
      const int r = q / NORB, m = q - r * NORB;
      const unsigned long long qv = s_hist[m * LP + r];
      if (qv != 0ull) atomic_add_global(&a.dos[(int64_t)(c0 + r) * NORB + m], (float)((double)(long long)qv * inv_S));
    }
    __syncthreads();
  }
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

template <int NORB>
hipError_t launch_fwd(const FwdArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(dos_forward_kernel<NORB>, dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t forward_f32(const tetra_desc& d, const float* eps, const float* w, float* dos, hipStream_t s) {
  FwdArgs a;
  a.eps = eps;
  a.w = w;
  a.dos = dos;
  a.n1 = d.n1;
  a.n2 = d.n2;
  a.n3 = d.n3;
  a.ne = d.ne;
  a.e0 = d.e0;
  a.de = d.de;
  a.inv_de = 1.0f / d.de;
  a.V = (float)(1.0 / (24.0 * (double)d.n1 * d.n2 * d.n3));  // V_T / (4 V_G)
  a.t1 = (d.n1 + TX - 1) / TX;
  a.t2 = (d.n2 + TY - 1) / TY;
  a.t3 = (d.n3 + TZ - 1) / TZ;
  a.ntiles = a.t1 * a.t2 * a.t3;
  a.nunits = a.ntiles * d.nb;
  a.per_xcd = (a.nunits + NXCD - 1) / NXCD;
  const int grid = a.per_xcd * NXCD;
  hipError_t e = fill_zero(dos, (int64_t)d.ne * d.norb, s);
  if (e != hipSuccess) return e;
  switch (d.norb) {
#define TETRA_CASE(N) \
  case N:             \
    return launch_fwd<N>(a, grid, s);
    TETRA_CASE(1) TETRA_CASE(2) TETRA_CASE(3) TETRA_CASE(4) TETRA_CASE(5) TETRA_CASE(6) TETRA_CASE(7)
    TETRA_CASE(8) TETRA_CASE(9) TETRA_CASE(10) TETRA_CASE(11) TETRA_CASE(12) TETRA_CASE(13)
    TETRA_CASE(14) TETRA_CASE(15) TETRA_CASE(16)
#undef TETRA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace tetra
