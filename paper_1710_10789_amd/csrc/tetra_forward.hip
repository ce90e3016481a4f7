// Forward kernel: orbital-resolved tetrahedron DOS on gfx950.
//
// Sum of eq. (tetracontriborbitalresolved) over the tetrahedra and bands of a periodic k-grid
// (eq. tetmethoorbitalresolved, Guterding & Jeschke, arXiv:1710.10789, Sec. II.C), with the
// tetrahedra of Table I.
//
// Work decomposition (differs from the paper's Sec. III.B on purpose):
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
//    left is that of each FP32 contribution. When the tile's weights are non-negative and its bound
//    is not dominated by narrow tetrahedra (E41 < 2 de, whose spikes would make B loose), two orbitals
//    share one 64-bit atomic as two 32-bit fields with B*S <= 2^30 (no carry between fields), which
//    halves the LDS atomic traffic;
//  * one global float atomic per touched (energy, orbital) bin when the workgroup finishes.
// Workgroups are assigned so that each XCD (eight per MI355X, each with its own L2) works through a
// contiguous range of tiles of the same band, keeping shared halo points in one L2.

#include <atomic>

#include "tetra_device.h"
#include "tetra_internal.h"
#include "tetra_weights.h"

namespace tetra {

namespace {

constexpr int NT = kTileCubes;      // one lane per cube of the tile
constexpr int NPMAX = kTilePointsMax;  // staged grid points (cube corners) of the largest tile shape
// LDS histogram capacity in 64-bit words, sized so that one more workgroup fits a CU, and the waves
// per SIMD the kernel is held to. Up to 8 orbitals: 25.6 KB of LDS, 6 workgroups, 80 VGPRs (4 %
// faster at 64^3 x 8 x 8 x 1000 than 2048 words at 5 waves; its tile-band energy spans stay within
// 150 bins, one histogram pass). 16 orbitals: 39.7 KB, 4 workgroups, 128 VGPRs (10 % faster at
// 128^3 x 16 x 16 x 2000 than 3 waves).
template <int NORB>
constexpr int fwd_hist_words() { return NORB <= 8 ? 1280 : NORB == 16 ? 1344 : 2048; }
template <int NORB>
constexpr int fwd_waves() { return NORB <= 8 ? 6 : NORB == 16 ? 4 : 1; }
constexpr int NXCD = 8;

struct FwdArgs {
  const float* eps;
  const void* w;        // float, _Float16 or float2 (complex amplitude) [nb][norb][nk]
  const float* w_scale;  // per-band scale of _Float16 weights
  float* dos;
  int* gexp;                 // exact mode: largest bound exponent of any workgroup (atomicMax in mode 1)
  unsigned long long* gacc;  // exact mode: [ne][norb] sums in the common 64-bit fixed point (mode 2)
  int lg_units;              // exact mode: ceil(log2(nunits))
  int wtype;  // TETRA_W_* of w
  int n1, n2, n3, ne;
  float e0, de, inv_de, V;
  int TX, TY, TZ;  // cubes per tile along grid axes 1, 2, 3 (TX*TY*TZ = NT)
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

// Common fixed point of the exact mode: with E the largest bound exponent of any workgroup (each
// workgroup's bins sum to at most 2^E in magnitude) and L = ceil(log2(workgroups)), the total of any
// bin is below 2^(E + L), so the scale 2^(62 - E - L) keeps every partial and total sum of the
// 64-bit two's-complement accumulator in range.
__device__ __forceinline__ int exact_scale_exp(int gexp, int lg_units) { return 62 - gexp - lg_units; }

// One work unit (tile, band) of the forward pass; every lane of the workgroup calls it.
// MODE 0: DOS with per-workgroup scales, flushed with float atomics;
// 1: only the workgroup's bound exponent, into *gexp (atomicMax: independent of the order);
// 2: DOS with per-workgroup scales as in mode 0; each bin's exact per-workgroup sum is rounded once
//    to the common fixed point fixed by *gexp and added to gacc with a 64-bit integer atomic. Both
//    steps are independent of the order in which workgroups run, so the result is bitwise
//    reproducible.
template <int NORB, typename WT, int MODE>
__device__ __forceinline__ void forward_unit(const FwdArgs& a, int unit) {
  constexpr int NPAIR = (NORB + 1) / 2;
  // Histogram rows (one per orbital pair in the packed form, one per orbital in the wide form) have a
  // fixed, odd stride in 64-bit words: the row offsets of a deposit are immediates, and the flush
  // reads across rows without bank conflicts.
  constexpr int HCAP = fwd_hist_words<NORB>();
  constexpr int RSP = (HCAP / NPAIR - 1) | 1, RSW = (HCAP / NORB - 1) | 1;
  __shared__ float s_eps[NPMAX];
  __shared__ float s_w[NPMAX * NORB];
  __shared__ unsigned long long s_hist[HCAP];
  __shared__ float s_red[4 * (NT / 64)];

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

  // Stage the tile's grid points (periodic wrap) and find their energy range.
  float lmin = __builtin_huge_valf(), lmax = -__builtin_huge_valf(), lbmax = 0.0f, lbmin = 0.0f;
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
      const float b = weight_value(w_n[(int64_t)m * nk + k], wscale);
      s_w[p * NORB + m] = b;
      lbmax = fmaxf(lbmax, fabsf(b));
      lbmin = fminf(lbmin, b);
    }
  }
  lmin = wave_min(lmin);
  lmax = wave_max(lmax);
  lbmax = wave_max(lbmax);
  lbmin = wave_min(lbmin);
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = lmin;
    s_red[(NT / 64) + (tid >> 6)] = lmax;
    s_red[2 * (NT / 64) + (tid >> 6)] = lbmax;
    s_red[3 * (NT / 64) + (tid >> 6)] = lbmin;
  }
  __syncthreads();
  float emin = s_red[0], emax = s_red[NT / 64], bmax = s_red[2 * (NT / 64)], bmin = s_red[3 * (NT / 64)];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    emin = fminf(emin, s_red[i]);
    emax = fmaxf(emax, s_red[NT / 64 + i]);
    bmax = fmaxf(bmax, s_red[2 * (NT / 64) + i]);
    bmin = fminf(bmin, s_red[3 * (NT / 64) + i]);
  }
  if (!(emin <= emax)) return;  // no finite energy in this tile-band (uniform across the block)
  int J0, J1;
  range_window(emin, emax, a.e0, a.inv_de, a.ne, J0, J1);

  // This lane's cube; corner slot s sits at LDS point pbase + point_offset(s).
  const int cz = tid % TZ, cy = (tid / TZ) % TY, cx = tid / (TZ * TY);
  const bool valid = (x0 + cx < a.n1) && (y0 + cy < a.n2) && (z0 + cz < a.n3);
  const int pbase = (cx * PY + cy) * PZ + cz;
  auto point_offset = [PY, PZ](int s) { return (s & 1) * (PY * PZ) + ((s >> 1) & 1) * PZ + (s >> 2); };

  // Bound on any bin's sum: sum over tetrahedra with a possibly non-empty window of 12 V bmax / E41.
  float bound = 0.0f, narrow = 0.0f;
  const float c12 = 12.0f * a.V * bmax;
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
      const float term = c12 * rcp(hi - lo);
      bound += term;
      if (hi - lo < 2.0f * a.de) narrow += term;
    }
  }
  bound = wave_sum(fminf(bound, 1.0e37f));
  narrow = wave_sum(fminf(narrow, 1.0e37f));
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
  if (MODE == 1) {
    if (tid == 0) {
      int be;
      frexpf(fminf(B, 3.0e38f), &be);
      atomicMax(a.gexp, be);
    }
    return;
  }
  const bool packed = bmin >= 0.0f && Bn <= 0.5f * B;  // uniform across the block
  const int rows = packed ? NPAIR : NORB;
  const int RS = packed ? RSP : RSW;
  // Copies: lane l adds into copy l % CP of a bin (each bin's copies are adjacent words), so the lanes
  // of neighbouring cubes, which usually hit the same bins at the same time, do not serialise on one
  // LDS address. As many copies (up to eight) as keep the tile-band's energy range in one pass.
  const int span = J1 - J0 + 1;
  const int cpl = span <= (RS >> 3) ? 3 : span <= (RS >> 2) ? 2 : span <= (RS >> 1) ? 1 : 0;  // log2 of the copy count
  const int CP = 1 << cpl;
  const int LC = RS >> cpl;  // bins per pass
  int bexp;
  frexpf(fminf(B, 3.0e38f), &bexp);  // B <= 2^bexp
  const int sexp = min((packed ? 30 : 62) - bexp, 126);
  const float S = ldexpf(1.0f, sexp);  // B * S <= 2^30 (packed) or 2^62
  // exact mode: shift from this workgroup's fixed point to the common one (negative: to the right)
  const int dshift = MODE == 2 ? exact_scale_exp(*a.gexp, a.lg_units) - sexp : 0;
  // Fold the power-of-two scale into the staged weights (exact): every deposit is then an integer-valued
  // float without a per-orbital multiply.
  for (int q = tid; q < NP * NORB; q += NT) s_w[q] *= S;
  __syncthreads();

  for (int c0 = J0; c0 <= J1; c0 += LC) {
    const int c1 = min(c0 + LC - 1, J1);
    const int L = c1 - c0 + 1;
    const int LW = L << cpl;  // words per row in this pass
    // The lane index again, opaque: the addresses derived from it are formed in each pass instead of
    // being kept live (in scratch) over the whole unit. (Not in the exact mode's second pass, whose
    // register allocation it upsets.)
    int tid = threadIdx.x;
    if constexpr (MODE != 2) asm volatile("" : "+v"(tid));
    for (int q = tid; q < rows * LW; q += NT) {
      const int r = q / LW;
      s_hist[r * RS + (q - r * LW)] = 0ull;
    }
    __syncthreads();
    if (valid) {
#pragma unroll 1
      for (int t = 0; t < 6; ++t) {
        const uint32_t slots = tet_slots(t);
        float e[4];
        int pt[4];  // LDS point of each corner, carried through the sort
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          pt[l] = pbase + point_offset((slots >> (4 * l)) & 7);
          e[l] = s_eps[pt[l]];
        }
        if (!finite4(e[0], e[1], e[2], e[3])) continue;
        sort4(e, pt);
        int jlo, jhi;
        energy_window(e[0], e[3], a.e0, a.inv_de, c0, c1, jlo, jhi);
        if (jlo > jhi + 2) continue;  // empty even after moving both ends by one
        const TetSetup cs = tet_setup(e, a.e0, a.V);
        tet_window(cs, a.de, c0, c1, jlo, jhi);
        if (jlo > jhi) continue;
        float bb[4][NORB];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
#pragma unroll
          for (int m = 0; m < NORB; ++m) bb[l][m] = s_w[pt[l] * NORB + m];
        }
        // The window splits into the three energy cases at jA and jB.
        int jA, jB;
        case_split(cs, a.de, a.inv_de, jlo, jhi, jA, jB);
        // Packed: two orbitals per 64-bit word as unsigned 32-bit fields; every term is non-negative
        // (the weights are, and the corner weights are clamped at zero against rounding), so the
        // truncating conversion of 0.5 + v rounds v to the nearest integer (halves up).
        auto deposit = [&](int j, const float g[4]) {
          unsigned long long* h = &s_hist[((j - c0) << cpl) + (tid & (CP - 1))];
          if (packed) {
#pragma unroll
            for (int pr = 0; pr < NPAIR; ++pr) {
              const int m0 = 2 * pr, m1 = 2 * pr + 1;
              float v0 = __builtin_fmaf(g[0], bb[0][m0], 0.5f);
              v0 = __builtin_fmaf(g[1], bb[1][m0], v0);
              v0 = __builtin_fmaf(g[2], bb[2][m0], v0);
              v0 = __builtin_fmaf(g[3], bb[3][m0], v0);
              unsigned long long word = (unsigned long long)(unsigned)v0;
              if (m1 < NORB) {
                float v1 = __builtin_fmaf(g[0], bb[0][m1], 0.5f);
                v1 = __builtin_fmaf(g[1], bb[1][m1], v1);
                v1 = __builtin_fmaf(g[2], bb[2][m1], v1);
                v1 = __builtin_fmaf(g[3], bb[3][m1], v1);
                word |= (unsigned long long)(unsigned)v1 << 32;
              }
              atomicAdd(&h[pr * RSP], word);
            }
          } else {
#pragma unroll
            for (int m = 0; m < NORB; ++m) {
              const float v = g[0] * bb[0][m] + g[1] * bb[1][m] + g[2] * bb[2][m] + g[3] * bb[3][m];
              atomicAdd(&h[m * RSW], (unsigned long long)__float2ll_rn(v));
            }
          }
        };
        // One loop over the whole window: a wavefront runs as long as its longest window instead of
        // the sum of its longest per-case ranges; each energy evaluates its own case's weights.
        float coef[4][4];
        if (jB > jA) corner_dos_B_coeffs(cs, a.V, coef);
        for (int j = jlo; j <= jhi; ++j) {
          float g[4];
          if (j <= jA) {
            corner_dos_A(cs, local_x(cs, j, a.de), g);
            g[0] = fmaxf(g[0], 0.0f);  // g[1..3] are products of non-negative factors
          } else if (j <= jB) {
            corner_dos_B_poly(coef, local_z(cs, j, a.de), g);
#pragma unroll
            for (int l = 0; l < 4; ++l) g[l] = fmaxf(g[l], 0.0f);
          } else {
            corner_dos_C(cs, local_y(cs, j, a.de), g);
            g[3] = fmaxf(g[3], 0.0f);
          }
          deposit(j, g);
        }
      }
    }
    __syncthreads();
    for (int q = tid; q < L * NORB; q += NT) {
      const int r = q / NORB, m = q - r * NORB;
      const int row = packed ? (m >> 1) : m;
      const unsigned long long* hw = &s_hist[row * RS + (r << cpl)];
      if (MODE == 2) {
        // exact sum of the copies in this workgroup's fixed point (|v| <= B S <= 2^62), then one
        // rounding (halves up) to the common fixed point
        long long v = 0;
        for (int c = 0; c < CP; ++c) {
          const unsigned long long w = hw[c];
          v += packed ? (long long)(unsigned)((m & 1) ? (w >> 32) : (w & 0xffffffffull)) : (long long)w;
        }
        long long q;
        if (dshift >= 0) q = (long long)((unsigned long long)v << dshift);
        else if (dshift > -63) q = (v + (1ll << (-dshift - 1))) >> (-dshift);
        else q = 0;  // |v| < 2^62 <= half a unit of the common fixed point
        if (q != 0) atomicAdd(&a.gacc[(int64_t)(c0 + r) * NORB + m], (unsigned long long)q);
      } else {
        double sum = 0.0;
        for (int c = 0; c < CP; ++c) {
          const unsigned long long w = hw[c];
          sum += packed ? (double)(unsigned)((m & 1) ? (w >> 32) : (w & 0xffffffffull)) : (double)(long long)w;
        }
        // the scale formed here rather than kept live over the passes (a register less there)
        if (sum != 0.0) atomic_add_global(&a.dos[(int64_t)(c0 + r) * NORB + m], (float)ldexp(sum, -sexp));
      }
    }
    __syncthreads();
  }
}

template <int NORB, typename WT, int MODE>
__global__ __launch_bounds__(NT, fwd_waves<NORB>()) void dos_forward_kernel(FwdArgs a) {
  // XCD-aware mapping: hardware dispatches block b to XCD b % 8; give each XCD a contiguous range.
  const int b = blockIdx.x;
  const int unit = (b % NXCD) * a.per_xcd + b / NXCD;
  if (unit < a.nunits) forward_unit<NORB, WT, MODE>(a, unit);
}


__global__ void fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// ---------------------------------------------------------------------------------------------
// Batched forward: one persistent launch over the flattened (item, band, tile) work queue of up to
// kMaxBatch problems with the same orbital count. Workgroups pull units from an atomic counter in the
// caller's workspace, so problems of very different sizes balance across the chip.

struct BatchItem {
  const float* eps;
  const void* w;
  const float* w_scale;
  float* dos;
  int n1, n2, n3, ne;
  float e0, de;
  int TX, TY, TZ;
  int t1, t2, t3, ntiles;
  int unit_begin;  // first global unit of this item (items in order, units band-major)
};

struct BatchArgs {
  int n, total;
  unsigned* counter;
  BatchItem it[kMaxBatch];
};

template <int NORB, typename WT>
__global__ __launch_bounds__(NT, NORB <= 8 ? 5 : 2) void dos_batched_kernel(BatchArgs b) {
  __shared__ int s_unit;
  for (;;) {
    __syncthreads();  // the previous unit's LDS reads are done
    if (threadIdx.x == 0) s_unit = (int)atomicAdd(b.counter, 1u);
    __syncthreads();
    const int u = s_unit;
    if (u >= b.total) return;  // every lane read the same u: the whole workgroup leaves
    int i = 0;
    while (i + 1 < b.n && b.it[i + 1].unit_begin <= u) ++i;
    const BatchItem& it = b.it[i];
    FwdArgs a;
    a.eps = it.eps;
    a.w = it.w;
    a.w_scale = it.w_scale;
    a.wtype = 0;  // not read by the unit body (the type is the template argument)
    a.dos = it.dos;
    a.gexp = nullptr;
    a.gacc = nullptr;
    a.lg_units = 0;
    a.n1 = it.n1;
    a.n2 = it.n2;
    a.n3 = it.n3;
    a.ne = it.ne;
    a.e0 = it.e0;
    a.de = it.de;
    a.inv_de = 1.0f / it.de;
    a.V = (float)(1.0 / (24.0 * (double)it.n1 * it.n2 * it.n3));
    a.TX = it.TX;
    a.TY = it.TY;
    a.TZ = it.TZ;
    a.t1 = it.t1;
    a.t2 = it.t2;
    a.t3 = it.t3;
    a.ntiles = it.ntiles;
    a.nunits = 0;
    a.per_xcd = 0;
    forward_unit<NORB, WT, 0>(a, u - it.unit_begin);
  }
}

// Zero every item's DOS (blockIdx.y = item) and the work counter.
__global__ void batched_zero_kernel(BatchArgs b, int norb) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *b.counter = 0u;
  const BatchItem& it = b.it[blockIdx.y];
  const int64_t n = (int64_t)it.ne * norb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    it.dos[i] = 0.0f;
}

template <int NORB, typename WT>
hipError_t occupancy_batched(int* occ) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, dos_batched_kernel<NORB, WT>, NT, 0);
}

template <int NORB>
hipError_t launch_batched(const BatchArgs& b, int wtype, hipStream_t s) {
  hipLaunchKernelGGL(batched_zero_kernel, dim3(64, b.n), dim3(256), 0, s, b, NORB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Persistent grid: resident workgroups per CU times the CU count of the current device (cached
  // per device and weight type; concurrent first calls store the same values).
  constexpr int kDevCache = 64;
  static std::atomic<int> cache_cus[kDevCache], cache_occ[kDevCache][3];
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  const bool cached = dev >= 0 && dev < kDevCache;
  int cus = cached ? cache_cus[dev].load(std::memory_order_relaxed) : 0;
  if (!cus) {
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if (cached) cache_cus[dev].store(cus, std::memory_order_relaxed);
  }
  int occ = cached ? cache_occ[dev][wtype].load(std::memory_order_relaxed) : 0;
  if (!occ) {
    e = wtype == TETRA_W_F16   ? occupancy_batched<NORB, _Float16>(&occ)
        : wtype == TETRA_W_C32 ? occupancy_batched<NORB, float2>(&occ)
                               : occupancy_batched<NORB, float>(&occ);
    if (e != hipSuccess) return e;
    if (occ < 1) occ = 1;
    if (cached) cache_occ[dev][wtype].store(occ, std::memory_order_relaxed);
  }
  const int grid = std::min(b.total, occ * cus);
  if (wtype == TETRA_W_F16)
    hipLaunchKernelGGL((dos_batched_kernel<NORB, _Float16>), dim3(grid), dim3(NT), 0, s, b);
  else if (wtype == TETRA_W_C32)
    hipLaunchKernelGGL((dos_batched_kernel<NORB, float2>), dim3(grid), dim3(NT), 0, s, b);
  else
    hipLaunchKernelGGL((dos_batched_kernel<NORB, float>), dim3(grid), dim3(NT), 0, s, b);
  return hipGetLastError();
}

template <int NORB, int MODE>
hipError_t launch_fwd_mode(const FwdArgs& a, int grid, hipStream_t s) {
  if (a.wtype == TETRA_W_F16)
    hipLaunchKernelGGL((dos_forward_kernel<NORB, _Float16, MODE>), dim3(grid), dim3(NT), 0, s, a);
  else if (a.wtype == TETRA_W_C32)
    hipLaunchKernelGGL((dos_forward_kernel<NORB, float2, MODE>), dim3(grid), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((dos_forward_kernel<NORB, float, MODE>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

constexpr int kNoBound = -100000;  // *gexp before any workgroup has a bound

// Exact-mode set-up: no bound yet, every accumulator at zero (plain stores: capturable in a graph).
__global__ void exact_init_kernel(int* gexp, unsigned long long* acc, int64_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *gexp = kNoBound;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc[i] = 0ull;
}

// dos = acc / S with S the common scale of mode 2 (all zero when no workgroup had anything to add).
__global__ void fixed_to_float_kernel(const unsigned long long* acc, const int* gexp, int lg_units, float* dos,
                                      int64_t n) {
  const int ge = *gexp;
  const double inv_S = ge == kNoBound ? 0.0 : ldexp(1.0, -exact_scale_exp(ge, lg_units));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dos[i] = (float)((double)(long long)acc[i] * inv_S);
}

template <int NORB>
hipError_t launch_fwd(const FwdArgs& a, int grid, hipStream_t s) {
  if (!a.gacc) return launch_fwd_mode<NORB, 0>(a, grid, s);
  hipError_t e = launch_fwd_mode<NORB, 1>(a, grid, s);
  if (e != hipSuccess) return e;
  e = launch_fwd_mode<NORB, 2>(a, grid, s);
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)a.ne * NORB;
  hipLaunchKernelGGL(fixed_to_float_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                     a.gacc, a.gexp, a.lg_units, a.dos, n);
  return hipGetLastError();
}

}  // namespace

hipError_t fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t forward(const tetra_desc& d, const float* eps, const void* w, int wtype, const float* w_scale, float* dos,
                   void* exact_scratch, int shape, hipStream_t s) {
  FwdArgs a;
  a.wtype = wtype;
  // exact_scratch (exact mode): 256 bytes holding the largest bound exponent, then ne*norb 64-bit sums
  a.gexp = exact_scratch ? static_cast<int*>(exact_scratch) : nullptr;
  a.gacc = exact_scratch ? reinterpret_cast<unsigned long long*>(static_cast<char*>(exact_scratch) + 256) : nullptr;
  a.eps = eps;
  a.w = w;
  a.w_scale = w_scale;
  a.dos = dos;
  a.n1 = d.n1;
  a.n2 = d.n2;
  a.n3 = d.n3;
  a.ne = d.ne;
  a.e0 = d.e0;
  a.de = d.de;
  a.inv_de = 1.0f / d.de;
  a.V = (float)(1.0 / (24.0 * (double)d.n1 * d.n2 * d.n3));  // V_T / (4 V_G)
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
  a.lg_units = 0;
  while ((1ll << a.lg_units) < (long long)a.nunits) ++a.lg_units;
  const int grid = a.per_xcd * NXCD;
  hipError_t e = hipSuccess;
  if (exact_scratch) {
    const int64_t n = (int64_t)d.ne * d.norb;
    hipLaunchKernelGGL(exact_init_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                       a.gexp, a.gacc, n);
    e = hipGetLastError();
  } else {
    e = fill_zero(dos, (int64_t)d.ne * d.norb, s);
  }
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

size_t batched_launches(const tetra_item* items, int n) {
  size_t launches = 0;
  for (int norb = 1; norb <= 16; ++norb) {
    int cnt = 0;
    for (int i = 0; i < n; ++i) cnt += items[i].d.norb == norb;
    launches += (cnt + kMaxBatch - 1) / kMaxBatch;
  }
  return launches;
}

hipError_t batched(const tetra_item* items, const int* shapes, int n, int wtype, void* workspace, hipStream_t s) {
  unsigned* counters = static_cast<unsigned*>(workspace);
  int launch = 0;
  for (int norb = 1; norb <= 16; ++norb) {
    BatchArgs b;
    b.n = 0;
    b.total = 0;
    for (int i = 0; i <= n; ++i) {
      const bool flush = (i == n && b.n > 0) || b.n == kMaxBatch;
      if (flush) {
        b.counter = counters + 64 * launch++;  // one 256-byte line per launch
        hipError_t e = hipSuccess;
        switch (norb) {
#define TETRA_CASE(N) \
  case N:             \
    e = launch_batched<N>(b, wtype, s); \
    break;
          TETRA_CASE(1) TETRA_CASE(2) TETRA_CASE(3) TETRA_CASE(4) TETRA_CASE(5) TETRA_CASE(6) TETRA_CASE(7)
          TETRA_CASE(8) TETRA_CASE(9) TETRA_CASE(10) TETRA_CASE(11) TETRA_CASE(12) TETRA_CASE(13)
          TETRA_CASE(14) TETRA_CASE(15) TETRA_CASE(16)
#undef TETRA_CASE
          default:
            e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        b.n = 0;
        b.total = 0;
      }
      if (i == n) break;
      const tetra_desc& d = items[i].d;
      if (d.norb != norb) continue;
      BatchItem& it = b.it[b.n++];
      it.eps = items[i].eps;
      it.w = items[i].w;
      it.w_scale = wtype == TETRA_W_F16 ? items[i].w_scale : nullptr;
      it.dos = items[i].dos;
      it.n1 = d.n1;
      it.n2 = d.n2;
      it.n3 = d.n3;
      it.ne = d.ne;
      it.e0 = d.e0;
      it.de = d.de;
      const TileShape sh = tile_shape(shapes ? shapes[i] : 0);
      it.TX = sh.x;
      it.TY = sh.y;
      it.TZ = sh.z;
      it.t1 = (d.n1 + sh.x - 1) / sh.x;
      it.t2 = (d.n2 + sh.y - 1) / sh.y;
      it.t3 = (d.n3 + sh.z - 1) / sh.z;
      it.ntiles = it.t1 * it.t2 * it.t3;
      it.unit_begin = b.total;
      b.total += it.ntiles * d.nb;
    }
  }
  return hipSuccess;
}

}  // namespace tetra
