// Host-side declarations shared by the library's translation units. Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tetra.h"

namespace tetra {

constexpr int kMaxBatch = 32;  // problems per persistent batched launch

// Tile shapes (cubes along grid axes 1, 2, 3) of the forward and adjoint kernels: one lane per cube,
// kTileCubes lanes per workgroup. Shape 0 is the default; the others are for the autotuner.
constexpr int kTileCubes = 256;
constexpr int kTileShapes = 6;
struct TileShape {
  int x, y, z;
};
// Every shape stages at most 425 points, the default's count, so LDS use (and occupancy) matches
// the default.
constexpr TileShape kTileShape[kTileShapes] = {{4, 4, 16}, {8, 8, 4}, {4, 8, 8}, {8, 4, 8}, {4, 16, 4}, {16, 4, 4}};
constexpr int kTilePointsMax = 5 * 5 * 17;  // largest (x+1)(y+1)(z+1) above
__host__ __device__ inline TileShape tile_shape(int id) {
  return (id >= 0 && id < kTileShapes) ? kTileShape[id] : kTileShape[0];
}

hipError_t fill_zero(float* p, int64_t n, hipStream_t s);
// Weights w by wtype: TETRA_W_F32 float, TETRA_W_F16 _Float16 with the per-band w_scale, TETRA_W_C32
// complex amplitudes (float2). exact_scratch (or null) is device memory of
// forward_exact_scratch_bytes(d) for the exact cross-workgroup accumulation.
hipError_t forward(const tetra_desc& d, const float* eps, const void* w, int wtype, const float* w_scale, float* dos,
                   void* exact_scratch, int shape, hipStream_t s);
// Batched forward: items grouped by orbital count, up to kMaxBatch per persistent launch. The
// workspace holds one 256-byte work counter per launch.
size_t batched_launches(const tetra_item* items, int n);
hipError_t batched(const tetra_item* items, const int* shapes, int n, int wtype, void* workspace, hipStream_t s);
// Exact mode of the forward: 256 bytes (the largest bound exponent), then ne*norb 64-bit sums.
inline size_t forward_exact_scratch_bytes(const tetra_desc& d) { return 256 + 8 * (size_t)d.ne * d.norb; }
// FP16 weights with a per-band power-of-two scale: w [nb][per_band] -> w16, w_scale [nb].
hipError_t pack_f16(int nb, int64_t per_band, const float* w, void* w16, float* w_scale, hipStream_t s);
// Number of states (binned = false) or bin-averaged DOS (binned = true) into out[ne][norb].
hipError_t nos(const tetra_desc& d, const float* eps, const void* w, int wtype, const float* w_scale, float* out,
               bool binned, int shape, hipStream_t s);
// grad_w is [nb][norb][nk] floats, or [nb][norb][nk][2] for complex amplitudes. With a workspace of
// backward_workspace_bytes(d, shape) bytes (non-zero only where the grid sides are multiples of the
// tile's, with more than one tile per axis), tile-boundary points take the two-phase output; with
// none, global atomics into zero-filled outputs.
size_t backward_workspace_bytes(const tetra_desc& d, int shape);
hipError_t backward(const tetra_desc& d, const float* eps, const void* w, int wtype, const float* w_scale,
                    const float* G, float* grad_eps, float* grad_w, int shape, void* workspace, hipStream_t s);

// Susceptibility spectral weight into out[ne][norb] (the energy grid of d is the transfer-energy
// grid) for the transfer (q1, q2, q3) in grid steps and Fermi energy e_fermi; every band pair.
// ranges_ws: NULL, or device memory for chi_range_entries(d, shape) float2 values (the first pass's
// energy range of every (tile, band) at k and at k + q).
int64_t chi_units(const tetra_desc& d, int shape);
int64_t chi_range_entries(const tetra_desc& d, int shape);
hipError_t chi(const tetra_desc& d, int q1, int q2, int q3, float e_fermi, const float* eps, const void* w, int wtype,
               const float* w_scale, float* out, int shape, void* ranges_ws, hipStream_t s);

}  // namespace tetra
