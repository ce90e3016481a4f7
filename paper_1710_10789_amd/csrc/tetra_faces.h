// Tile-face indexing for the two-phase output of the adjoint.
//
// A tile of TX x TY x TZ cubes stages the (TX+1)(TY+1)(TZ+1) grid points of its cubes' corners. A point
// with every local coordinate strictly inside (1 <= p < T on each axis) has all eight of its cubes in
// the tile; the others lie on one of the six faces and receive contributions from up to eight tiles.
// face_index numbers the face points of one tile densely, in an order that keeps runs along the
// fastest grid axis contiguous:
//   * the two x faces (px = 0, px = TX), whole: 2 (TY+1)(TZ+1) points;
//   * the two y faces without the x edges (0 < px < TX, py in {0, TY}): 2 (TX-1)(TZ+1) points;
//   * the z faces without the x and y edges (0 < px < TX, 0 < py < TY, pz in {0, TZ}):
//     2 (TX-1)(TY-1) points.
// Host and device code share it (the host checks it is a bijection onto [0, face_count)).

#pragma once

#include <hip/hip_runtime.h>

namespace tetra {

__host__ __device__ __forceinline__ int face_count(int TX, int TY, int TZ) {
  return 2 * (TY + 1) * (TZ + 1) + 2 * (TX - 1) * (TZ + 1) + 2 * (TX - 1) * (TY - 1);
}

// Requires (px, py, pz) to be a face point of the tile.
__host__ __device__ __forceinline__ int face_index(int px, int py, int pz, int TX, int TY, int TZ) {
  const int PY = TY + 1, PZ = TZ + 1;
  if (px == 0 || px == TX) return (px == TX ? PY * PZ : 0) + py * PZ + pz;
  int base = 2 * PY * PZ;
  if (py == 0 || py == TY) return base + (2 * (px - 1) + (py == TY ? 1 : 0)) * PZ + pz;
  base += 2 * (TX - 1) * PZ;
  return base + 2 * ((px - 1) * (TY - 1) + (py - 1)) + (pz == TZ ? 1 : 0);
}

// The tiles holding a partial sum of grid coordinate c (0 <= c < n) along one axis with tile length
// T (n a multiple of T, more than one tile): the tile of cube c at local coordinate c mod T, and, when
// that is 0, also the previous tile (periodic) at local coordinate T. Returns the number of tiles (1
// or 2); tile[i], local[i] receive them.
__host__ __device__ __forceinline__ int face_tiles(int c, int T, int ntiles, int tile[2], int local[2]) {
  const int t = c / T, p = c - t * T;
  tile[0] = t;
  local[0] = p;
  if (p != 0) return 1;
  tile[1] = t == 0 ? ntiles - 1 : t - 1;
  local[1] = T;
  return 2;
}

}  // namespace tetra
