// Host check of the adjoint's two-phase output indexing (tetra_faces.h). Test harness only: compiled by
// tests/test_faces_host.py with g++.
//
// For every tile shape and several periodic grids whose sides are multiples of the tile sides (more
// than one tile per axis), with a random value for every (cube, corner):
//  * face_index maps the face points of a tile one-to-one onto [0, face_count);
//  * scatter as the adjoint kernel does (per tile, sums over its cubes at its local points; points with
//    every local coordinate in 1..T-1 stored as complete, the others into the tile's face slots), then
//    gather as the second pass does (for a grid point not complete in its own tile, the sum over the
//    tiles of face_tiles on each axis), and compare with the direct sum over the eight cubes of every
//    grid point.
// Prints "shape TX TY TZ grid n1 n2 n3 maxerr bijective" per case; exits non-zero on any failure.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "tetra_faces.h"

using namespace tetra;

static const int kShapes[6][3] = {{4, 4, 16}, {8, 8, 4}, {4, 8, 8}, {8, 4, 8}, {4, 16, 4}, {16, 4, 4}};

int main() {
  int failures = 0;
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (const auto& sh : kShapes) {
    const int TX = sh[0], TY = sh[1], TZ = sh[2];
    const int PY = TY + 1, PZ = TZ + 1, NP = (TX + 1) * PY * PZ, NF = face_count(TX, TY, TZ);
    // bijection of face_index
    std::vector<int> seen(NF, 0);
    bool bij = true;
    int nface = 0;
    for (int px = 0; px <= TX; ++px)
      for (int py = 0; py <= TY; ++py)
        for (int pz = 0; pz <= TZ; ++pz) {
          const bool interior = px >= 1 && px < TX && py >= 1 && py < TY && pz >= 1 && pz < TZ;
          if (interior) continue;
          ++nface;
          const int f = face_index(px, py, pz, TX, TY, TZ);
          if (f < 0 || f >= NF || seen[f]++) bij = false;
        }
    if (nface != NF || nface != NP - (TX - 1) * (TY - 1) * (TZ - 1)) bij = false;
    const int grids[3][3] = {{2 * TX, 2 * TY, 2 * TZ}, {3 * TX, 2 * TY, 4 * TZ}, {2 * TX, 5 * TY, 2 * TZ}};
    for (const auto& g : grids) {
      const int n1 = g[0], n2 = g[1], n3 = g[2];
      const int t1 = n1 / TX, t2 = n2 / TY, t3 = n3 / TZ, ntiles = t1 * t2 * t3;
      const long nk = (long)n1 * n2 * n3;
      // val[cube][corner s], corner offsets (s & 1, s >> 1 & 1, s >> 2)
      std::vector<double> val(nk * 8);
      for (auto& v : val) v = U(rng);
      std::vector<double> direct(nk, 0.0), out(nk, std::nan("")), part((size_t)ntiles * NF, std::nan(""));
      for (int x = 0; x < n1; ++x)
        for (int y = 0; y < n2; ++y)
          for (int z = 0; z < n3; ++z)
            for (int s = 0; s < 8; ++s) {
              const long k = ((long)((x + (s & 1)) % n1) * n2 + (y + ((s >> 1) & 1)) % n2) * n3 + (z + (s >> 2)) % n3;
              direct[k] += val[(((long)x * n2 + y) * n3 + z) * 8 + s];
            }
      // first phase, per tile
      for (int tile = 0; tile < ntiles; ++tile) {
        const int tz = tile % t3, ty = (tile / t3) % t2, tx = tile / (t3 * t2);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        std::vector<double> acc(NP, 0.0);
        for (int cx = 0; cx < TX; ++cx)
          for (int cy = 0; cy < TY; ++cy)
            for (int cz = 0; cz < TZ; ++cz)
              for (int s = 0; s < 8; ++s) {
                const int p = ((cx + (s & 1)) * PY + cy + ((s >> 1) & 1)) * PZ + cz + (s >> 2);
                acc[p] += val[(((long)(x0 + cx) * n2 + y0 + cy) * n3 + z0 + cz) * 8 + s];
              }
        for (int px = 0; px <= TX; ++px)
          for (int py = 0; py <= TY; ++py)
            for (int pz = 0; pz <= TZ; ++pz) {
              const double v = acc[(px * PY + py) * PZ + pz];
              const bool interior = px >= 1 && px < TX && py >= 1 && py < TY && pz >= 1 && pz < TZ;
              if (interior) {
                out[((long)(x0 + px) * n2 + y0 + py) * n3 + z0 + pz] = v;
              } else {
                part[(size_t)tile * NF + face_index(px, py, pz, TX, TY, TZ)] = v;
              }
            }
      }
      // second phase, per grid point not complete in its own tile
      for (int x = 0; x < n1; ++x)
        for (int y = 0; y < n2; ++y)
          for (int z = 0; z < n3; ++z) {
            int ta[2], pa[2], tb[2], pb[2], tc[2], pc[2];
            const int na = face_tiles(x, TX, t1, ta, pa), nb = face_tiles(y, TY, t2, tb, pb), nc = face_tiles(z, TZ, t3, tc, pc);
            if (pa[0] && pb[0] && pc[0]) continue;
            double sum = 0.0;
            for (int i = 0; i < na; ++i)
              for (int j = 0; j < nb; ++j)
                for (int l = 0; l < nc; ++l)
                  sum += part[(size_t)((ta[i] * t2 + tb[j]) * t3 + tc[l]) * NF + face_index(pa[i], pb[j], pc[l], TX, TY, TZ)];
            out[((long)x * n2 + y) * n3 + z] = sum;
          }
      double err = 0.0;
      for (long k = 0; k < nk; ++k) {
        const double e = std::fabs(out[k] - direct[k]);
        err = std::isnan(e) ? INFINITY : std::max(err, e);
      }
      std::printf("shape %d %d %d grid %d %d %d %.3e %d\n", TX, TY, TZ, n1, n2, n3, err, bij ? 1 : 0);
      if (!(err <= 1e-12) || !bij) ++failures;
    }
  }
  return failures ? 1 : 0;
}
