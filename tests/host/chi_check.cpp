// Host build of the susceptibility kernel's per-tetrahedron arithmetic (tetra_chi_device.h: the
// corner reordering and the occupation clipping into sub-tetrahedra, their volumes, the corner
// weights put back from sorted-vertex order and the parent-corner weights; tetra_device.h: the corner
// weights) against the FP64 oracle's
// one-tetrahedron spectral weight. Test harness only: compiled by tests/test_chi_host.py with g++ and
// linked with the oracle library.
//
// For random tetrahedra (corner energies of band n at k and of band n' at k + q, weights W, a Fermi
// energy inside both ranges) and transfer energies inside the range of eps' - eps, prints the largest
// |S_fp32 - S_oracle| relative to the tetrahedron's scale vol * max W / (max - min of eps' - eps), the
// number of cases and the number with a non-zero oracle value.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "tetra_chi_device.h"

extern "C" double tetra_oracle_tet_chi(const double e[4], const double ep[4], const double W[4], double ef, double E,
                                       double vol);

using namespace tetra;

// S of one tetrahedron at transfer energy E in FP32, as the kernel forms it (V = vol / 4).
static float chi_fp32(const float e[4], const float ep[4], const float W[4], float ef, float E, float V) {
  float emin = e[0], emax = e[0], epmin = ep[0], epmax = ep[0];
  for (int c = 1; c < 4; ++c) {
    emin = fminf(emin, e[c]);
    emax = fmaxf(emax, e[c]);
    epmin = fminf(epmin, ep[c]);
    epmax = fmaxf(epmax, ep[c]);
  }
  float total = 0.0f;
  for (int r = 0; r < 2; ++r) {
    if (!region_possible(r, emin, emax, epmin, epmax, ef)) continue;
    // as the kernel: corners reordered inside-first for the first plane, first clipping from the
    // identity, the second from the first's pieces
    float f1[4], f2c[4], dd[4];
    int q[4];
    region_planes(r, e, ep, ef, f1, f2c);
    for (int c = 0; c < 4; ++c) {
      dd[c] = ep[c] - e[c];
      q[c] = c;
    }
    const int ni1 = (f1[0] <= 0.0f) + (f1[1] <= 0.0f) + (f1[2] <= 0.0f) + (f1[3] <= 0.0f);
    if (ni1 > 0 && ni1 < 4) inside_first_corners(f1, f2c, dd, q);
    float Wq[4];
    for (int c = 0; c < 4; ++c) Wq[c] = W[q[c]];
    const float I[4][4] = {{1.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 1.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 1.0f, 0.0f},
                           {0.0f, 0.0f, 0.0f, 1.0f}};
    for (int ia = 0; ia < clip_pieces(ni1); ++ia) {
      float A[4][4], f2[4];
      if (ni1 == 4) {
        for (int i = 0; i < 4; ++i)
          for (int c = 0; c < 4; ++c) A[i][c] = I[i][c];
      } else {
        clip_piece(I, f1, ni1, ia, A);
      }
      for (int i = 0; i < 4; ++i) {
        f2[i] = 0.0f;
        for (int c = 0; c < 4; ++c) f2[i] = __builtin_fmaf(A[i][c], f2c[c], f2[i]);
      }
      const int ni2 = (f2[0] <= 0.0f) + (f2[1] <= 0.0f) + (f2[2] <= 0.0f) + (f2[3] <= 0.0f);
      if (ni2 > 0 && ni2 < 4) inside_first(A, f2);
      for (int ib = 0; ib < clip_pieces(ni2); ++ib) {
        float S[4][4];
        if (ni2 == 4) {
          for (int i = 0; i < 4; ++i)
            for (int c = 0; c < 4; ++c) S[i][c] = A[i][c];
        } else {
          clip_piece(A, f2, ni2, ib, S);
        }
        const float frac = (ni1 == 4 && ni2 == 4) ? 1.0f : sub_volume(S);
        if (!(frac > 0.0f)) continue;
        float d[4];
        for (int i = 0; i < 4; ++i) {
          d[i] = 0.0f;
          for (int c = 0; c < 4; ++c) d[i] = __builtin_fmaf(S[i][c], dd[c], d[i]);
        }
        int tag[4] = {0, 1, 2, 3};
        bool sw[5];
        sort4(d, tag, sw);
        if (!(E > d[0] && E < d[3])) continue;
        const TetSetup cs = tet_setup(d, E, V * frac);  // local frames with e0 = E, j = 0
        float g[4];
        if (E <= d[1]) {
          corner_dos_A(cs, local_x(cs, 0, 1.0f), g);
        } else if (E <= d[2]) {
          float coef[4][4];
          corner_dos_B_coeffs(cs, V * frac, coef);
          corner_dos_B_poly(coef, local_z(cs, 0, 1.0f), g);
        } else {
          corner_dos_C(cs, local_y(cs, 0, 1.0f), g);
        }
        unsort4(sw, g);
        float G[4];
        parent_weights(S, g, G);
        const float v = G[0] * Wq[0] + G[1] * Wq[1] + G[2] * Wq[2] + G[3] * Wq[3];
        total += r == 0 ? v : -v;
      }
    }
  }
  return total;
}

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 20000;
  std::mt19937 rng(23);
  std::uniform_real_distribution<float> U(-1.0f, 1.0f), P(0.1f, 1.0f);
  double worst = 0.0;
  long cases = 0, nonzero = 0;
  for (int it = 0; it < n; ++it) {
    float e[4], ep[4], W[4];
    for (int c = 0; c < 4; ++c) {
      e[c] = U(rng);
      ep[c] = U(rng);
      W[c] = P(rng);
    }
    if (it % 5 == 1) ep[1] = ep[0] + 1.0e-4f * U(rng);  // nearly equal corners
    if (it % 5 == 2) e[2] = e[3] + 1.0e-4f * U(rng);
    const float ef = 0.5f * U(rng);
    float dmin = 1e30f, dmax = -1e30f;
    for (int c = 0; c < 4; ++c) {
      dmin = fminf(dmin, ep[c] - e[c]);
      dmax = fmaxf(dmax, ep[c] - e[c]);
    }
    if (!(dmax - dmin > 1.0e-3f)) continue;
    const float vol = 0.25f;
    for (int k = 0; k < 8; ++k) {
      const float E = dmin + (dmax - dmin) * (0.5f * U(rng) + 0.5f);
      double ed[4], epd[4], Wd[4];
      for (int c = 0; c < 4; ++c) {
        ed[c] = e[c];
        epd[c] = ep[c];
        Wd[c] = W[c];
      }
      const double ref = tetra_oracle_tet_chi(ed, epd, Wd, ef, E, vol);
      const float got = chi_fp32(e, ep, W, ef, E, vol / 4.0f);
      const double scale = vol * 1.0 / (dmax - dmin);
      worst = fmax(worst, fabs(got - ref) / scale);
      ++cases;
      nonzero += ref != 0.0;
    }
  }
  printf("chi %ld %ld %.3e\n", cases, nonzero, worst);
  return 0;
}
