// Host build of the susceptibility kernel's per-tetrahedron arithmetic (tetra_chi_device.h: the
// corner reordering and the occupation clipping into sub-tetrahedra, their volumes, the vertices sorted
// with their barycentric rows and W formed at them; the whole-tetrahedron regions as a plain DOS of
// eps' - eps; tetra_device.h: the corner weights) against the FP64 oracle's
// one-tetrahedron spectral weight. Test harness only: compiled by tests/test_chi_host.py with g++ and
// linked with the oracle library.
//
// For random tetrahedra (corner energies of band n at k and of band n' at k + q, weights W, a Fermi
// energy inside both ranges) and transfer energies inside the range of eps' - eps, prints the largest
// |S_fp32 - S_oracle| relative to the tetrahedron's scale vol * max W / (max - min of eps' - eps), the
// number of cases, the number with a non-zero oracle value and the number of those whose non-empty
// region is the whole tetrahedron (the kernel's unclipped path).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "tetra_chi_device.h"

extern "C" double tetra_oracle_tet_chi(const double e[4], const double ep[4], const double W[4], double ef, double E,
                                       double vol);

using namespace tetra;

// Corner weights dw/dE of sorted energies d at E (local frames with e0 = E, j = 0), as the kernel's
// energy loop forms them.
static void corner_g(const float d[4], float E, float V, float g[4]) {
  const TetSetup cs = tet_setup(d, E, V);
  if (E <= d[1]) {
    corner_dos_A(cs, local_x(cs, 0, 1.0f), g);
  } else if (E <= d[2]) {
    float coef[4][4];
    corner_dos_B_coeffs(cs, V, coef);
    corner_dos_B_poly(coef, local_z(cs, 0, 1.0f), g);
  } else {
    corner_dos_C(cs, local_y(cs, 0, 1.0f), g);
  }
}

// S of one tetrahedron at transfer energy E in FP32, as the kernel forms it (V = vol / 4).
static float chi_fp32(const float e[4], const float ep[4], const float W[4], float ef, float E, float V) {
  float emin = e[0], emax = e[0], epmin = ep[0], epmax = ep[0];
  for (int c = 1; c < 4; ++c) {
    emin = fminf(emin, e[c]);
    emax = fmaxf(emax, e[c]);
    epmin = fminf(epmin, ep[c]);
    epmax = fmaxf(epmax, ep[c]);
  }
  const int whole = (emax <= ef && epmin >= ef) ? 0 : (emin >= ef && epmax <= ef) ? 1 : -1;
  float total = 0.0f;
  for (int r = 0; r < 2; ++r) {
    if (!region_possible(r, emin, emax, epmin, epmax, ef)) continue;
    if (r == whole) {
      // the region is the whole tetrahedron: the DOS of eps' - eps with the corners sorted with their
      // indices and the weights taken in sorted order
      float d[4];
      int q[4] = {0, 1, 2, 3};
      for (int c = 0; c < 4; ++c) d[c] = ep[c] - e[c];
      sort4(d, q);
      if (!(E > d[0] && E < d[3])) continue;
      float g[4];
      corner_g(d, E, V, g);
      const float v = __builtin_fmaf(g[0], W[q[0]], __builtin_fmaf(g[1], W[q[1]],
                      __builtin_fmaf(g[2], W[q[2]], __builtin_fmaf(g[3], W[q[3]], 0.0f))));
      total += r == 0 ? v : -v;
      continue;
    }
    // as the kernel: corners reordered inside-first for the first plane, first clipping from the
    // identity, the second from the first's pieces, each piece's vertices sorted with their rows and
    // W formed at them
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
      for (int i = 0; i < 4; ++i)
        f2[i] = __builtin_fmaf(A[i][0], f2c[0], __builtin_fmaf(A[i][1], f2c[1],
                               __builtin_fmaf(A[i][2], f2c[2], A[i][3] * f2c[3])));
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
        for (int i = 0; i < 4; ++i)
          d[i] = __builtin_fmaf(S[i][0], dd[0], __builtin_fmaf(S[i][1], dd[1],
                                __builtin_fmaf(S[i][2], dd[2], S[i][3] * dd[3])));
        sort4_rows(d, S);
        if (!(E > d[0] && E < d[3])) continue;
        float g[4];
        corner_g(d, E, V * frac, g);
        float v = 0.0f;
        for (int l = 0; l < 4; ++l) {
          float wv = 0.0f;
          for (int c = 0; c < 4; ++c) wv = __builtin_fmaf(S[l][c], Wq[c], wv);
          v = __builtin_fmaf(g[l], wv, v);
        }
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
  long cases = 0, nonzero = 0, whole_cases = 0;
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
    // regions that are the whole tetrahedron: band n occupied and n' empty at every corner, or the reverse
    if (it % 7 == 3 || it % 7 == 4) {
      const float s = it % 7 == 3 ? 1.0f : -1.0f;
      for (int c = 0; c < 4; ++c) {
        e[c] = ef - s * (0.05f + 0.5f * fabsf(e[c]));
        ep[c] = ef + s * (0.05f + 0.5f * fabsf(ep[c]));
      }
    }
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
      float mn = e[0], mx = e[0], pn = ep[0], px = ep[0];
      for (int c = 1; c < 4; ++c) {
        mn = fminf(mn, e[c]);
        mx = fmaxf(mx, e[c]);
        pn = fminf(pn, ep[c]);
        px = fmaxf(px, ep[c]);
      }
      whole_cases += ref != 0.0 && ((mx <= ef && pn >= ef) || (mn >= ef && px <= ef));
    }
  }
  printf("chi %ld %ld %.3e %ld\n", cases, nonzero, worst, whole_cases);
  return 0;
}
