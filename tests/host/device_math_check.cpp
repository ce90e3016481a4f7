// Host build of the kernels' per-tetrahedron arithmetic (tetra_device.h) against the FP64 oracle's
// corner weights and their dual-number energy derivatives. Test harness only: compiled by
// tests/test_device_math_host.py with g++ and linked with the oracle library.
//
// For random tetrahedra (generic, and with one pair of neighbouring corner energies within 1e-3) on
// an equidistant energy grid, with random loss gradients G[j][m] and orbital weights b_l[m]:
//  * the corner weights of every in-window energy, per case (the middle case in its cubic form),
//    against the oracle's;
//  * per case range, the adjoint as the kernel forms it: power sums H_k[m] = sum_j G[j][m] t_j^k over
//    the range, then adjoint_range_* for the weight gradient sum_j G[j][m] g_l(E_j) and the energy
//    gradient sum_j sum_l s_l dg_l/dE_i (s_l = sum_m G[j][m] b_l[m]), against the oracle's sums.
// Prints one line per case: ranges, max weight error (relative to the tetrahedron's largest weight),
// max energy-gradient error (relative to the range's sum of per-energy |derivatives|) for generic and
// nearly degenerate tetrahedra, and max weight-gradient error (relative to sum_j |G| |g|).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <random>

#include "tetra_device.h"
#include "tetra_nos_device.h"

extern "C" void tetra_oracle_corner_weights(const double e_sorted[4], double E, double vol, double w[4], double g[4]);
extern "C" void tetra_oracle_corner_weights_grad(const double e_sorted[4], double E, double vol, double g[4],
                                                 double dg[16]);

using namespace tetra;

constexpr int NO = 3;  // orbitals

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 100000;
  std::mt19937 rng(11);
  std::uniform_real_distribution<float> U(-1.0f, 1.0f), P(0.0f, 1.0f);
  const float V = 1.0e-3f, e0 = -1.5f, de = 3.0f / 1999.0f;
  double werr[3] = {0, 0, 0}, eerr[3][2] = {{0, 0}, {0, 0}, {0, 0}}, berr[3] = {0, 0, 0};
  long ranges[3] = {0, 0, 0};
  for (int it = 0; it < n; ++it) {
    float e[4];
    for (int l = 0; l < 4; ++l) e[l] = U(rng);
    const int kind = it % 4;  // 0 generic; 1..3 one pair of neighbouring corners within 1e-3
    if (kind > 0) e[kind] = e[kind - 1] + 1.0e-3f * U(rng);
    int p[4] = {0, 1, 2, 3};
    sort4(e, p);
    const double ed[4] = {e[0], e[1], e[2], e[3]};
    const TetSetup cs = tet_setup(e, e0, V);
    int jlo, jhi;
    energy_window(e[0], e[3], e0, 1.0f / de, 0, 1999, jlo, jhi);
    tet_window(cs, de, 0, 1999, jlo, jhi);
    if (jlo > jhi) continue;
    int jA, jB;
    case_split(cs, de, 1.0f / de, jlo, jhi, jA, jB);
    float b[4][NO];
    for (int l = 0; l < 4; ++l)
      for (int m = 0; m < NO; ++m) b[l][m] = P(rng);
    const float* const brow[4] = {b[0], b[1], b[2], b[3]};
    double gmax = 0;
    for (int j = jlo; j <= jhi; ++j) {
      double g[4], dg[16];
      tetra_oracle_corner_weights_grad(ed, (double)e0 + (double)j * de, 4.0 * V, g, dg);
      for (int l = 0; l < 4; ++l) gmax = std::fmax(gmax, std::fabs(g[l]));
    }
    const int lo[3] = {jlo, jA + 1, jB + 1}, hi[3] = {jA, jB, jhi};
    float coef[4][4];
    corner_dos_B_coeffs(cs, V, coef);
    for (int k = 0; k < 3; ++k) {
      if (hi[k] < lo[k]) continue;
      float H[4][NO] = {};  // powers 1..3 (first, third case) or 0..3 (middle case)
      double eref[4] = {0, 0, 0, 0}, escale = 0, bref[4][NO] = {}, bscale = 0;
      for (int j = lo[k]; j <= hi[k]; ++j) {
        float G[NO];
        for (int m = 0; m < NO; ++m) G[m] = U(rng);
        double g[4], dg[16];
        tetra_oracle_corner_weights_grad(ed, (double)e0 + (double)j * de, 4.0 * V, g, dg);
        double s[4];
        for (int l = 0; l < 4; ++l) {
          s[l] = 0;
          for (int m = 0; m < NO; ++m) s[l] += (double)G[m] * b[l][m];
          for (int m = 0; m < NO; ++m) {
            bref[l][m] += (double)G[m] * g[l];
            bscale += std::fabs((double)G[m] * g[l]);
          }
        }
        for (int i = 0; i < 4; ++i) {
          double acc = 0;
          for (int l = 0; l < 4; ++l) acc += s[l] * dg[4 * l + i];
          eref[i] += acc;
          escale += std::fabs(acc);
        }
        float gk[4], t;
        if (k == 0) {
          t = local_x(cs, j, de);
          corner_dos_A(cs, t, gk);
        } else if (k == 1) {
          t = local_z(cs, j, de);
          corner_dos_B_poly(coef, t, gk);
        } else {
          t = local_y(cs, j, de);
          corner_dos_C(cs, t, gk);
        }
        for (int l = 0; l < 4; ++l) werr[k] = std::fmax(werr[k], std::fabs(gk[l] - g[l]) / gmax);
        const float t2 = t * t, t3 = t2 * t;
        for (int m = 0; m < NO; ++m) {
          if (k == 1) {
            H[0][m] += G[m];
            H[1][m] = std::fma(G[m], t, H[1][m]);
            H[2][m] = std::fma(G[m], t2, H[2][m]);
            H[3][m] = std::fma(G[m], t3, H[3][m]);
          } else {
            H[0][m] = std::fma(G[m], t, H[0][m]);
            H[1][m] = std::fma(G[m], t2, H[1][m]);
            H[2][m] = std::fma(G[m], t3, H[2][m]);
          }
        }
      }
      float gb[4][NO] = {}, Eb[4];
      if (k == 0) adjoint_range_A<NO>(cs, V, brow, H, gb, Eb);
      else if (k == 1) adjoint_range_B<NO>(cs, V, brow, H, gb, Eb);
      else adjoint_range_C<NO>(cs, V, brow, H, gb, Eb);
      double de_ = 0, db_ = 0;
      for (int i = 0; i < 4; ++i) de_ = std::isfinite(Eb[i]) ? std::fmax(de_, std::fabs(Eb[i] - eref[i])) : INFINITY;
      for (int l = 0; l < 4; ++l)
        for (int m = 0; m < NO; ++m)
          db_ = std::isfinite(gb[l][m]) ? std::fmax(db_, std::fabs(gb[l][m] - bref[l][m])) : INFINITY;
      double& slot = eerr[k][kind == 0 ? 0 : 1];
      slot = std::fmax(slot, de_ / escale);
      berr[k] = std::fmax(berr[k], db_ / bscale);
      ++ranges[k];
    }
  }
  const char* names[3] = {"first", "middle", "third"};
  for (int k = 0; k < 3; ++k)
    std::printf("%s %ld %.6e %.6e %.6e %.6e\n", names[k], ranges[k], werr[k], eerr[k][0], eerr[k][1], berr[k]);

  // Integrated weights (number of states) as the kernel forms them: the exact steps ja (first E_j > E1)
  // and js (first E_j >= E4) of step_window on the FP32 frames, the case split of the window [ja, js),
  // the case polynomials in FP64 and in FP32, and V from js on, on the grid E_j = e0 + (j + joff) de for joff = 0
  // and -1/2 (the bin midpoints). Compared with the oracle's w_l(E_j) for every j from ja - 2 to
  // js + 1, relative to V; a step index that disagrees with the FP64 comparison by more than FP32
  // rounding is counted. Then the increments w_l(E_j) - w_l(E_{j-1}) on grids 1e3 and 1e5 times finer
  // than the tetrahedron, relative to the largest increment of the tetrahedron.
  for (int half = 0; half < 2; ++half) {
    const float joff = half ? -0.5f : 0.0f;
    double nerr = 0.0, nerr32 = 0.0;
    long npts = 0, nbad = 0;
    for (int it = 0; it < n; ++it) {
      float e[4];
      for (int l = 0; l < 4; ++l) e[l] = U(rng);
      const int kind = it % 4;
      if (kind > 0) e[kind] = e[kind - 1] + 1.0e-3f * U(rng);
      if (it % 97 == 0) e[1] = e[0];  // exactly equal neighbours
      int p[4] = {0, 1, 2, 3};
      sort4(e, p);
      const double ed[4] = {e[0], e[1], e[2], e[3]};
      TetSetup cs = tet_setup(e, e0, V);
      shift_frames(cs, joff * de);
      const NosSetup ns = nos_setup(e, e0, joff, de, (double)V);
      int ja, js;
      step_window(cs, e[0], e[3], e0, joff, de, 1.0f / de, ja, js);
      auto Ej = [&](int j) { return (double)e0 + ((double)j + (double)joff) * (double)de; };
      int ta = ja, ts = js;  // FP64 steps
      while (Ej(ta) > ed[0]) --ta;
      while (!(Ej(ta) > ed[0])) ++ta;
      while (Ej(ts) >= ed[3]) --ts;
      while (!(Ej(ts) >= ed[3])) ++ts;
      // a few FP32 roundings of the local frame x_j and of E41
      const double tol = 1.0e-6 * de + 2.5e-7 * (ed[3] - ed[0]) + 1.2e-7 * std::fabs(Ej(js) - e0);
      if (ta != ja && std::fabs(Ej(std::min(ta, ja)) - ed[0]) > tol) ++nbad;
      if (ts != js && std::fabs(Ej(std::min(ts, js)) - ed[3]) > tol) ++nbad;
      const int lo = std::min(ja, js), jlast = js - 1;
      int jA = lo - 1, jB = lo - 1;
      if (jlast >= lo) case_split(cs, de, 1.0f / de, lo, jlast, jA, jB);
      double coef[4][5];
      corner_nos_B_coeffs(ns, (double)V, coef);
      float coef32[4][5];
      corner_nos_B_coeffs(cs, V, coef32);
      for (int j = lo - 2; j <= js + 1; ++j) {
        double w[4];
        float w32[4];
        if (j < lo) {
          for (int l = 0; l < 4; ++l) w[l] = w32[l] = 0.0f;
        } else if (j >= js) {
          for (int l = 0; l < 4; ++l) w[l] = w32[l] = V;
        } else if (j <= jA) {
          corner_nos_A(ns, std::fma((double)j, (double)de, ns.x0), w);
          corner_nos_A(cs, local_x(cs, j, de), w32);
        } else if (j <= jB) {
          corner_nos_B_poly(coef, std::fma((double)j, (double)de, ns.z0), w);
          corner_nos_B_poly(coef32, local_z(cs, j, de), w32);
        } else {
          corner_nos_C(ns, (double)V, std::fma(-(double)j, (double)de, ns.y0), w);
          corner_nos_C(cs, V, local_y(cs, j, de), w32);
        }
        double wr[4], gr[4];
        tetra_oracle_corner_weights(ed, Ej(j), 4.0 * V, wr, gr);
        for (int l = 0; l < 4; ++l) {
          nerr = std::fmax(nerr, std::isfinite(w[l]) ? std::fabs(w[l] - wr[l]) / V : INFINITY);
          nerr32 = std::fmax(nerr32, std::isfinite(w32[l]) ? std::fabs(w32[l] - wr[l]) / V : INFINITY);
        }
        ++npts;
      }
    }
    std::printf("%s %ld %.6e %ld\n", half ? "nos_half" : "nos", npts, nerr, nbad);
    std::printf("%s %ld %.6e %ld\n", half ? "nos32_half" : "nos32", npts, nerr32, nbad);
  }
  for (int fine = 0; fine < 2; ++fine) {
    const double ratio = fine ? 1.0e5 : 1.0e3;  // E41 / de
    double ierr = 0.0;
    long ninc = 0;
    for (int it = 0; it < n / 10; ++it) {
      float e[4];
      for (int l = 0; l < 4; ++l) e[l] = U(rng);
      int p[4] = {0, 1, 2, 3};
      sort4(e, p);
      const double ed[4] = {e[0], e[1], e[2], e[3]};
      if (!(ed[3] - ed[0] > 1e-2)) continue;
      const float dg = (float)((ed[3] - ed[0]) / ratio), g0 = -1.5f;
      const NosSetup ns = nos_setup(e, g0, 0.0f, dg, (double)V);
      double coef[4][5];
      corner_nos_B_coeffs(ns, (double)V, coef);
      // three sample bins per case, away from the case boundaries (the kernel splits the window at them)
      const double bnd[4] = {ed[0], ed[1], ed[2], ed[3]};
      double incmax = 0.0, emax = 0.0;
      for (int cse = 0; cse < 3; ++cse) {
        if (!(bnd[cse + 1] - bnd[cse] > 10.0 * dg)) continue;
        for (int q = 1; q <= 3; ++q) {
          const double Emid = bnd[cse] + (bnd[cse + 1] - bnd[cse]) * q / 4.0;
          const int j = (int)std::floor((Emid - g0) / dg);
          double w1[4], w0[4];
          for (int side = 0; side < 2; ++side) {
            double* w = side ? w1 : w0;
            const double jd = (double)(j - 1 + side);
            if (cse == 0) corner_nos_A(ns, std::fma(jd, (double)dg, ns.x0), w);
            else if (cse == 1) corner_nos_B_poly(coef, std::fma(jd, (double)dg, ns.z0), w);
            else corner_nos_C(ns, (double)V, std::fma(-jd, (double)dg, ns.y0), w);
          }
          double r1[4], r0[4], gr[4];
          tetra_oracle_corner_weights(ed, (double)g0 + (double)j * dg, 4.0 * V, r1, gr);
          tetra_oracle_corner_weights(ed, (double)g0 + (double)(j - 1) * dg, 4.0 * V, r0, gr);
          for (int l = 0; l < 4; ++l) {
            const float inc = (float)std::fmax(w1[l] - w0[l], 0.0);
            incmax = std::fmax(incmax, r1[l] - r0[l]);
            emax = std::fmax(emax, std::fabs((double)inc - (r1[l] - r0[l])));
          }
          ++ninc;
        }
      }
      if (incmax > 0.0) ierr = std::fmax(ierr, emax / incmax);
    }
    std::printf("inc%s %ld %.6e\n", fine ? "_1e5" : "_1e3", ninc, ierr);
  }
  return 0;
}
