// Host build of the kernels' per-tetrahedron arithmetic (tetra_device.h) against the FP64 oracle's
// corner weights and their dual-number energy derivatives. Test harness only: compiled by
// tests/test_device_math_host.py with g++ and linked with the oracle library.
//
// For random tetrahedra (generic and with nearly equal corner energies) on an equidistant energy grid:
//  * corner weights of every in-window energy, per case, against the oracle's;
//  * per case range, the gradient of sum_j sum_l s_l g_l(E_j) with respect to the four sorted corner
//    energies from the moment forms (*_acc per energy, *_finish per range) against the sum of the
//    oracle's per-energy derivatives.
// Prints one line per case: max weight error (relative to the tetrahedron's largest weight) and max
// gradient error (relative to the sum of the per-energy |derivatives| of the range).
#include <cmath>
#include <cstdio>
#include <random>

#include "tetra_device.h"

extern "C" void tetra_oracle_corner_weights_grad(const double e_sorted[4], double E, double vol, double g[4],
                                                 double dg[16]);

using namespace tetra;

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 100000;
  std::mt19937 rng(11);
  std::uniform_real_distribution<float> U(-1.0f, 1.0f);
  const float V = 1.0e-3f, e0 = -1.5f, de = 3.0f / 1999.0f;
  double werr[3] = {0, 0, 0}, gerr[3][2] = {{0, 0}, {0, 0}, {0, 0}};
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
    const int lo[3] = {jlo, jA + 1, jB + 1}, hi[3] = {jA, jB, jhi};
    double gmax = 0;
    for (int j = jlo; j <= jhi; ++j) {
      double g[4], dg[16];
      tetra_oracle_corner_weights_grad(ed, (double)e0 + (double)j * de, 4.0 * V, g, dg);
      for (int l = 0; l < 4; ++l) gmax = std::fmax(gmax, std::fabs(g[l]));
    }
    for (int k = 0; k < 3; ++k) {
      if (hi[k] < lo[k]) continue;
      float m9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      float M[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
      double ref[4] = {0, 0, 0, 0}, scale = 0;
      for (int j = lo[k]; j <= hi[k]; ++j) {
        const float s[4] = {U(rng), U(rng), U(rng), U(rng)};
        double g[4], dg[16];
        tetra_oracle_corner_weights_grad(ed, (double)e0 + (double)j * de, 4.0 * V, g, dg);
        for (int i = 0; i < 4; ++i) {
          double acc = 0;
          for (int l = 0; l < 4; ++l) acc += (double)s[l] * dg[4 * l + i];
          ref[i] += acc;
          scale += std::fabs(acc);
        }
        float gk[4];
        const float x = local_x(cs, j, de);
        if (k == 0) {
          corner_dos_A(cs, x, gk);
          corner_dos_moments_acc_A(x, s, m9);
        } else if (k == 1) {
          const float z = local_z(cs, j, de);
          corner_dos_B(cs, z, gk);
          corner_dos_moments_acc_B(z, s, M);
        } else {
          const float y = local_y(cs, j, de);
          corner_dos_C(cs, y, gk);
          corner_dos_moments_acc_C(y, s, m9);
        }
        for (int l = 0; l < 4; ++l) werr[k] = std::fmax(werr[k], std::fabs(gk[l] - g[l]) / gmax);
      }
      float Eb[4];
      if (k == 0) corner_dos_moments_finish_A(cs, V, m9, Eb);
      else if (k == 1) corner_dos_moments_finish_B(cs, V, M, Eb);
      else corner_dos_moments_finish_C(cs, V, m9, Eb);
      double d = 0;
      for (int i = 0; i < 4; ++i) {
        if (!std::isfinite(Eb[i])) d = INFINITY;
        d = std::fmax(d, std::fabs(Eb[i] - ref[i]));
      }
      double& slot = gerr[k][kind == 0 ? 0 : 1];
      slot = std::fmax(slot, d / scale);
      ++ranges[k];
    }
  }
  const char* names[3] = {"first", "middle", "third"};
  for (int k = 0; k < 3; ++k)
    std::printf("%s %ld %.6e %.6e %.6e\n", names[k], ranges[k], werr[k], gerr[k][0], gerr[k][1]);
  return 0;
}
