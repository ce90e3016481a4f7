// Driver for the sanitizer build of the FP64 oracle (oracle/tetra_oracle.cpp compiled with
// -fsanitize=address,undefined by tests/test_sanitizers_host.py). Test harness only.
//
// Calls every exported oracle function on small seeded inputs (ragged grids, a band with non-finite
// energies, degenerate corners, several thread counts) and on invalid arguments (the -1 returns),
// so that an out-of-bounds access, a use of uninitialised memory through UB, a signed overflow or a
// leak stops the run with the sanitizer's report. Prints "ok <checksum>" at the end.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
void tetra_oracle_table(int out[24]);
void tetra_oracle_corner_weights(const double e_sorted[4], double E, double vol, double w[4], double g[4]);
void tetra_oracle_corner_weights_grad(const double e_sorted[4], double E, double vol, double g[4], double dg[16]);
double tetra_oracle_tet_dos(const double e[4], const double b[4], double E, double vol);
double tetra_oracle_tet_nos(const double e[4], const double b[4], double E, double vol);
long long tetra_oracle_dos(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne, const float* eps,
                           const float* w, double* dos, int nthreads);
int tetra_oracle_nos(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne, const float* eps,
                     const float* w, double* nos, int nthreads);
int tetra_oracle_dos_backward(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne,
                              const float* eps, const float* w, const double* G, double* grad_eps, double* grad_w,
                              int nthreads);
double tetra_oracle_tet_chi(const double e[4], const double ep[4], const double W[4], double ef, double E,
                            double vol);
long long tetra_oracle_chi(int n1, int n2, int n3, int nb, int norb, int q1, int q2, int q3, double ef, double w0,
                           double dw, int nw, const float* eps, const float* w, double* out, int nthreads);
}

int main() {
  std::mt19937 rng(11);
  std::uniform_real_distribution<double> U(-1.0, 1.0), P(0.0, 1.0);
  double sum = 0.0;
  int table[24];
  tetra_oracle_table(table);
  for (int v : table) sum += v;
  // single tetrahedra: generic, degenerate (equal corners) and energies outside the range
  for (int it = 0; it < 2000; ++it) {
    double e[4], b[4], ep[4], W[4], w[4], g[4], dg[16];
    for (int c = 0; c < 4; ++c) {
      e[c] = U(rng);
      ep[c] = U(rng);
      b[c] = P(rng);
      W[c] = P(rng);
    }
    if (it % 4 == 1) e[1] = e[0];
    if (it % 4 == 2) e[3] = e[2] = e[1];
    const double E = 1.5 * U(rng);
    double es[4] = {e[0], e[1], e[2], e[3]};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (es[j] < es[i]) std::swap(es[i], es[j]);
    tetra_oracle_corner_weights(es, E, 0.25, w, g);
    tetra_oracle_corner_weights_grad(es, E, 0.25, g, dg);
    sum += w[0] + g[3] + dg[5];
    sum += tetra_oracle_tet_dos(e, b, E, 0.25) + tetra_oracle_tet_nos(e, b, E, 0.25);
    sum += tetra_oracle_tet_chi(e, ep, W, 0.1 * U(rng), E, 0.25);
  }
  // grids: ragged sides, one band all NaN, several thread counts
  const int grids[3][3] = {{3, 2, 5}, {4, 4, 4}, {1, 3, 2}};
  for (const auto& gr : grids) {
    const int n1 = gr[0], n2 = gr[1], n3 = gr[2], nb = 3, norb = 2, ne = 37;
    const int nk = n1 * n2 * n3;
    std::vector<float> eps((size_t)nb * nk), w((size_t)nb * norb * nk);
    for (auto& x : eps) x = (float)U(rng);
    for (auto& x : w) x = (float)P(rng);
    for (int k = 0; k < nk; ++k) eps[(size_t)nk + k] = NAN;  // band 1
    std::vector<double> dos((size_t)ne * norb), nos((size_t)ne * norb), G((size_t)ne * norb);
    std::vector<double> ge((size_t)nb * nk), gw((size_t)nb * norb * nk), chi((size_t)ne * norb);
    for (auto& x : G) x = U(rng);
    for (int threads : {1, 3}) {
      if (tetra_oracle_dos(n1, n2, n3, nb, norb, -1.2, 0.07, ne, eps.data(), w.data(), dos.data(), threads) < 0)
        return 2;
      if (tetra_oracle_nos(n1, n2, n3, nb, norb, -1.2, 0.07, ne, eps.data(), w.data(), nos.data(), threads) != 0)
        return 3;
      if (tetra_oracle_dos_backward(n1, n2, n3, nb, norb, -1.2, 0.07, ne, eps.data(), w.data(), G.data(), ge.data(),
                                    gw.data(), threads) != 0)
        return 4;
      if (tetra_oracle_chi(n1, n2, n3, nb, norb, 1, -1, 2, 0.05, -2.0, 0.11, ne, eps.data(), w.data(), chi.data(),
                           threads) < 0)
        return 5;
      for (double x : dos) sum += x;
      for (double x : nos) sum += x;
      for (double x : ge) sum += x;
      for (double x : gw) sum += x;
      for (double x : chi) sum += x;
    }
  }
  // invalid arguments are rejected before any work
  std::vector<float> one(64, 0.5f);
  std::vector<double> out(64);
  if (tetra_oracle_dos(0, 2, 2, 1, 1, 0.0, 0.1, 4, one.data(), one.data(), out.data(), 1) != -1) return 6;
  if (tetra_oracle_dos(2, 2, 2, 1, 1, 0.0, -0.1, 4, one.data(), one.data(), out.data(), 1) != -1) return 7;
  if (tetra_oracle_nos(2, 2, 2, 1, 1, 0.0, 0.1, 0, one.data(), one.data(), out.data(), 1) != -1) return 8;
  if (tetra_oracle_dos_backward(2, 2, 2, 1, 1, 0.0, 0.1, 4, nullptr, one.data(), out.data(), out.data(), out.data(),
                                1) != -1)
    return 9;
  if (tetra_oracle_chi(2, 2, 2, 1, 1, 0, 0, 0, NAN, 0.0, 0.1, 4, one.data(), one.data(), out.data(), 1) != -1)
    return 10;
  if (!std::isfinite(sum)) return 11;
  std::printf("ok %.6e\n", sum);
  return 0;
}
