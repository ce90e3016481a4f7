// FP64 CPU oracle for the orbital-resolved tetrahedron density of states.
//
// Paper: D. Guterding and H. O. Jeschke, "An efficient GPU algorithm for tetrahedron-based
// Brillouin-zone integration" (arXiv:1710.10789), Sec. II.
//
// TEST INFRASTRUCTURE ONLY. This library is loaded only by the test suite, by the smoke check and by
// the benchmark's CPU-baseline leg. It shares no code, header, table or helper with the HIP path;
// the product library never links or loads it.
//
// What it computes, as plainly as possible:
//   DOS[j][m] = sum_cubes sum_{tetrahedra of Table I} sum_n sum_{l=1..4} b[n][m][k_l] dw_{n,l}/dE (E_j)
// i.e. eq. (tetracontriborbitalresolved) summed as in eq. (tetmethoorbitalresolved), with the corner
// weights w_l and their energy derivatives taken from the five energy cases of Sec. II.C, evaluated
// on the four corner energies of each tetrahedron sorted ascending (Sec. II.C).
//
// Readings of points the paper leaves open:
//  R1 cube corner label L = 1 + o1 + 2*o2 + 4*o3, o_a in {0,1} the offset along grid axis a
//     (axis 1 is the slowest array index, k = (i1*n2 + i2)*n3 + i3); Table I is used as printed.
//  R2 periodic grid of n1*n2*n3 cubes, so V_T/V_G = 1/(6*n1*n2*n3).
//  R3 E <= E1: zero; E1 < E <= E2: first case; E2 < E <= E3: second case; E3 < E < E4: third case;
//     E >= E4: weights V_T/(4V_G), derivatives zero.
//  R4 second case: the last term of dw3/dE is (C2+C3)/E32 (the printed C1+C3 is not the derivative
//     of the printed w3).
//  R5 third case: the lower-case e in w4 and dw4/dE is E.
//  R6 corner sort is stable (equal energies keep Table I order).
//  R7 point values on E_j = e0 + j*de, j = 0..ne-1; no spin factor.
//  R8 a tetrahedron-band with a non-finite corner energy contributes nothing.
//
// Susceptibility (the paper's stated future work, Sec. I and Sec. V; it prints no formulas): the
// orbital-resolved imaginary part of the bare (Lindhard) susceptibility at zero temperature for a
// momentum transfer q on the k-grid, as a spectral weight
//   S_m(q, w) = sum_cubes sum_{tetrahedra of Table I} sum_{n,n'} (1/V_G) integral over the tetrahedron of
//               W_m [theta(E_F - eps) theta(eps' - E_F) - theta(eps - E_F) theta(E_F - eps')] delta(w - (eps' - eps))
// with eps = eps_n(k), eps' = eps_n'(k + q) and W_m = b_mn(k) b_mn'(k + q), each the linear interpolant
// of its corner values within the tetrahedron (the linear tetrahedron method, as for the DOS), and
// the step functions applied exactly. Im chi_0(q, w) = -pi S(q, w) in the convention
// chi_0 = (1/N) sum [f(eps) - f(eps')] / (w + eps - eps' + i0). Evaluated by clipping each
// tetrahedron (in barycentric coordinates) by the two occupation half-spaces into sub-tetrahedra and
// summing, on each, the corner weights dw/dE of Sec. II.C with the difference energy eps' - eps in the
// role of the band energy and the sub-tetrahedron's share of V_T.
//
// Parity: pinned in the CPU test suite against closed forms and independent geometry (cross-section
// integrals of barycentric coordinates), derivative and normalisation identities, symmetries,
// degenerate limits, a separable-grid closed form, histogram convergence and finite differences.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------------------------
// Forward-mode dual number with four tangent directions (the four sorted corner energies).
struct Dual {
  double v;
  double d[4];
};

inline Dual mk(double v) { Dual r; r.v = v; r.d[0] = r.d[1] = r.d[2] = r.d[3] = 0.0; return r; }
inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v / b.v;
  for (int i = 0; i < 4; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + mk(b); }
inline Dual operator+(double a, const Dual& b) { return mk(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - mk(b); }
inline Dual operator-(double a, const Dual& b) { return mk(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * mk(b); }
inline Dual operator*(double a, const Dual& b) { return mk(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / mk(b); }
inline Dual operator/(double a, const Dual& b) { return mk(a) / b; }
inline double val(const Dual& a) { return a.v; }
inline double val(double a) { return a; }

template <class T> inline T lift(double x);
template <> inline double lift<double>(double x) { return x; }
template <> inline Dual lift<Dual>(double x) { return mk(x); }

// ---------------------------------------------------------------------------------------------
// Sec. II.C: integrated corner weights w_l(E) and their energy derivatives dw_l/dE for sorted corner
// energies e[0] <= e[1] <= e[2] <= e[3] (E1..E4 in the paper). V = V_T / (4 V_G).
// The formulas are written in the order and notation in which the paper lists them.
template <class T>
void corner_weights(const T e[4], double E, double V, T w[4], T g[4]) {
  const T& E1 = e[0];
  const T& E2 = e[1];
  const T& E3 = e[2];
  const T& E4 = e[3];
  if (E <= val(E1)) {  // energy below the tetrahedron: no contribution
    for (int l = 0; l < 4; ++l) { w[l] = lift<T>(0.0); g[l] = lift<T>(0.0); }
    return;
  }
  if (E >= val(E4)) {  // energy above the tetrahedron: constant weights, zero derivative
    for (int l = 0; l < 4; ++l) { w[l] = lift<T>(V); g[l] = lift<T>(0.0); }
    return;
  }
  if (E <= val(E2)) {  // E1 < E < E2
    const T E21 = E2 - E1, E31 = E3 - E1, E41 = E4 - E1;
    const T C = V * (E - E1) * (E - E1) * (E - E1) / (E21 * E31 * E41);
    const T dC = 3.0 * V * (E - E1) * (E - E1) / (E21 * E31 * E41);
    const T S = 1.0 / E21 + 1.0 / E31 + 1.0 / E41;
    w[0] = C * (4.0 - (E - E1) * S);
    g[0] = dC * (4.0 - (E - E1) * S) - C * S;
    const T Ej1[3] = {E21, E31, E41};
    for (int l = 1; l < 4; ++l) {
      w[l] = C * (E - E1) / Ej1[l - 1];
      g[l] = dC * (E - E1) / Ej1[l - 1] + C / Ej1[l - 1];
    }
    return;
  }
  if (E <= val(E3)) {  // E2 < E < E3
    const T E31 = E3 - E1, E32 = E3 - E2, E41 = E4 - E1, E42 = E4 - E2;
    const T C1 = V * (E - E1) * (E - E1) / (E31 * E41);
    const T dC1 = 2.0 * V * (E - E1) / (E31 * E41);
    const T C2 = V * (E - E1) * (E - E2) * (E3 - E) / (E31 * E32 * E41);
    const T dC2 = V / (E31 * E32 * E41) *
                  ((E - E1) * (E2 - E) + (E - E1) * (E3 - E) + (E - E2) * (E3 - E));
    const T C3 = V * (E - E2) * (E - E2) * (E4 - E) / (E32 * E41 * E42);
    const T dC3 = V * (E - E2) / (E32 * E41 * E42) * (2.0 * (E4 - E) + (E2 - E));
    w[0] = C1 + (C1 + C2) * (E3 - E) / E31 + (C1 + C2 + C3) * (E4 - E) / E41;
    g[0] = dC1 + (dC1 + dC2) * (E3 - E) / E31 - (C1 + C2) / E31 +
           (dC1 + dC2 + dC3) * (E4 - E) / E41 - (C1 + C2 + C3) / E41;
    w[1] = C1 + C2 + C3 + (C2 + C3) * (E3 - E) / E32 + C3 * (E4 - E) / E42;
    g[1] = dC1 + dC2 + dC3 + (dC2 + dC3) * (E3 - E) / E32 - (C2 + C3) / E32 +
           dC3 * (E4 - E) / E42 - C3 / E42;
    w[2] = (C1 + C2) * (E - E1) / E31 + (C2 + C3) * (E - E2) / E32;
    g[2] = (dC1 + dC2) * (E - E1) / E31 + (C1 + C2) / E31 +
           (dC2 + dC3) * (E - E2) / E32 + (C2 + C3) / E32;  // reading R4
    w[3] = (C1 + C2 + C3) * (E - E1) / E41 + C3 * (E - E2) / E42;
    g[3] = (dC1 + dC2 + dC3) * (E - E1) / E41 + (C1 + C2 + C3) / E41 +
           dC3 * (E - E2) / E42 + C3 / E42;
    return;
  }
  {  // E3 < E < E4
    const T E41 = E4 - E1, E42 = E4 - E2, E43 = E4 - E3;
    const T C = V * (E4 - E) * (E4 - E) * (E4 - E) / (E41 * E42 * E43);
    const T dC = -3.0 * V * (E4 - E) * (E4 - E) / (E41 * E42 * E43);
    const T E4j[3] = {E41, E42, E43};
    for (int l = 0; l < 3; ++l) {
      w[l] = V - C * (E4 - E) / E4j[l];
      g[l] = -1.0 * dC * (E4 - E) / E4j[l] + C / E4j[l];
    }
    const T S = 1.0 / E41 + 1.0 / E42 + 1.0 / E43;
    w[3] = V - C * (4.0 - S * (E4 - E));  // reading R5
    g[3] = -1.0 * dC * (4.0 - S * (E4 - E)) - C * S;
  }
}

// Table I, corner labels 1..8 of the six tetrahedra of an elemental cube.
const int kTable1[6][4] = {{1, 2, 3, 6}, {2, 3, 4, 6}, {1, 3, 5, 6}, {3, 4, 6, 8}, {3, 5, 6, 7}, {3, 6, 7, 8}};

// Reading R1: corner label -> grid offsets (o1, o2, o3).
inline void label_offsets(int label, int o[3]) {
  const int c = label - 1;
  o[0] = c & 1;
  o[1] = (c >> 1) & 1;
  o[2] = (c >> 2) & 1;
}

// Reading R6: stable ascending sort of four energies, keeping the original positions.
inline void sort4(const double in[4], double out[4], int perm[4]) {
  for (int i = 0; i < 4; ++i) { out[i] = in[i]; perm[i] = i; }
  for (int i = 1; i < 4; ++i) {
    const double v = out[i];
    const int p = perm[i];
    int k = i;
    while (k > 0 && out[k - 1] > v) { out[k] = out[k - 1]; perm[k] = perm[k - 1]; --k; }
    out[k] = v;
    perm[k] = p;
  }
}

struct Grid {
  int n1, n2, n3, nb, norb, ne;
  double e0, de;
  int64_t nk() const { return (int64_t)n1 * n2 * n3; }
  double energy(int j) const { return e0 + (double)j * de; }  // reading R7
};

bool grid_ok(const Grid& g) {
  return g.n1 >= 1 && g.n2 >= 1 && g.n3 >= 1 && g.nb >= 1 && g.norb >= 1 && g.ne >= 1 && std::isfinite(g.e0) &&
         std::isfinite(g.de) && g.de > 0.0;
}

// First grid index with E_j > lo (exact comparison), searched from a rounded guess.
int first_above(const Grid& g, double lo) {
  double guess = std::floor((lo - g.e0) / g.de);
  if (guess < 0.0) guess = 0.0;
  if (guess > (double)g.ne) guess = (double)g.ne;
  int j = (int)guess;
  while (j > 0 && g.energy(j - 1) > lo) --j;
  while (j < g.ne && g.energy(j) <= lo) ++j;
  return j;
}

// The k-point indices of the four corners of tetrahedron t of cube (i1, i2, i3), reading R1/R2.
inline void tet_kpoints(const Grid& g, int i1, int i2, int i3, int t, int64_t kk[4]) {
  for (int l = 0; l < 4; ++l) {
    int o[3];
    label_offsets(kTable1[t][l], o);
    const int64_t a = (i1 + o[0]) % g.n1, b = (i2 + o[1]) % g.n2, c = (i3 + o[2]) % g.n3;
    kk[l] = (a * g.n2 + b) * g.n3 + c;
  }
}

}  // namespace

extern "C" {

// Table I as 0-based corner slots s = o1 + 2*o2 + 4*o3 (reading R1), 24 ints.
void tetra_oracle_table(int out[24]) {
  for (int t = 0; t < 6; ++t)
    for (int l = 0; l < 4; ++l) out[4 * t + l] = kTable1[t][l] - 1;
}

// Corner weights w_l(E) and dw_l/dE of one tetrahedron with sorted energies (Sec. II.C);
// vol = V_T/V_G. The energies must be sorted ascending.
void tetra_oracle_corner_weights(const double e_sorted[4], double E, double vol, double w[4], double g[4]) {
  corner_weights<double>(e_sorted, E, vol / 4.0, w, g);
}

// Partial derivatives of the four dw_l/dE with respect to the four sorted energies:
// dg[4*l + i] = d(dw_l/dE)/dE_i, by forward-mode dual numbers through the same case formulas.
void tetra_oracle_corner_weights_grad(const double e_sorted[4], double E, double vol, double g[4], double dg[16]) {
  Dual e[4], w[4], gd[4];
  for (int i = 0; i < 4; ++i) { e[i] = mk(e_sorted[i]); e[i].d[i] = 1.0; }
  corner_weights<Dual>(e, E, vol / 4.0, w, gd);
  for (int l = 0; l < 4; ++l) {
    g[l] = gd[l].v;
    for (int i = 0; i < 4; ++i) dg[4 * l + i] = gd[l].d[i];
  }
}

// Contribution sum_l b_l dw_l/dE of one tetrahedron whose corner energies are given in any order
// (the corners are sorted here, carrying their b values along). vol = V_T/V_G.
double tetra_oracle_tet_dos(const double e[4], const double b[4], double E, double vol) {
  double es[4], w[4], g[4];
  int perm[4];
  sort4(e, es, perm);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(es[i])) return 0.0;
  corner_weights<double>(es, E, vol / 4.0, w, g);
  double s = 0.0;
  for (int l = 0; l < 4; ++l) s += b[perm[l]] * g[l];
  return s;
}

// Same for the integrated weights: sum_l b_l w_l(E).
double tetra_oracle_tet_nos(const double e[4], const double b[4], double E, double vol) {
  double es[4], w[4], g[4];
  int perm[4];
  sort4(e, es, perm);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(es[i])) return 0.0;
  corner_weights<double>(es, E, vol / 4.0, w, g);
  double s = 0.0;
  for (int l = 0; l < 4; ++l) s += b[perm[l]] * w[l];
  return s;
}

// Orbital-resolved DOS on the periodic grid (eq. tetmethoorbitalresolved).
//   eps  [nb][nk]        FP32 band energies (host memory)
//   w    [nb][norb][nk]  FP32 orbital weights b = |a|^2 (host memory)
//   dos  [ne][norb]      FP64 result, overwritten
// Only the energies inside each tetrahedron-band's open window (E1, E4) are visited; all other
// terms are exact zeros, so the sum equals the dense definition bit for bit.
// Returns the number of in-window (tetrahedron, band, energy) updates, or -1 on invalid arguments.
// Work is split into slabs of constant i1 with one FP64 partial per slab, reduced in slab order, so
// the result does not depend on the thread count.
long long tetra_oracle_dos(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne,
                           const float* eps, const float* w, double* dos, int nthreads) {
  const Grid g{n1, n2, n3, nb, norb, ne, e0, de};
  if (!grid_ok(g) || !eps || !w || !dos) return -1;
  const int64_t nk = g.nk();
  const double vol = 1.0 / (6.0 * (double)nk);  // reading R2
  const double V = vol / 4.0;
  const size_t nbins = (size_t)ne * norb;
  std::vector<double> partial((size_t)n1 * nbins, 0.0);
  std::vector<long long> counts(n1, 0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int i1 = 0; i1 < n1; ++i1) {
    double* acc = &partial[(size_t)i1 * nbins];
    long long cnt = 0;
    for (int i2 = 0; i2 < n2; ++i2)
      for (int i3 = 0; i3 < n3; ++i3)
        for (int t = 0; t < 6; ++t) {
          int64_t kk[4];
          tet_kpoints(g, i1, i2, i3, t, kk);
          for (int n = 0; n < nb; ++n) {
            double e[4], es[4];
            int perm[4];
            for (int l = 0; l < 4; ++l) e[l] = (double)eps[(int64_t)n * nk + kk[l]];
            sort4(e, es, perm);
            bool finite = true;
            for (int l = 0; l < 4; ++l) finite = finite && std::isfinite(es[l]);
            if (!finite) continue;  // reading R8
            for (int j = first_above(g, es[0]); j < ne; ++j) {
              const double E = g.energy(j);
              if (E >= es[3]) break;
              double wl[4], gl[4];
              corner_weights<double>(es, E, V, wl, gl);
              ++cnt;
              for (int m = 0; m < norb; ++m) {
                const float* wm = w + ((int64_t)n * norb + m) * nk;
                double s = 0.0;
                for (int l = 0; l < 4; ++l) s += (double)wm[kk[perm[l]]] * gl[l];
                acc[(size_t)j * norb + m] += s;
              }
            }
          }
        }
    counts[i1] = cnt;
  }
  long long total = 0;
  std::fill(dos, dos + nbins, 0.0);
  for (int i1 = 0; i1 < n1; ++i1) {
    total += counts[i1];
    const double* acc = &partial[(size_t)i1 * nbins];
    for (size_t q = 0; q < nbins; ++q) dos[q] += acc[q];
  }
  return total;
}

// Orbital-resolved number of states N[j][m] = sum_{tets, n, l} b[n][m][k_l] w_{n,l}(E_j) with the
// integrated weights of Sec. II.C (eq. BZintegral with X = b and f = step function at E_j).
// Dense over all energies (every tetrahedron below E_j contributes V_T/(4V_G) per corner), so meant
// for small grids. Same argument conventions as tetra_oracle_dos; returns 0, or -1 on bad input.
int tetra_oracle_nos(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne, const float* eps,
                     const float* w, double* nos, int nthreads) {
  const Grid g{n1, n2, n3, nb, norb, ne, e0, de};
  if (!grid_ok(g) || !eps || !w || !nos) return -1;
  const int64_t nk = g.nk();
  const double V = 1.0 / (6.0 * (double)nk) / 4.0;
  const size_t nbins = (size_t)ne * norb;
  std::vector<double> partial((size_t)n1 * nbins, 0.0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int i1 = 0; i1 < n1; ++i1) {
    double* acc = &partial[(size_t)i1 * nbins];
    for (int i2 = 0; i2 < n2; ++i2)
      for (int i3 = 0; i3 < n3; ++i3)
        for (int t = 0; t < 6; ++t) {
          int64_t kk[4];
          tet_kpoints(g, i1, i2, i3, t, kk);
          for (int n = 0; n < nb; ++n) {
            double e[4], es[4];
            int perm[4];
            for (int l = 0; l < 4; ++l) e[l] = (double)eps[(int64_t)n * nk + kk[l]];
            sort4(e, es, perm);
            bool finite = true;
            for (int l = 0; l < 4; ++l) finite = finite && std::isfinite(es[l]);
            if (!finite) continue;
            for (int j = 0; j < ne; ++j) {
              double wl[4], gl[4];
              corner_weights<double>(es, g.energy(j), V, wl, gl);
              for (int m = 0; m < norb; ++m) {
                const float* wm = w + ((int64_t)n * norb + m) * nk;
                double s = 0.0;
                for (int l = 0; l < 4; ++l) s += (double)wm[kk[perm[l]]] * wl[l];
                acc[(size_t)j * norb + m] += s;
              }
            }
          }
        }
  }
  std::fill(nos, nos + nbins, 0.0);
  for (int i1 = 0; i1 < n1; ++i1) {
    const double* acc = &partial[(size_t)i1 * nbins];
    for (size_t q = 0; q < nbins; ++q) nos[q] += acc[q];
  }
  return 0;
}

// Gradient of a scalar loss L(DOS) given G[j][m] = dL/dDOS[j][m]:
//   grad_w[n][m][k]  = dL/db[n][m][k]   (exact: DOS is linear in b)
//   grad_eps[n][k]   = dL/deps[n][k]    (through the sorted corner energies, mapped back to corners)
// Either output may be NULL; both are overwritten (FP64, host memory). The work is split over
// (band, slab of constant i1) tasks. A slab's cubes touch the k-points of planes i1 and i1 + 1, so
// the slabs run in phases (even i1, odd i1, and the last slab on its own when n1 is odd) in which no
// two tasks touch the same output element: every element is summed in the same order whatever the
// thread count. Returns 0, or -1 on invalid arguments.
int tetra_oracle_dos_backward(int n1, int n2, int n3, int nb, int norb, double e0, double de, int ne,
                              const float* eps, const float* w, const double* G, double* grad_eps,
                              double* grad_w, int nthreads) {
  const Grid g{n1, n2, n3, nb, norb, ne, e0, de};
  if (!grid_ok(g) || !eps || !w || !G) return -1;
  const int64_t nk = g.nk();
  const double V = 1.0 / (6.0 * (double)nk) / 4.0;
  if (grad_eps) std::fill(grad_eps, grad_eps + (size_t)nb * nk, 0.0);
  if (grad_w) std::fill(grad_w, grad_w + (size_t)nb * norb * nk, 0.0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  const bool odd = n1 > 1 && (n1 % 2) == 1;
  const int last = odd ? n1 - 1 : n1;  // slabs below `last` go by parity, the odd last one alone
  for (int phase = 0; phase < (odd ? 3 : 2); ++phase) {
    std::vector<int> slabs;
    if (phase < 2) {
      for (int i1 = phase; i1 < last; i1 += 2) slabs.push_back(i1);
    } else {
      slabs.push_back(n1 - 1);
    }
    const int ntask = nb * (int)slabs.size();
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int task = 0; task < ntask; ++task) {
      const int n = task / (int)slabs.size();
      const int i1 = slabs[task % slabs.size()];
      std::vector<double> gb(4 * (size_t)norb);
      for (int i2 = 0; i2 < n2; ++i2)
        for (int i3 = 0; i3 < n3; ++i3)
          for (int t = 0; t < 6; ++t) {
            int64_t kk[4];
            tet_kpoints(g, i1, i2, i3, t, kk);
            double e[4], es[4];
            int perm[4];
            for (int l = 0; l < 4; ++l) e[l] = (double)eps[(int64_t)n * nk + kk[l]];
            sort4(e, es, perm);
            bool finite = true;
            for (int l = 0; l < 4; ++l) finite = finite && std::isfinite(es[l]);
            if (!finite) continue;
            double ge[4] = {0, 0, 0, 0};
            std::fill(gb.begin(), gb.end(), 0.0);
            Dual ed[4];
            for (int i = 0; i < 4; ++i) { ed[i] = mk(es[i]); ed[i].d[i] = 1.0; }
            for (int j = first_above(g, es[0]); j < ne; ++j) {
              const double E = g.energy(j);
              if (E >= es[3]) break;
              Dual wl[4], gl[4];
              corner_weights<Dual>(ed, E, V, wl, gl);
              const double* Gj = G + (size_t)j * norb;
              for (int l = 0; l < 4; ++l) {
                double sl = 0.0;
                for (int m = 0; m < norb; ++m) {
                  const double b = (double)w[((int64_t)n * norb + m) * nk + kk[perm[l]]];
                  gb[(size_t)l * norb + m] += Gj[m] * gl[l].v;
                  sl += Gj[m] * b;
                }
                for (int i = 0; i < 4; ++i) ge[i] += sl * gl[l].d[i];
              }
            }
            for (int l = 0; l < 4; ++l) {
              const int64_t k = kk[perm[l]];
              if (grad_eps) grad_eps[(int64_t)n * nk + k] += ge[l];
              if (grad_w)
                for (int m = 0; m < norb; ++m) grad_w[((int64_t)n * norb + m) * nk + k] += gb[(size_t)l * norb + m];
            }
          }
    }
  }
  return 0;
}

}  // extern "C"

namespace {

// A tetrahedron given by the barycentric coordinates (with respect to one tetrahedron of the grid) of
// its four vertices.
struct BaryTet {
  double v[4][4];
};

// Volume of a sub-tetrahedron as a fraction of the parent's: |det| of its edge vectors in the
// coordinates (lambda_1, lambda_2, lambda_3), which map the parent onto the unit simplex.
double bary_volume_fraction(const BaryTet& t) {
  double a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) a[i][c] = t.v[i + 1][c + 1] - t.v[0][c + 1];
  const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  return std::fabs(det);
}

// The part of tetrahedron `in` where the linear function f (values fc at the parent's corners) is
// <= 0, as at most three tetrahedra appended to out. One vertex inside: the corner tetrahedron cut off
// by the plane f = 0; two or three inside: a triangular prism (end triangles parallel to the cut),
// split into three tetrahedra.
void clip_halfspace(const BaryTet& in, const double fc[4], std::vector<BaryTet>& out) {
  double f[4];
  for (int i = 0; i < 4; ++i) {
    f[i] = 0.0;
    for (int c = 0; c < 4; ++c) f[i] += in.v[i][c] * fc[c];
  }
  int ins[4], outs[4], ni = 0, no = 0;
  for (int i = 0; i < 4; ++i) {
    if (f[i] <= 0.0) ins[ni++] = i;
    else outs[no++] = i;
  }
  if (ni == 0) return;
  if (ni == 4) {
    out.push_back(in);
    return;
  }
  // point on the edge from inside vertex a to outside vertex b where f = 0
  auto cut = [&](int a, int b, double p[4]) {
    const double t = f[a] / (f[a] - f[b]);
    for (int c = 0; c < 4; ++c) p[c] = in.v[a][c] + t * (in.v[b][c] - in.v[a][c]);
  };
  auto prism = [&](const double* p0, const double* p1, const double* p2, const double* q0, const double* q1,
                   const double* q2) {
    const double* tets[3][4] = {{p0, p1, p2, q2}, {p0, p1, q1, q2}, {p0, q0, q1, q2}};
    for (int k = 0; k < 3; ++k) {
      BaryTet t;
      for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 4; ++c) t.v[i][c] = tets[k][i][c];
      out.push_back(t);
    }
  };
  if (ni == 1) {
    BaryTet t;
    const int a = ins[0];
    for (int c = 0; c < 4; ++c) t.v[0][c] = in.v[a][c];
    for (int k = 0; k < 3; ++k) cut(a, outs[k], t.v[k + 1]);
    out.push_back(t);
  } else if (ni == 2) {
    const int a = ins[0], b = ins[1], c = outs[0], d = outs[1];
    double ac[4], ad[4], bc[4], bd[4];
    cut(a, c, ac);
    cut(a, d, ad);
    cut(b, c, bc);
    cut(b, d, bd);
    prism(in.v[a], ac, ad, in.v[b], bc, bd);
  } else {
    const int a = ins[0], b = ins[1], c = ins[2], d = outs[0];
    double ad[4], bd[4], cd[4];
    cut(a, d, ad);
    cut(b, d, bd);
    cut(c, d, cd);
    prism(in.v[a], in.v[b], in.v[c], ad, bd, cd);
  }
}

// Sub-tetrahedra of the region {f1 <= 0} and {f2 <= 0} of the parent tetrahedron.
void clip_two(const double f1[4], const double f2[4], std::vector<BaryTet>& out) {
  BaryTet whole;
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 4; ++c) whole.v[i][c] = i == c ? 1.0 : 0.0;
  std::vector<BaryTet> first;
  clip_halfspace(whole, f1, first);
  for (const BaryTet& t : first) clip_halfspace(t, f2, out);
}

// Spectral weight of one tetrahedron at transfer energy E (see the header): corner values eps, eps'
// and W in any order, Fermi energy ef, vol = V_T/V_G.
double tet_chi(const double e[4], const double ep[4], const double W[4], double ef, double E, double vol) {
  double total = 0.0;
  for (int region = 0; region < 2; ++region) {
    // region 0: eps <= E_F <= eps' (sign +1); region 1: eps' <= E_F <= eps (sign -1)
    double f1[4], f2[4];
    for (int c = 0; c < 4; ++c) {
      f1[c] = region == 0 ? e[c] - ef : ef - e[c];
      f2[c] = region == 0 ? ef - ep[c] : ep[c] - ef;
    }
    std::vector<BaryTet> subs;
    clip_two(f1, f2, subs);
    for (const BaryTet& t : subs) {
      const double frac = bary_volume_fraction(t);
      if (!(frac > 0.0)) continue;
      double d[4], w[4];
      for (int i = 0; i < 4; ++i) {
        d[i] = 0.0;
        w[i] = 0.0;
        for (int c = 0; c < 4; ++c) {
          d[i] += t.v[i][c] * (ep[c] - e[c]);
          w[i] += t.v[i][c] * W[c];
        }
      }
      const double v = tetra_oracle_tet_dos(d, w, E, vol * frac);
      total += region == 0 ? v : -v;
    }
  }
  return total;
}

// Adds one tetrahedron-band-pair's spectral weight at every grid energy inside its sub-tetrahedra's
// windows: acc[j][m] += S_m(w_j) for the corner weights Wc[c][m] (norb per corner). Returns the
// number of (sub-tetrahedron, energy) pairs visited, i.e. with the energy strictly inside the
// sub-tetrahedron's range of eps' - eps.
int chi_accumulate(const Grid& g, const double e[4], const double ep[4], const double* Wc, double ef, double vol,
                   double* acc) {
  const int norb = g.norb;
  int nsub = 0;
  for (int region = 0; region < 2; ++region) {
    double f1[4], f2[4];
    for (int c = 0; c < 4; ++c) {
      f1[c] = region == 0 ? e[c] - ef : ef - e[c];
      f2[c] = region == 0 ? ef - ep[c] : ep[c] - ef;
    }
    const double sign = region == 0 ? 1.0 : -1.0;
    std::vector<BaryTet> subs;
    clip_two(f1, f2, subs);
    for (const BaryTet& t : subs) {
      const double frac = bary_volume_fraction(t);
      if (!(frac > 0.0)) continue;
      double d[4], ds[4];
      int perm[4];
      for (int i = 0; i < 4; ++i) {
        d[i] = 0.0;
        for (int c = 0; c < 4; ++c) d[i] += t.v[i][c] * (ep[c] - e[c]);
      }
      sort4(d, ds, perm);
      for (int j = first_above(g, ds[0]); j < g.ne; ++j) {
        const double E = g.energy(j);
        if (E >= ds[3]) break;
        double wl[4], gl[4];
        corner_weights<double>(ds, E, vol * frac / 4.0, wl, gl);
        ++nsub;
        for (int m = 0; m < norb; ++m) {
          double s = 0.0;
          for (int l = 0; l < 4; ++l) {
            double wv = 0.0;  // W at sub-tetrahedron vertex perm[l]
            for (int c = 0; c < 4; ++c) wv += t.v[perm[l]][c] * Wc[c * norb + m];
            s += wv * gl[l];
          }
          acc[(size_t)j * norb + m] += sign * s;
        }
      }
    }
  }
  return nsub;
}

}  // namespace

extern "C" {

// One tetrahedron's contribution to the susceptibility spectral weight S (see the header) at transfer
// energy E: corner energies e (band n at k), ep (band n' at k + q), interpolated weight W, Fermi
// energy ef; vol = V_T/V_G. Corners in any order.
double tetra_oracle_tet_chi(const double e[4], const double ep[4], const double W[4], double ef, double E,
                            double vol) {
  for (int c = 0; c < 4; ++c)
    if (!std::isfinite(e[c]) || !std::isfinite(ep[c])) return 0.0;
  return tet_chi(e, ep, W, ef, E, vol);
}

// Orbital-resolved susceptibility spectral weight on the periodic grid for the transfer q = (q1, q2, q3)
// in grid steps (any sign, periodic): out[j][m] = S_m(q, w0 + j*dw) (header), FP64, overwritten.
//   eps [nb][nk] FP32, w [nb][norb][nk] FP32 (b = |a|^2), host memory.
// Sums over every band pair (n, n'). A tetrahedron with a non-finite corner energy in either band
// contributes nothing. Slabs of constant i1 with one partial each, reduced in slab order. Returns
// the number of (sub-tetrahedron, band pair, energy) updates inside the sub-tetrahedra's open
// windows, or -1 on invalid arguments.
long long tetra_oracle_chi(int n1, int n2, int n3, int nb, int norb, int q1, int q2, int q3, double ef,
                           double w0, double dw, int nw, const float* eps, const float* w, double* out,
                           int nthreads) {
  const Grid g{n1, n2, n3, nb, norb, nw, w0, dw};
  if (!grid_ok(g) || !eps || !w || !out || !std::isfinite(ef)) return -1;
  const int64_t nk = g.nk();
  const double vol = 1.0 / (6.0 * (double)nk);
  const size_t nbins = (size_t)nw * norb;
  const int s1 = ((q1 % n1) + n1) % n1, s2 = ((q2 % n2) + n2) % n2, s3 = ((q3 % n3) + n3) % n3;
  std::vector<double> partial((size_t)n1 * nbins, 0.0);
  std::vector<long long> counts(n1, 0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int i1 = 0; i1 < n1; ++i1) {
    double* acc = &partial[(size_t)i1 * nbins];
    long long nsub = 0;
    std::vector<double> Wc(4 * (size_t)norb);
    for (int i2 = 0; i2 < n2; ++i2)
      for (int i3 = 0; i3 < n3; ++i3)
        for (int t = 0; t < 6; ++t) {
          int64_t kk[4], kq[4];
          tet_kpoints(g, i1, i2, i3, t, kk);
          for (int l = 0; l < 4; ++l) {
            const int64_t a = kk[l] / ((int64_t)n2 * n3), b = (kk[l] / n3) % n2, c = kk[l] % n3;
            kq[l] = (((a + s1) % n1) * n2 + (b + s2) % n2) * n3 + (c + s3) % n3;
          }
          for (int n = 0; n < nb; ++n)
            for (int np = 0; np < nb; ++np) {
              double e[4], ep[4];
              bool finite = true;
              for (int l = 0; l < 4; ++l) {
                e[l] = (double)eps[(int64_t)n * nk + kk[l]];
                ep[l] = (double)eps[(int64_t)np * nk + kq[l]];
                finite = finite && std::isfinite(e[l]) && std::isfinite(ep[l]);
              }
              if (!finite) continue;
              for (int l = 0; l < 4; ++l)
                for (int m = 0; m < norb; ++m)
                  Wc[(size_t)l * norb + m] = (double)w[((int64_t)n * norb + m) * nk + kk[l]] *
                                             (double)w[((int64_t)np * norb + m) * nk + kq[l]];
              nsub += chi_accumulate(g, e, ep, Wc.data(), ef, vol, acc);
            }
        }
    counts[i1] = nsub;
  }
  long long total = 0;
  std::fill(out, out + nbins, 0.0);
  for (int i1 = 0; i1 < n1; ++i1) {
    total += counts[i1];
    const double* acc = &partial[(size_t)i1 * nbins];
    for (size_t q = 0; q < nbins; ++q) out[q] += acc[q];
  }
  return total;
}

}  // extern "C"
