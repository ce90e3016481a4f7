/*
 * tetra.h -- C ABI of the MI355X (gfx950) tetrahedron-method density-of-states library.
 *
 * Paper: D. Guterding and H. O. Jeschke, "An efficient GPU algorithm for tetrahedron-based
 * Brillouin-zone integration", arXiv:1710.10789.
 *
 * What the library computes (Sec. II, eqs. dos, tetracontriborbitalresolved, tetmethoorbitalresolved):
 *
 *   DOS[j][m] = sum over cubes of the periodic k-grid, over the six tetrahedra of Table I, over bands
 *               n and over the four corners l of  b[n][m][k_l] * dw_{n,l}/dE (E_j)
 *
 * with the corner weights of the five energy cases of Sec. II.C, evaluated on the four corner
 * energies of each tetrahedron-band sorted ascending, and E_j = e0 + j*de (an equidistant energy
 * grid, Sec. IV.A). The inputs follow the paper's statement of the problem: band energies E_n(k)
 * and orbital weights b_mn(k) = |a^m_n(k)|^2 (eq. matrixelements) on the k-grid, stored as
 * linearised arrays (Sec. III.B), or the amplitudes a^m_n(k) themselves. Besides the DOS and its
 * adjoint: the orbital-resolved number of states with the integrated weights w_{n,l} (eq.
 * BZintegral), the bin-averaged DOS derived from it, and the orbital-resolved spectral weight of the
 * bare susceptibility (its imaginary part at zero temperature; Sec. I and V name susceptibilities as
 * the method's next use) by the same corner weights applied to the difference energy.
 *
 * Conventions shared by every entry point:
 *  - k-grid: n1 x n2 x n3 points, periodic, k = (i1*n2 + i2)*n3 + i3 (i3 fastest). Every grid point
 *    is the corner 000 of one elemental cube. Corner label L of Table I (1..8) sits at offset
 *    (o1, o2, o3) with L = 1 + o1 + 2*o2 + 4*o3 along axes (1, 2, 3).
 *  - V_T/V_G = 1 / (6*n1*n2*n3); the DOS is per energy unit, per k-point (unit cell) and orbital;
 *    no spin factor.
 *  - Energy cases: E <= E1 and E >= E4 contribute nothing; (E1,E2], (E2,E3], (E3,E4) use the three
 *    formula sets of Sec. II.C (the middle-case dw3/dE taken as the derivative of the printed w3).
 *  - A tetrahedron-band with a non-finite corner energy contributes nothing.
 *  - All array pointers are DEVICE pointers (memory from hipMalloc or a caching allocator on top of
 *    it); the caller owns every buffer. Inputs are read-only; outputs are overwritten, never
 *    accumulated. Calls are asynchronous on `stream` (a hipStream_t; NULL means the null stream) and
 *    never synchronise the device.
 *  - Errors: every entry point returns a tetra_status and never aborts or throws. Argument
 *    validation happens on the host before any HIP call; on a validation failure nothing is
 *    launched and outputs are untouched. A failed launch returns TETRA_ERR_HIP (the HIP error text
 *    is available from tetra_last_hip_error()).
 *  - Layouts are structure-of-arrays: eps[nb][nk], w[nb][norb][nk], dos[ne][norb].
 *  - Limits: norb in 1..16 (the paper's largest realistic model, Sec. III.B); n1,n2,n3,nb,ne >= 1;
 *    nb*nk < 2^31 and nb*norb*nk < 2^31; ne <= 2^22; finite e0; finite de > 0.
 */
#ifndef TETRA_H
#define TETRA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TETRA_OK = 0,
  TETRA_ERR_ARG = -1,         /* null pointer, bad size, bad grid, bad flag */
  TETRA_ERR_UNSUPPORTED = -2, /* valid request the library does not implement (e.g. norb > 16) */
  TETRA_ERR_WORKSPACE = -3,   /* workspace missing or too small */
  TETRA_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed */
  TETRA_ERR_SCRATCH = -5      /* problem too large for the static scratch of tetra_dos_forward_noalloc */
} tetra_status;

/* Storage type of the orbital weights w. */
typedef enum {
  TETRA_W_F32 = 0, /* float w[nb][norb][nk]; w_scale must be NULL */
  TETRA_W_F16 = 1, /* _Float16/half w[nb][norb][nk]; value = w * w_scale[n] (per band) */
  TETRA_W_C32 = 2  /* complex amplitudes a^m_n(k) as interleaved float pairs (re, im), w[nb][norb][nk][2];
                      value b = re^2 + im^2 (eq. matrixelements), formed in the kernels as the paper's
                      kernel does from eigenvector components; w_scale must be NULL */
} tetra_wtype;

/* Flag bits. */
enum {
  /* Exact (compensated) accumulation of the forward DOS. Every workgroup sums its contributions
   * exactly in a 64-bit fixed point of its own (LDS); with this flag the cross-workgroup sum is
   * exact as well: a bound pass fixes one common 64-bit fixed point from the largest per-workgroup
   * bound exponent (an integer maximum), each workgroup's exact sums are rounded once to it and
   * added with integer atomics. What remains is the FP32 rounding of each contribution and one
   * rounding per workgroup and element to the common unit, 2^(L-62) of the largest workgroup bound
   * (rounded up to a power of two) for 2^L >= the number of (tile, band) workgroups. The result is
   * bitwise reproducible, independent of the order in which workgroups run. Needs a
   * workspace (tetra_dos_forward_ws). The adjoint sums at most eight partial values per output
   * element and ignores the flag. */
  TETRA_EXACT = 1u,
  TETRA_KAHAN = TETRA_EXACT, /* former name of TETRA_EXACT (same bit) */
  /* Bitwise reproducible result. tetra_dos_forward_ws takes the exact path of TETRA_EXACT for it
   * (same workspace, same result); tetra_dos_backward_ws with its two-phase output (a workspace)
   * is deterministic as well. The atomic path of tetra_dos_backward, tetra_dos_batched and the
   * number-of-states calls do not offer it (TETRA_ERR_UNSUPPORTED). */
  TETRA_DETERMINISTIC = 2u,
  /* Bits 8..11 select the tile shape of the forward and adjoint kernels (0 = default); an autotuner
   * picks it per problem class. Shapes are TX x TY x TZ cubes along grid axes (1, 2, 3):
   * 0: 4x4x16, 1: 8x8x4, 2: 4x8x8, 3: 8x4x8, 4: 4x16x4, 5: 16x4x4. */
  TETRA_TILE_MASK = 0xF00u
};
#define TETRA_TILE(v) (((unsigned)(v) & 0xFu) << 8)

/* Problem descriptor (host memory). */
typedef struct {
  int n1, n2, n3; /* periodic k-grid, each >= 1 */
  int nb;         /* bands, >= 1 */
  int norb;       /* orbitals, 1..16 */
  float e0, de;   /* energy grid E_j = e0 + j*de, de > 0 */
  int ne;         /* number of energies, >= 1 */
} tetra_desc;

/*
 * Orbital-resolved DOS (Sec. II.C, eq. tetmethoorbitalresolved).
 *   d        host descriptor
 *   eps      device, float [nb][nk]        band energies E_n(k)
 *   w        device, [nb][norb][nk]        orbital weights b_mn(k), or amplitudes a^m_n(k) (type by wtype)
 *   wtype    TETRA_W_F32, TETRA_W_F16 or TETRA_W_C32
 *   w_scale  device, float [nb]            per-band scale for TETRA_W_F16, else NULL
 *   dos      device, float [ne][norb]      result, overwritten
 *   flags    TETRA_TILE(shape) or 0; TETRA_EXACT and TETRA_DETERMINISTIC need a workspace and give
 *            TETRA_ERR_WORKSPACE here (use tetra_dos_forward_ws)
 *   stream   hipStream_t
 * Allocates nothing. Same as tetra_dos_forward_ws with no workspace.
 */
tetra_status tetra_dos_forward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                               const float* w_scale, float* dos, unsigned flags, void* stream);

/*
 * Bytes of device workspace tetra_dos_forward_ws needs for these flags: 256 + 8*ne*norb with
 * TETRA_EXACT or TETRA_DETERMINISTIC (the largest bound exponent, then one 64-bit fixed-point sum
 * per output element), 0 without them and for invalid arguments.
 */
size_t tetra_dos_forward_workspace(const tetra_desc* d, unsigned flags);

/*
 * tetra_dos_forward with a caller-owned workspace for the exact accumulation (TETRA_EXACT,
 * TETRA_DETERMINISTIC): device memory of at least tetra_dos_forward_workspace(d, flags) bytes,
 * 16-byte aligned (TETRA_ERR_ARG otherwise), contents ignored and overwritten, not to be used by
 * anything else until the work on the stream ends. Without those flags the workspace is not used
 * and may be NULL; with them a missing or short workspace gives TETRA_ERR_WORKSPACE. The exact
 * path is four launches (set-up, bound pass, main pass, conversion), all plain kernels, so a call
 * can be captured in a HIP graph. Allocates nothing.
 */
tetra_status tetra_dos_forward_ws(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                  const float* w_scale, float* dos, unsigned flags, void* workspace,
                                  size_t ws_bytes, void* stream);

/*
 * Largest ne*norb of an exact or deterministic call of tetra_dos_forward_noalloc: its static scratch
 * holds 256 + 8*TETRA_NOALLOC_MAX_BINS bytes (2 MiB + 256) per device.
 */
#define TETRA_NOALLOC_MAX_BINS 262144

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): tetra_dos_forward_ws with the exact path's workspace taken from a
 * static device array of the library instead of the caller. Same arguments, flags and result as
 * tetra_dos_forward_ws (the caller still passes eps, w, w_scale and dos). With TETRA_EXACT or
 * TETRA_DETERMINISTIC, ne*norb above TETRA_NOALLOC_MAX_BINS gives TETRA_ERR_SCRATCH before any HIP
 * call; without them nothing of the scratch is used (the plain forward).
 *
 * The scratch is file-scope device memory that each device holds from the library's first call on
 * it until the process ends; its device address is looked up once per device on that first call
 * (hipGetSymbolAddress), so make the first call on a device outside graph capture. Every call on a
 * device shares that device's one scratch: each call clears what must start at zero (with a kernel,
 * no memset) and the scratch keeps the last call's contents afterwards, so exact calls that overlap
 * on one device (concurrent streams, host threads, or graph replays in flight together) race and give
 * wrong results; serialise them. Calls no hipMalloc, hipFree or allocating routine.
 */
tetra_status tetra_dos_forward_noalloc(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                       const float* w_scale, float* dos, unsigned flags, void* stream);

/*
 * Adjoint of tetra_dos_forward for a scalar loss L with G = dL/dDOS (not in the paper; the
 * derivative of the same sum with respect to its inputs).
 *   grad_dos  device, float [ne][norb]     G
 *   grad_eps  device, float [nb][nk]       dL/deps, overwritten; may be NULL
 *   grad_w    device, float [nb][norb][nk] dL/dw (always FP32, of the dequantised weights),
 *                                           overwritten; may be NULL. For TETRA_W_C32 it is
 *                                           float [nb][norb][nk][2]: dL/d(re a), dL/d(im a)
 *                                           = 2 (re a, im a) dL/db, interleaved like the input
 *   flags     TETRA_TILE(shape) or 0; TETRA_EXACT is accepted and ignored (each output element sums at
 *             most eight partial values); TETRA_DETERMINISTIC gives TETRA_ERR_UNSUPPORTED here (points
 *             on the boundary of a tile are summed with global float atomics, in no fixed order; the
 *             two-phase output of tetra_dos_backward_ws is deterministic)
 * At least one of grad_eps, grad_w must be non-NULL. Where an energy E_j equals a corner energy the
 * loss is not differentiable; the one-sided value of the case containing E_j is returned.
 * Allocates nothing. Same as tetra_dos_backward_ws with no workspace.
 */
tetra_status tetra_dos_backward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                const float* w_scale, const float* grad_dos, float* grad_eps,
                                float* grad_w, unsigned flags, void* stream);

/*
 * Bytes of device workspace for the two-phase output of tetra_dos_backward_ws: 4 (norb + 1) F nb T,
 * with T the tiles of the grid and F the face points of one tile (for tile shape (a, b, c):
 * 2 (b+1)(c+1) + 2 (a-1)(c+1) + 2 (a-1)(b-1)). Returns 0 where the two-phase output does not apply
 * (a grid side that is not a multiple of the tile's, or only one tile along an axis) and for invalid
 * arguments. flags as for tetra_dos_backward_ws (the tile shape matters).
 */
size_t tetra_dos_backward_workspace(const tetra_desc* d, unsigned flags);

/*
 * tetra_dos_backward with a caller-owned workspace (device memory of at least
 * tetra_dos_backward_workspace(d, flags) bytes, 16-byte aligned (TETRA_ERR_ARG otherwise), contents
 * ignored and overwritten, not used after the work on the stream ends). Each tile writes the partial sums of its boundary points to its own
 * slots with plain stores, and a second pass adds the 2 to 8 partials of every boundary grid point in
 * a fixed order: no zero-fill of the outputs, no atomics, and the gradients are bitwise the same from
 * run to run, so TETRA_DETERMINISTIC is accepted here. workspace NULL: the atomic path of
 * tetra_dos_backward (TETRA_DETERMINISTIC then gives TETRA_ERR_UNSUPPORTED). A workspace where the
 * two-phase output does not apply, or ws_bytes below the size, gives TETRA_ERR_WORKSPACE.
 * Allocates nothing.
 */
tetra_status tetra_dos_backward_ws(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                   const float* w_scale, const float* grad_dos, float* grad_eps, float* grad_w,
                                   unsigned flags, void* workspace, size_t ws_bytes, void* stream);

/*
 * Orbital-resolved number of states (eq. BZintegral with X = b of eq. matrixelements and the step
 * occupation at E_j; the integrated corner weights w_l of Sec. II.C):
 *
 *   nos[j][m] = sum over cubes, tetrahedra of Table I, bands n and corners l of b[n][m][k_l] w_{n,l}(E_j)
 *
 * with w_l = 0 for E_j <= E1 and w_l = V_T/(4 V_G) for E_j >= E4, so nos[j][m] counts the states of
 * orbital m up to E_j per k-point (unit cell). Arguments as for tetra_dos_forward; nos is device
 * float [ne][norb], overwritten. flags: TETRA_TILE(shape) or 0 (TETRA_EXACT and TETRA_DETERMINISTIC
 * give TETRA_ERR_UNSUPPORTED). The kernels add the increments of each tetrahedron-band's weights
 * between neighbouring grid energies; the weights are evaluated in FP32, or in FP64 on the tiles
 * where a tetrahedron spans more than 64 energy steps (FP32 increments there would lose about
 * 1e-7 E41/de of their value to cancellation). Allocates nothing.
 */
tetra_status tetra_nos_forward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                               const float* w_scale, float* nos, unsigned flags, void* stream);

/*
 * Bin-averaged orbital-resolved DOS: the increase of the number of states across the bin of width de
 * centred on each grid energy,
 *
 *   dos[j][m] = (N_m(E_j + de/2) - N_m(E_j - de/2)) / de,
 *
 * with N_m as in tetra_nos_forward. Each tetrahedron-band contributes the exact integral of its
 * piecewise-polynomial corner DOS over the bin, so sum_j dos[j][m] de equals
 * N_m(e0 + (ne - 1/2) de) - N_m(e0 - de/2) (no sampling of peaks narrower than de). Arguments and
 * flags as for tetra_nos_forward; dos is device float [ne][norb], overwritten. Allocates nothing.
 */
tetra_status tetra_dos_binned(const tetra_desc* d, const float* eps, const void* w, int wtype,
                              const float* w_scale, float* dos, unsigned flags, void* stream);

/*
 * Orbital-resolved susceptibility spectral weight: the imaginary part of the bare (Lindhard)
 * susceptibility at zero temperature for a transfer q on the k-grid, by the linear tetrahedron method
 * (the paper names susceptibilities as the next application of its method, Sec. I and Sec. V):
 *
 *   out[j][m] = S_m(q, w_j) = sum over tetrahedra of Table I and band pairs (n, n') of
 *     (1/V_G) int_T W_m [theta(E_F - eps) theta(eps' - E_F) - theta(eps - E_F) theta(E_F - eps')]
 *                       delta(w_j - (eps' - eps)) d^3k,
 *
 * with eps = eps_n(k), eps' = eps_n'(k + q), W_m = b_mn(k) b_mn'(k + q), each linear inside a
 * tetrahedron between its corner values, the step functions applied exactly (each tetrahedron is
 * clipped at eps = E_F and eps' = E_F into sub-tetrahedra, each of which takes the corner weights of
 * Sec. II.C with eps' - eps as its energy). Im chi_0(q, w) = -pi S(q, w) for
 * chi_0 = (1/N) sum [f(eps) - f(eps')] / (w + eps - eps' + i0); S is per energy unit per k-point,
 * no spin factor; positive for w > 0 (transitions from occupied n to empty n'), negative for w < 0.
 *   d        host descriptor; its energy grid (e0, de, ne) is the transfer-energy grid w_j = e0 + j*de
 *   q1,q2,q3 transfer in grid steps along the three axes (any sign; periodic)
 *   e_fermi  Fermi energy (finite)
 *   eps, w, wtype, w_scale   as for tetra_dos_forward (FP32, FP16 with scale, or complex amplitudes)
 *   out      device, float [ne][norb], overwritten
 *   flags    TETRA_TILE(shape) or 0 (TETRA_EXACT and TETRA_DETERMINISTIC give TETRA_ERR_UNSUPPORTED)
 * One workgroup per (tile, band pair): nb*nb*(tiles) must stay below 2^31 (TETRA_ERR_UNSUPPORTED).
 * A tetrahedron with a non-finite corner energy in either band contributes nothing for that pair.
 * Allocates nothing. Same as tetra_chi_spectral_ws with no workspace.
 */
tetra_status tetra_chi_spectral(const tetra_desc* d, int q1, int q2, int q3, float e_fermi, const float* eps,
                                const void* w, int wtype, const float* w_scale, float* out, unsigned flags,
                                void* stream);

/*
 * Bytes of device workspace for tetra_chi_spectral_ws: 16 nb T, with T the tiles of the grid for the
 * tile shape in flags (two energy ranges of 8 bytes per (tile, band)). 0 for invalid arguments.
 * flags: TETRA_TILE(shape) or 0.
 */
size_t tetra_chi_spectral_workspace(const tetra_desc* d, unsigned flags);

/*
 * tetra_chi_spectral with a caller-owned workspace (device memory of at least
 * tetra_chi_spectral_workspace(d, flags) bytes, 16-byte aligned (TETRA_ERR_ARG otherwise), contents
 * ignored and overwritten, not used after the work on the stream ends). A first pass writes the
 * energy range of every (tile, band) there, at the tile's points and at the points shifted by q, so
 * that a (tile, band pair) unit whose bands cannot be occupied on one side of E_F and empty on the
 * other, or whose range of eps' - eps misses the transfer-energy grid, leaves before loading anything
 * (most units of a model with many bands). The tests bound the exact ones, so the result is the one
 * tetra_chi_spectral computes (up to the order of the float atomics that add the units' partial
 * sums). workspace NULL: tetra_chi_spectral. ws_bytes below the size: TETRA_ERR_WORKSPACE.
 * Other arguments and errors as for tetra_chi_spectral. Allocates nothing.
 */
tetra_status tetra_chi_spectral_ws(const tetra_desc* d, int q1, int q2, int q3, float e_fermi, const float* eps,
                                   const void* w, int wtype, const float* w_scale, float* out, unsigned flags,
                                   void* workspace, size_t ws_bytes, void* stream);

/* One problem of a batch: its descriptor and device buffers (same meaning as tetra_dos_forward). */
typedef struct {
  tetra_desc d;
  const float* eps;
  const void* w;
  const float* w_scale;
  float* dos;
  int tile; /* tile shape id as for TETRA_TILE (0 = default) */
} tetra_item;

/*
 * Bytes of device workspace tetra_dos_batched needs for these items (host array of n items):
 * 256 per persistent launch. Returns 0 for invalid input.
 */
size_t tetra_dos_batched_workspace(const tetra_item* items, int n, int wtype, unsigned flags);

/*
 * Many independent problems (uneven grids, energy grids, band counts) through one persistent launch
 * per group of up to 32 items with the same orbital count: workgroups pull (item, band, tile) units
 * from a work counter, so problems of very different sizes share the chip. `items` is host memory
 * read during the call (the descriptors travel as kernel arguments); `workspace` is device memory of
 * at least tetra_dos_batched_workspace() bytes (one 256-byte counter per launch), owned by the caller
 * and not used by anything else until the work on `stream` completes. Each item's dos is
 * overwritten. Every item uses weight type wtype (with its own w_scale for TETRA_W_F16).
 * Allocates nothing and copies nothing to the device, so a call can be captured in a HIP graph.
 * flags must be 0 (TETRA_EXACT and TETRA_DETERMINISTIC are not supported here:
 * TETRA_ERR_UNSUPPORTED).
 */
tetra_status tetra_dos_batched(const tetra_item* items, int n, int wtype, unsigned flags,
                               void* workspace, size_t ws_bytes, void* stream);

/*
 * FP16 storage of orbital weights with a per-band power-of-two scale (the input format of
 * TETRA_W_F16; the precision variant's storage, not in the paper, which is FP32 throughout):
 *   w_scale[n] = 2^e_n, e_n = ceil(log2 max_{m,k} |w[n][m][k]|) clamped to [-126, 126], e_n = 0 for
 *                an all-zero band (e_n from the exponent and mantissa fields of that maximum);
 *   w16[n][m][k] = w[n][m][k] / w_scale[n] rounded to the nearest FP16 value (ties to even).
 * The division by a power of two is exact, so the only error is the FP16 rounding.
 *   w        device, float [nb][norb][nk]  input weights (finite; other values are unspecified)
 *   w16      device, FP16 [nb][norb][nk]   output, overwritten
 *   w_scale  device, float [nb]            output, overwritten (used as scratch until the last launch)
 * nb, norb, nk >= 1 and nb*norb*nk < 2^31 (TETRA_ERR_ARG otherwise). Four launches on `stream`;
 * allocates nothing.
 */
tetra_status tetra_pack_f16(int nb, int norb, int nk, const float* w, void* w16, float* w_scale, void* stream);

/* Static text for a status code. */
const char* tetra_status_string(int status);

/* Text of the last HIP error seen by this library in the calling thread ("" if none). */
const char* tetra_last_hip_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int tetra_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TETRA_H */
