// Driver for the sanitizer build of the C ABI's host code (every csrc/*.hip compiled with
// -Xarch_host -fsanitize=address,undefined by tests/test_sanitizers_host.py and linked into this
// executable). Test harness only; needs no GPU: every call below is rejected by the argument checks
// before any HIP call, or is a pure size query.
//
// Each entry point gets a valid descriptor with one defect at a time (null or malformed descriptor,
// null pointers, weight types and scales that do not match, unknown flag bits, tile shapes out of
// range, sizes past the 32-bit index range, missing, short or misaligned workspaces, an exact
// request beyond the allocation-free scratch) and must return the documented status; the size
// queries must return their documented values. Prints "ok <checks>" at the end; any mismatch exits
// non-zero with its line.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>

#include "tetra.h"

static int checks = 0;
#define EXPECT(expr, want)                                                                               \
  do {                                                                                                   \
    ++checks;                                                                                            \
    const long long got_ = (long long)(expr);                                                            \
    if (got_ != (long long)(want)) {                                                                     \
      std::printf("line %d: %s = %lld, want %lld\n", __LINE__, #expr, got_, (long long)(want));          \
      return 1;                                                                                          \
    }                                                                                                    \
  } while (0)

static tetra_desc good() {
  tetra_desc d;
  d.n1 = 8;
  d.n2 = 8;
  d.n3 = 32;
  d.nb = 2;
  d.norb = 3;
  d.e0 = -1.0f;
  d.de = 0.01f;
  d.ne = 100;
  return d;
}

int main() {
  // Host stand-ins for device pointers: never dereferenced, every call below stops at its checks.
  alignas(16) static unsigned char buf[4096];
  float* F = reinterpret_cast<float*>(buf);
  void* V = buf;
  void* misaligned = buf + 4;
  const float* noscale = nullptr;

  // descriptors
  tetra_desc d = good();
  EXPECT(tetra_dos_forward(nullptr, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  const int bad_ints[][2] = {{0, 0}, {1, 0}, {2, 0}, {3, 0}, {4, 0}, {5, 0}};
  for (const auto& b : bad_ints) {
    d = good();
    int* fields[] = {&d.n1, &d.n2, &d.n3, &d.nb, &d.norb, &d.ne};
    *fields[b[0]] = b[1];
    EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
    EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F32, noscale, F, F, F, 0, nullptr), TETRA_ERR_ARG);
    EXPECT(tetra_nos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
    EXPECT(tetra_chi_spectral(&d, 0, 0, 0, 0.0f, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
    EXPECT(tetra_dos_forward_workspace(&d, TETRA_EXACT), 0);
    EXPECT(tetra_dos_backward_workspace(&d, 0), 0);
  }
  d = good();
  d.norb = 17;
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_UNSUPPORTED);
  d = good();
  d.de = 0.0f;
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  d.de = -0.5f;
  EXPECT(tetra_dos_binned(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  d.de = std::numeric_limits<float>::quiet_NaN();
  EXPECT(tetra_dos_forward_ws(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr, 0, nullptr), TETRA_ERR_ARG);
  d = good();
  d.e0 = std::numeric_limits<float>::infinity();
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  d = good();
  d.e0 = 3.0e38f;
  d.de = 1.0e37f;  // last grid energy overflows FP32
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  d = good();
  d.ne = (1 << 22) + 1;
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  d = good();
  d.n1 = d.n2 = d.n3 = 1291;  // nk nb past 2^31
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_backward_workspace(&d, 0), 0);

  // pointers, weight types and scales
  d = good();
  EXPECT(tetra_dos_forward(&d, nullptr, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, nullptr, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, nullptr, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, F, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F16, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_C32, F, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, 7, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F32, noscale, F, nullptr, nullptr, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F32, noscale, nullptr, F, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F16, noscale, F, F, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_nos_forward(&d, nullptr, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_binned(&d, F, V, TETRA_W_F32, noscale, nullptr, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_chi_spectral(&d, 1, 2, 3, NAN, F, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_chi_spectral(&d, 1, 2, 3, 0.0f, F, V, TETRA_W_F16, noscale, F, 0, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_pack_f16(0, 3, 10, F, V, F, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_pack_f16(2, 3, 10, nullptr, V, F, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_pack_f16(2, 3, 10, F, V, nullptr, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_pack_f16(1 << 16, 1 << 8, 1 << 8, F, V, F, nullptr), TETRA_ERR_ARG);

  // flags and tile shapes
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, 0x10, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward(&d, F, V, TETRA_W_F32, noscale, F, TETRA_TILE(6), nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F32, noscale, F, F, F, TETRA_TILE(15), nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_nos_forward(&d, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, nullptr), TETRA_ERR_UNSUPPORTED);
  EXPECT(tetra_dos_binned(&d, F, V, TETRA_W_F32, noscale, F, TETRA_DETERMINISTIC, nullptr), TETRA_ERR_UNSUPPORTED);
  EXPECT(tetra_chi_spectral(&d, 0, 0, 0, 0.0f, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, nullptr),
         TETRA_ERR_UNSUPPORTED);
  EXPECT(tetra_dos_backward(&d, F, V, TETRA_W_F32, noscale, F, F, F, TETRA_DETERMINISTIC, nullptr),
         TETRA_ERR_UNSUPPORTED);

  // workspaces: sizes, missing, short, misaligned
  EXPECT(tetra_dos_forward_workspace(&d, 0), 0);
  EXPECT(tetra_dos_forward_workspace(&d, TETRA_EXACT), 256 + 8 * 100 * 3);
  EXPECT(tetra_dos_forward_workspace(&d, TETRA_DETERMINISTIC | TETRA_TILE(3)), 256 + 8 * 100 * 3);
  EXPECT(tetra_dos_forward_workspace(&d, 0x10), 0);
  EXPECT(tetra_dos_forward_ws(&d, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, nullptr, 0, nullptr),
         TETRA_ERR_WORKSPACE);
  EXPECT(tetra_dos_forward_ws(&d, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, V, 256 + 8 * 100 * 3 - 1, nullptr),
         TETRA_ERR_WORKSPACE);
  EXPECT(tetra_dos_forward_ws(&d, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, misaligned, 1 << 20, nullptr),
         TETRA_ERR_ARG);
  // two-phase adjoint: 8 x 8 x 32 with 4 x 4 x 16 tiles: 2 x 2 x 2 tiles of 290 face points
  const size_t need = (size_t)4 * (3 + 1) * 290 * 2 * 8;
  EXPECT(tetra_dos_backward_workspace(&d, 0), need);
  EXPECT(tetra_dos_backward_workspace(&d, 0x10), 0);
  EXPECT(tetra_dos_backward_ws(&d, F, V, TETRA_W_F32, noscale, F, F, F, 0, V, need - 1, nullptr),
         TETRA_ERR_WORKSPACE);
  EXPECT(tetra_dos_backward_ws(&d, F, V, TETRA_W_F32, noscale, F, F, F, 0, misaligned, need, nullptr),
         TETRA_ERR_ARG);
  // susceptibility first pass: two 8-byte ranges per (tile, band), 2 x 2 x 2 tiles of 4 x 4 x 16, 2 bands
  EXPECT(tetra_chi_spectral_workspace(&d, 0), (size_t)16 * 2 * 8);
  EXPECT(tetra_chi_spectral_workspace(&d, TETRA_TILE(1)), (size_t)16 * 2 * 1 * 1 * 8);  // 1 x 1 x 8 tiles of 8 x 8 x 4
  EXPECT(tetra_chi_spectral_workspace(&d, TETRA_EXACT), 0);
  EXPECT(tetra_chi_spectral_ws(&d, 1, 0, 0, 0.0f, F, V, TETRA_W_F32, noscale, F, 0, V, 16 * 2 * 8 - 1, nullptr),
         TETRA_ERR_WORKSPACE);
  EXPECT(tetra_chi_spectral_ws(&d, 1, 0, 0, 0.0f, F, V, TETRA_W_F32, noscale, F, 0, misaligned, 1 << 20, nullptr),
         TETRA_ERR_ARG);
  EXPECT(tetra_chi_spectral_ws(&d, 1, 0, 0, NAN, F, V, TETRA_W_F32, noscale, F, 0, V, 1 << 20, nullptr),
         TETRA_ERR_ARG);
  tetra_desc r = good();
  r.n3 = 31;  // ragged: no two-phase output
  EXPECT(tetra_dos_backward_workspace(&r, 0), 0);
  EXPECT(tetra_dos_backward_ws(&r, F, V, TETRA_W_F32, noscale, F, F, F, 0, V, need, nullptr), TETRA_ERR_WORKSPACE);

  // the allocation-free forward: an exact request past its static scratch
  tetra_desc big = good();
  big.ne = TETRA_NOALLOC_MAX_BINS / 3 + 1;
  EXPECT(tetra_dos_forward_noalloc(&big, F, V, TETRA_W_F32, noscale, F, TETRA_EXACT, nullptr), TETRA_ERR_SCRATCH);
  EXPECT(tetra_dos_forward_noalloc(&d, F, V, TETRA_W_F32, noscale, F, 0x10, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_forward_noalloc(&d, nullptr, V, TETRA_W_F32, noscale, F, 0, nullptr), TETRA_ERR_ARG);

  // batched
  tetra_item items[2];
  std::memset(items, 0, sizeof(items));
  for (auto& it : items) {
    it.d = good();
    it.eps = F;
    it.w = V;
    it.dos = F;
  }
  EXPECT(tetra_dos_batched_workspace(items, 2, TETRA_W_F32, 0), 256);
  EXPECT(tetra_dos_batched_workspace(items, 0, TETRA_W_F32, 0), 0);
  EXPECT(tetra_dos_batched_workspace(items, 2, 9, 0), 0);
  EXPECT(tetra_dos_batched(nullptr, 2, TETRA_W_F32, 0, V, 256, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_batched(items, 2, TETRA_W_F32, 0, nullptr, 0, nullptr), TETRA_ERR_WORKSPACE);
  EXPECT(tetra_dos_batched(items, 2, TETRA_W_F32, 0, V, 255, nullptr), TETRA_ERR_WORKSPACE);
  EXPECT(tetra_dos_batched(items, 2, TETRA_W_F32, TETRA_EXACT, V, 256, nullptr), TETRA_ERR_UNSUPPORTED);
  items[1].tile = 6;
  EXPECT(tetra_dos_batched(items, 2, TETRA_W_F32, 0, V, 256, nullptr), TETRA_ERR_ARG);
  items[1].tile = 0;
  items[1].d.ne = 0;
  EXPECT(tetra_dos_batched(items, 2, TETRA_W_F32, 0, V, 256, nullptr), TETRA_ERR_ARG);
  EXPECT(tetra_dos_batched_workspace(items, 2, TETRA_W_F32, 0), 0);

  // status strings
  for (int s = -8; s <= 1; ++s) checks += std::strlen(tetra_status_string(s)) > 0 ? 1 : 0;
  EXPECT(std::strcmp(tetra_status_string(TETRA_ERR_WORKSPACE), "workspace missing or too small"), 0);
  EXPECT(tetra_version() > 0, 1);
  EXPECT(tetra_last_hip_error() != nullptr, 1);
  std::printf("ok %d\n", checks);
  return 0;
}
