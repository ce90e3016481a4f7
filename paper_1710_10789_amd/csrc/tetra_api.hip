// C ABI entry points (include/tetra.h): argument validation on the host, then kernel launches.

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "tetra_internal.h"

namespace {

thread_local char g_last_hip_error[256] = "";

tetra_status hip_status(hipError_t e) {
  if (e == hipSuccess) return TETRA_OK;
  std::strncpy(g_last_hip_error, hipGetErrorString(e), sizeof(g_last_hip_error) - 1);
  g_last_hip_error[sizeof(g_last_hip_error) - 1] = '\0';
  return TETRA_ERR_HIP;
}

// Shape and range checks shared by every entry point (no HIP call).
tetra_status check_desc(const tetra_desc* d) {
  if (!d) return TETRA_ERR_ARG;
  if (d->n1 < 1 || d->n2 < 1 || d->n3 < 1 || d->nb < 1 || d->norb < 1 || d->ne < 1) return TETRA_ERR_ARG;
  if (!std::isfinite(d->e0) || !std::isfinite(d->de) || !(d->de > 0.0f)) return TETRA_ERR_ARG;
  if (d->ne > (1 << 22)) return TETRA_ERR_ARG;  // keeps FP32 window estimates within one index
  const double nk = (double)d->n1 * d->n2 * d->n3;
  if (nk * d->nb >= 2147483648.0 || nk * d->nb * d->norb >= 2147483648.0) return TETRA_ERR_ARG;
  if ((double)d->ne * d->norb >= 2147483648.0) return TETRA_ERR_ARG;
  if (d->norb > 16) return TETRA_ERR_UNSUPPORTED;
  // The last grid energy must be finite in FP32.
  if (!std::isfinite(d->e0 + (float)(d->ne - 1) * d->de)) return TETRA_ERR_ARG;
  return TETRA_OK;
}

tetra_status check_weights(int wtype, const float* w_scale) {
  if (wtype == TETRA_W_F32 || wtype == TETRA_W_C32) return w_scale ? TETRA_ERR_ARG : TETRA_OK;
  if (wtype == TETRA_W_F16) return w_scale ? TETRA_OK : TETRA_ERR_ARG;
  return TETRA_ERR_ARG;
}

const float* scale_of(int wtype, const float* w_scale) { return wtype == TETRA_W_F16 ? w_scale : nullptr; }

}  // namespace

extern "C" {

size_t tetra_dos_forward_workspace(const tetra_desc* d, unsigned flags) {
  if (check_desc(d) != TETRA_OK) return 0;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return 0;
  if ((int)((flags & TETRA_TILE_MASK) >> 8) >= tetra::kTileShapes) return 0;
  return (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) ? tetra::forward_exact_scratch_bytes(*d) : 0;
}

tetra_status tetra_dos_forward_ws(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                  const float* w_scale, float* dos, unsigned flags, void* workspace,
                                  size_t ws_bytes, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !dos) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return TETRA_ERR_ARG;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return TETRA_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0) return TETRA_ERR_ARG;
  // the exact accumulation is also the deterministic one; only it uses the workspace
  const bool exact = (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) != 0;
  if (exact && (!workspace || ws_bytes < tetra::forward_exact_scratch_bytes(*d))) return TETRA_ERR_WORKSPACE;
  return hip_status(tetra::forward(*d, eps, w, wtype, scale_of(wtype, w_scale), dos, exact ? workspace : nullptr,
                                   shape, (hipStream_t)stream));
}

tetra_status tetra_dos_forward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                               const float* w_scale, float* dos, unsigned flags, void* stream) {
  return tetra_dos_forward_ws(d, eps, w, wtype, w_scale, dos, flags, nullptr, 0, stream);
}

}  // extern "C"

namespace {

// Device memory of the allocation-free forward (tetra_dos_forward_noalloc): the exact path's bound
// exponent and fixed-point sums live in this file-scope array instead of a caller's workspace. Each
// device holds its own copy for the life of the process. In host code `scratch` is only a host-side
// stand-in for the symbol: its device address comes from hipGetSymbolAddress, once per device with
// that device current, and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = 256 + 8 * (size_t)TETRA_NOALLOC_MAX_BINS;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kScratchDevices = 64;
std::atomic<void*> g_scratch_ptr[kScratchDevices];

// Device address of `scratch` on the current device (looked up on the first call per device;
// concurrent first calls store the same address).
hipError_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return hipSuccess;
}

}  // namespace

extern "C" {

tetra_status tetra_dos_forward_noalloc(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                       const float* w_scale, float* dos, unsigned flags, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !dos) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return TETRA_ERR_ARG;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return TETRA_ERR_ARG;
  const bool exact = (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) != 0;
  if (exact && tetra::forward_exact_scratch_bytes(*d) > kStaticScratchBytes) return TETRA_ERR_SCRATCH;
  void* ws = nullptr;
  if (exact) {
    const hipError_t e = static_scratch(&ws);
    if (e != hipSuccess) return hip_status(e);
  }
  return hip_status(
      tetra::forward(*d, eps, w, wtype, scale_of(wtype, w_scale), dos, ws, shape, (hipStream_t)stream));
}

tetra_status tetra_pack_f16(int nb, int norb, int nk, const float* w, void* w16, float* w_scale, void* stream) {
  if (nb < 1 || norb < 1 || nk < 1 || !w || !w16 || !w_scale) return TETRA_ERR_ARG;
  if ((double)nb * norb * nk >= 2147483648.0) return TETRA_ERR_ARG;
  return hip_status(tetra::pack_f16(nb, (int64_t)norb * nk, w, w16, w_scale, (hipStream_t)stream));
}

tetra_status tetra_dos_backward_ws(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                   const float* w_scale, const float* grad_dos, float* grad_eps, float* grad_w,
                                   unsigned flags, void* workspace, size_t ws_bytes, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !grad_dos || (!grad_eps && !grad_w)) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return TETRA_ERR_ARG;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return TETRA_ERR_ARG;
  const size_t need = tetra::backward_workspace_bytes(*d, shape);
  if (workspace && (need == 0 || ws_bytes < need)) return TETRA_ERR_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0) return TETRA_ERR_ARG;
  // the two-phase output is deterministic; the atomic one is not
  if ((flags & TETRA_DETERMINISTIC) && !workspace) return TETRA_ERR_UNSUPPORTED;
  return hip_status(tetra::backward(*d, eps, w, wtype, scale_of(wtype, w_scale), grad_dos, grad_eps, grad_w, shape,
                                    workspace, (hipStream_t)stream));
}

tetra_status tetra_dos_backward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                const float* w_scale, const float* grad_dos, float* grad_eps,
                                float* grad_w, unsigned flags, void* stream) {
  return tetra_dos_backward_ws(d, eps, w, wtype, w_scale, grad_dos, grad_eps, grad_w, flags, nullptr, 0, stream);
}

size_t tetra_dos_backward_workspace(const tetra_desc* d, unsigned flags) {
  if (check_desc(d) != TETRA_OK) return 0;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return 0;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return 0;
  return tetra::backward_workspace_bytes(*d, shape);
}

namespace {

tetra_status nos_entry(const tetra_desc* d, const float* eps, const void* w, int wtype, const float* w_scale,
                       float* out, unsigned flags, void* stream, bool binned) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !out) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return TETRA_ERR_ARG;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return TETRA_ERR_ARG;
  if (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) return TETRA_ERR_UNSUPPORTED;
  return hip_status(tetra::nos(*d, eps, w, wtype, scale_of(wtype, w_scale), out, binned, shape, (hipStream_t)stream));
}

}  // namespace

tetra_status tetra_nos_forward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                               const float* w_scale, float* nos, unsigned flags, void* stream) {
  return nos_entry(d, eps, w, wtype, w_scale, nos, flags, stream, false);
}

tetra_status tetra_dos_binned(const tetra_desc* d, const float* eps, const void* w, int wtype,
                              const float* w_scale, float* dos, unsigned flags, void* stream) {
  return nos_entry(d, eps, w, wtype, w_scale, dos, flags, stream, true);
}

tetra_status tetra_chi_spectral_ws(const tetra_desc* d, int q1, int q2, int q3, float e_fermi, const float* eps,
                                   const void* w, int wtype, const float* w_scale, float* out, unsigned flags,
                                   void* workspace, size_t ws_bytes, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !out) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (!std::isfinite(e_fermi)) return TETRA_ERR_ARG;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC | TETRA_TILE_MASK)) return TETRA_ERR_ARG;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return TETRA_ERR_ARG;
  if (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) return TETRA_ERR_UNSUPPORTED;
  if (tetra::chi_units(*d, shape) > 2147483647 - 8) return TETRA_ERR_UNSUPPORTED;  // one workgroup per unit
  if (workspace) {
    if (ws_bytes < 8 * (size_t)tetra::chi_range_entries(*d, shape)) return TETRA_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0) return TETRA_ERR_ARG;
  }
  return hip_status(tetra::chi(*d, q1, q2, q3, e_fermi, eps, w, wtype, scale_of(wtype, w_scale), out, shape,
                               workspace, (hipStream_t)stream));
}

tetra_status tetra_chi_spectral(const tetra_desc* d, int q1, int q2, int q3, float e_fermi, const float* eps,
                                const void* w, int wtype, const float* w_scale, float* out, unsigned flags,
                                void* stream) {
  return tetra_chi_spectral_ws(d, q1, q2, q3, e_fermi, eps, w, wtype, w_scale, out, flags, nullptr, 0, stream);
}

size_t tetra_chi_spectral_workspace(const tetra_desc* d, unsigned flags) {
  if (check_desc(d) != TETRA_OK || (flags & ~(unsigned)TETRA_TILE_MASK)) return 0;
  const int shape = (int)((flags & TETRA_TILE_MASK) >> 8);
  if (shape >= tetra::kTileShapes) return 0;
  return 8 * (size_t)tetra::chi_range_entries(*d, shape);
}

size_t tetra_dos_batched_workspace(const tetra_item* items, int n, int wtype, unsigned flags) {
  if (!items || n < 1 || (wtype != TETRA_W_F32 && wtype != TETRA_W_F16 && wtype != TETRA_W_C32) || flags != 0)
    return 0;
  for (int i = 0; i < n; ++i)
    if (check_desc(&items[i].d) != TETRA_OK) return 0;
  return 256 * tetra::batched_launches(items, n);
}

tetra_status tetra_dos_batched(const tetra_item* items, int n, int wtype, unsigned flags, void* workspace,
                               size_t ws_bytes, void* stream) {
  if (!items || n < 1) return TETRA_ERR_ARG;
  if (wtype != TETRA_W_F32 && wtype != TETRA_W_F16 && wtype != TETRA_W_C32) return TETRA_ERR_ARG;
  if (flags & ~(unsigned)(TETRA_EXACT | TETRA_DETERMINISTIC)) return TETRA_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    const tetra_item& it = items[i];
    const tetra_status st = check_desc(&it.d);
    if (st != TETRA_OK) return st;
    if (!it.eps || !it.w || !it.dos) return TETRA_ERR_ARG;
    if (check_weights(wtype, it.w_scale) != TETRA_OK) return TETRA_ERR_ARG;
    if (it.tile < 0 || it.tile >= tetra::kTileShapes) return TETRA_ERR_ARG;
  }
  if (flags & (TETRA_EXACT | TETRA_DETERMINISTIC)) return TETRA_ERR_UNSUPPORTED;
  if (!workspace || ws_bytes < 256 * tetra::batched_launches(items, n)) return TETRA_ERR_WORKSPACE;
  std::vector<int> shapes(n);
  for (int i = 0; i < n; ++i) shapes[i] = items[i].tile;
  return hip_status(tetra::batched(items, shapes.data(), n, wtype, workspace, (hipStream_t)stream));
}

const char* tetra_status_string(int status) {
  switch (status) {
    case TETRA_OK: return "ok";
    case TETRA_ERR_ARG: return "invalid argument";
    case TETRA_ERR_UNSUPPORTED: return "unsupported request";
    case TETRA_ERR_WORKSPACE: return "workspace missing or too small";
    case TETRA_ERR_HIP: return "HIP runtime error";
    case TETRA_ERR_SCRATCH: return "problem exceeds the static scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

const char* tetra_last_hip_error(void) { return g_last_hip_error; }

int tetra_version(void) { return 100; }

}  // extern "C"
