// C ABI entry points (include/tetra.h): argument validation on the host, then kernel launches.

#include <cmath>
#include <cstring>

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
  if (d->ne >= (1 << 24)) return TETRA_ERR_ARG;
  const double nk = (double)d->n1 * d->n2 * d->n3;
  if (nk * d->nb >= 2147483648.0 || nk * d->nb * d->norb >= 2147483648.0) return TETRA_ERR_ARG;
  if ((double)d->ne * d->norb >= 2147483648.0) return TETRA_ERR_ARG;
  if (d->norb > 16) return TETRA_ERR_UNSUPPORTED;
  // The last grid energy must be finite in FP32.
  if (!std::isfinite(d->e0 + (float)(d->ne - 1) * d->de)) return TETRA_ERR_ARG;
  return TETRA_OK;
}

tetra_status check_weights(int wtype, const float* w_scale) {
  if (wtype == TETRA_W_F32) return w_scale ? TETRA_ERR_ARG : TETRA_OK;
  if (wtype == TETRA_W_F16) return w_scale ? TETRA_ERR_UNSUPPORTED : TETRA_ERR_ARG;
  return TETRA_ERR_ARG;
}

}  // namespace

extern "C" {

tetra_status tetra_dos_forward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                               const float* w_scale, float* dos, unsigned flags, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !dos) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)TETRA_KAHAN) return TETRA_ERR_ARG;
  if (flags & TETRA_KAHAN) return TETRA_ERR_UNSUPPORTED;
  return hip_status(tetra::forward_f32(*d, eps, static_cast<const float*>(w), dos, (hipStream_t)stream));
}

tetra_status tetra_dos_backward(const tetra_desc* d, const float* eps, const void* w, int wtype,
                                const float* w_scale, const float* grad_dos, float* grad_eps,
                                float* grad_w, unsigned flags, void* stream) {
  tetra_status st = check_desc(d);
  if (st != TETRA_OK) return st;
  if (!eps || !w || !grad_dos || (!grad_eps && !grad_w)) return TETRA_ERR_ARG;
  if ((st = check_weights(wtype, w_scale)) != TETRA_OK) return st;
  if (flags & ~(unsigned)TETRA_KAHAN) return TETRA_ERR_ARG;
  return hip_status(tetra::backward_f32(*d, eps, static_cast<const float*>(w), grad_dos, grad_eps, grad_w,
                                        (hipStream_t)stream));
}

size_t tetra_dos_batched_workspace(const tetra_item* items, int n, int wtype, unsigned flags) {
  (void)items;
  (void)n;
  (void)wtype;
  (void)flags;
  return 0;
}

tetra_status tetra_dos_batched(const tetra_item* items, int n, int wtype, unsigned flags, void* workspace,
                               size_t ws_bytes, void* stream) {
  if (!items || n < 1) return TETRA_ERR_ARG;
  (void)wtype;
  (void)flags;
  (void)workspace;
  (void)ws_bytes;
  (void)stream;
  return TETRA_ERR_UNSUPPORTED;
}

const char* tetra_status_string(int status) {
  switch (status) {
    case TETRA_OK: return "ok";
    case TETRA_ERR_ARG: return "invalid argument";
    case TETRA_ERR_UNSUPPORTED: return "unsupported request";
    case TETRA_ERR_WORKSPACE: return "workspace missing or too small";
    case TETRA_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* tetra_last_hip_error(void) { return g_last_hip_error; }

int tetra_version(void) { return 100; }

}  // extern "C"
