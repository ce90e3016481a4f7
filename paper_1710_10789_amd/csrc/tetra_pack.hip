// FP16 storage of the orbital weights with a per-band power-of-two scale (the precision variant's
// input format): for band n,
//   scale_n = 2^e_n,  e_n = ceil(log2 max_{m,k} |w[n][m][k]|) clamped to [-126, 126] (0 for an all-zero band),
//   w16[n][m][k] = RNE_fp16(w[n][m][k] / scale_n).
// Dividing by a power of two is exact, so the only error is the FP16 rounding (at most 2^-11 of the
// value, or 2^-25 of the scale in the FP16 subnormal range). e_n comes from the integer fields of the
// largest magnitude, so host and device give the same scale bit for bit. Weights must be finite.

#include "tetra_internal.h"

namespace tetra {

namespace {

// Largest |w| per band, as the bit pattern of a non-negative float (which orders like an unsigned
// integer): one atomicMax per workgroup into w_scale[n], cleared first.
__global__ void pack_clear_kernel(unsigned* bits, int nb) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < nb) bits[n] = 0u;
}

__global__ __launch_bounds__(256) void pack_max_kernel(const float* w, int64_t per_band, int nb, unsigned* bits) {
  __shared__ unsigned s_mx[4];
  for (int n = blockIdx.y; n < nb; n += gridDim.y) {  // uniform across the workgroup
    const float* wn = w + (int64_t)n * per_band;
    unsigned mx = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_band;
         i += (int64_t)gridDim.x * blockDim.x) {
      const float v = fabsf(wn[i]);
      if (__builtin_isfinite(v)) mx = max(mx, __float_as_uint(v));
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned)__shfl_xor((int)mx, o));
    if ((threadIdx.x & 63) == 0) s_mx[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      mx = max(max(s_mx[0], s_mx[1]), max(s_mx[2], s_mx[3]));
      if (mx) atomicMax(&bits[n], mx);
    }
    __syncthreads();  // s_mx is read before the next band overwrites it
  }
}

// ceil(log2 x) of a non-negative finite float given by its bits, clamped to [-126, 126]; 0 for x = 0.
__device__ __forceinline__ int scale_exponent(unsigned bits) {
  if (bits == 0u) return 0;
  const int ex = (int)(bits >> 23);           // biased exponent (0: subnormal, below 2^-126)
  const unsigned man = bits & 0x7fffffu;
  int e = ex == 0 ? -126 : ex - 127 + (man != 0u);
  return min(max(e, -126), 126);
}

__global__ __launch_bounds__(256) void pack_quantize_kernel(const float* w, int64_t per_band, int nb,
                                                            const unsigned* bits, _Float16* w16) {
  for (int n = blockIdx.y; n < nb; n += gridDim.y) {
    const float inv = ldexpf(1.0f, -scale_exponent(bits[n]));  // a normal power of two
    const float* wn = w + (int64_t)n * per_band;
    _Float16* on = w16 + (int64_t)n * per_band;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_band;
         i += (int64_t)gridDim.x * blockDim.x)
      on[i] = (_Float16)(wn[i] * inv);  // v_cvt_f16_f32: round to nearest even
  }
}

// Runs after the quantisation on the same stream: the bits become the scale itself.
__global__ void pack_finish_kernel(unsigned* bits, int nb) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < nb) bits[n] = __float_as_uint(ldexpf(1.0f, scale_exponent(bits[n])));
}

}  // namespace

hipError_t pack_f16(int nb, int64_t per_band, const float* w, void* w16, float* w_scale, hipStream_t s) {
  unsigned* bits = reinterpret_cast<unsigned*>(w_scale);
  const unsigned nbb = (unsigned)((nb + 255) / 256);
  hipLaunchKernelGGL(pack_clear_kernel, dim3(nbb), dim3(256), 0, s, bits, nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // about 2048 elements per workgroup, at most about 4096 workgroups in all
  const unsigned by = (unsigned)std::min(nb, 4096);
  const int64_t per = (per_band + 2047) / 2048;
  const int64_t cap = (4096 + by - 1) / by;
  const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(per, cap));
  hipLaunchKernelGGL(pack_max_kernel, dim3(bx, by), dim3(256), 0, s, w, per_band, nb, bits);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(pack_quantize_kernel, dim3(bx, by), dim3(256), 0, s, w, per_band, nb, bits,
                     static_cast<_Float16*>(w16));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(pack_finish_kernel, dim3(nbb), dim3(256), 0, s, bits, nb);
  return hipGetLastError();
}

}  // namespace tetra
