// Benchmark-only measurement helper, built into libtetra_probe.so with the LDS-atomic probe and not part
// of the DOS library or its C ABI: the issue rate of plain (non-packed) FP32 fused multiply-adds, the
// ceiling of kernels built, as every kernel of the DOS library is, without packed FP32 instructions.
// Each lane runs sixteen independent chains `x = x * a + b`, so consecutive instructions never wait
// for one another and the rate measured is that of VALU issue alone.

#include <hip/hip_runtime.h>

namespace {

constexpr int kFmaThreads = 256;
constexpr int kFmaChains = 16;

__global__ __launch_bounds__(kFmaThreads) void fma_rate_probe_kernel(float* out, int iters, float a, float b) {
  float x[kFmaChains];
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) x[c] = __builtin_fmaf((float)threadIdx.x, 1e-3f, (float)c);
#pragma unroll 1
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) s += x[c];
  out[(size_t)blockIdx.x * kFmaThreads + threadIdx.x] = s;
}

}  // namespace

// `blocks` workgroups of 256 lanes, each lane issuing `iters` x 16 FP32 FMAs (2 flops each); out
// (device, float [blocks * 256]) receives one value per lane, overwritten. Returns 0, -1 for invalid
// arguments (blocks or iters outside 1..2^24, out NULL), -4 for a failed launch. Asynchronous on
// `stream`; allocates nothing.
extern "C" int tetra_probe_fma_f32(int blocks, int iters, float* out, void* stream) {
  if (!out || blocks < 1 || blocks > (1 << 24) || iters < 1 || iters > (1 << 24)) return -1;
  hipLaunchKernelGGL(fma_rate_probe_kernel, dim3(blocks), dim3(kFmaThreads), 0, (hipStream_t)stream, out, iters,
                     0.999f, 1e-4f);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
