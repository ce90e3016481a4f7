// Benchmark-only measurement helper, built into its own library (libtetra_probe.so) and not part of
// the DOS library or its C ABI: the throughput of 64-bit integer LDS atomics on gfx950, the instruction the
// forward and number-of-states kernels deposit with. Every lane adds to its own 64-bit word (a lane's
// word index is its lane number plus a multiple of 64, so the 64 lanes of a wavefront touch 64
// different words and no two adds of one instruction go to the same address). That is the best case
// of the histogram deposits, whose lanes may share bins; its rate bounds how fast a kernel that
// issues a given number of LDS atomics can be.

#include <hip/hip_runtime.h>

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 2048;  // 16 KiB of LDS, as the kernels' histograms

__global__ __launch_bounds__(kProbeThreads) void lds_atomic_probe_kernel(unsigned long long* out, int iters) {
  __shared__ unsigned long long s_h[kProbeWords];
  for (int q = threadIdx.x; q < kProbeWords; q += kProbeThreads) s_h[q] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long v = (unsigned long long)threadIdx.x + 1ull;
  // four rows as in a packed deposit of eight orbitals; each wavefront its own quarter of the words
  unsigned long long* row = &s_h[wave * (kProbeWords / 4) + lane];
#pragma unroll 1
  for (int i = 0; i < iters; ++i) {
    unsigned long long* h = row + 64 * (i & 1);
    atomicAdd(&h[0], v);
    atomicAdd(&h[128], v);
    atomicAdd(&h[256], v);
    atomicAdd(&h[384], v);
  }
  __syncthreads();
  unsigned long long sum = 0ull;
  for (int q = threadIdx.x; q < kProbeWords; q += kProbeThreads) sum += s_h[q];
  // one word per workgroup keeps the adds observable
  if (threadIdx.x == 0) out[blockIdx.x] = 0ull;
  __syncthreads();
  atomicAdd(&out[blockIdx.x], sum);
}

}  // namespace

// `blocks` workgroups of 256 lanes, each lane issuing `iters` x 4 64-bit LDS atomic adds to a word of
// its own; out (device, uint64 [blocks]) receives one checksum per workgroup, overwritten.
// Returns 0, -1 for invalid arguments (blocks or iters outside 1..2^24, out NULL), -4 for a failed
// launch. Asynchronous on `stream`; allocates nothing.
extern "C" int tetra_probe_lds_atomics(int blocks, int iters, unsigned long long* out, void* stream) {
  if (!out || blocks < 1 || blocks > (1 << 24) || iters < 1 || iters > (1 << 24)) return -1;
  hipLaunchKernelGGL(lds_atomic_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, (hipStream_t)stream, out, iters);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
