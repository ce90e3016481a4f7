// Measurement helper of the library (not part of the DOS computation). Internal header.
#pragma once

#include <hip/hip_runtime.h>

namespace tetra {

// 256-lane workgroups issuing iters x 4 conflict-free 64-bit LDS atomic adds per lane; out[blocks]
// receives one checksum per workgroup.
hipError_t probe_lds_atomics(int blocks, int iters, unsigned long long* out, hipStream_t s);

}  // namespace tetra
