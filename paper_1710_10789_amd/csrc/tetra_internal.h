// Host-side declarations shared by the library's translation units. Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tetra.h"

namespace tetra {

hipError_t fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t forward_f32(const tetra_desc& d, const float* eps, const float* w, float* dos, hipStream_t s);
hipError_t backward_f32(const tetra_desc& d, const float* eps, const float* w, const float* G, float* grad_eps,
                        float* grad_w, hipStream_t s);

}  // namespace tetra
