// Stored forms of the orbital weights, for the kernels' staging loops (gfx950). Internal header.
#pragma once

#include <hip/hip_runtime.h>

namespace tetra {

// Orbital weight b from its stored form: FP32 as is; FP16 times its band's power-of-two scale; a complex
// amplitude a = (re, im) as |a|^2 (eq. matrixelements of arXiv:1710.10789).
__device__ __forceinline__ float weight_value(float v, float) { return v; }
__device__ __forceinline__ float weight_value(_Float16 v, float scale) { return (float)v * scale; }
__device__ __forceinline__ float weight_value(float2 a, float) { return a.x * a.x + a.y * a.y; }

}  // namespace tetra
