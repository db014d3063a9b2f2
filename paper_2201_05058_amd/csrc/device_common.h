// Device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcsdf {

// Signed squared voxel distance -> signed metres:
// F(x) = sign(x) * ((float)h * sqrtf(|x|)), +-inf for +-INT32_MAX.
// The square root is taken first, then one fp32 multiply; hipcc's default
// -fhip-fp32-correctly-rounded-divide-sqrt makes sqrtf correctly rounded.
__device__ __forceinline__ float ssq_to_metres(int32_t x, float hf) {
  if (x == INT32_MAX) return __builtin_inff();
  if (x == -INT32_MAX) return -__builtin_inff();
  const float a = (float)(x < 0 ? -x : x);  // exact: |x| < 2^24
  const float r = hf * sqrtf(a);
  return x < 0 ? -r : r;
}

}  // namespace pcsdf
