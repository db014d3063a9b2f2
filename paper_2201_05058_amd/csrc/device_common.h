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

// Value of the humans' signed field at a voxel of layer k whose planar
// signed value is p (E_D outside D, -E_{Gxy\D} inside, +-INT32_MAX if the other
// set is empty).  dz2o = max(0, k-Kt)^2; zin = (k <= Kt); dz2i =
// (Kt+1-k)^2 when layer Kt+1 exists, else INT32_MAX.
__device__ __forceinline__ int32_t human_value(int32_t p, int dz2o, bool zin,
                                               int32_t dz2i) {
  if (p == INT32_MAX) return INT32_MAX;  // no human voxel in this slice
  if (p > 0) return p + dz2o;  // column outside the disks
  if (!zin) return dz2o;       // above the cylinders: nearest is the top
  const int32_t din = -p;      // INT32_MAX when the disks cover the plane
  return -(din < dz2i ? din : dz2i);
}

}  // namespace pcsdf
