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
  const float a = (float)(x < 0 ? -x : x);  // exact: |x| < 2^24
  const float r = hf * sqrtf(a);
  const float m = (x == INT32_MAX || x == -INT32_MAX) ? __builtin_inff() : r;
  return x < 0 ? -m : m;
}

// Value of the humans' signed field at a voxel of layer k whose planar
// signed value is p (E_D outside D, -E_{Gxy\D} inside, +-INT32_MAX if the other
// set is empty).  dz2o = max(0, k-Kt)^2; zin = (k <= Kt); dz2i =
// (Kt+1-k)^2 when layer Kt+1 exists, else INT32_MAX.
__device__ __forceinline__ int32_t human_value(int32_t p, int dz2o, bool zin,
                                               int32_t dz2i) {
  // Written as selects (no branches): p + dz2o outside the disks (wrapping
  // arithmetic, used only when p < INT32_MAX), the top of the cylinders
  // above them, min(-p, dz2i) negated inside (-p is INT32_MAX when the
  // disks cover the plane), INT32_MAX when the slice has no human voxel.
  const int32_t outside = (int32_t)((uint32_t)p + (uint32_t)dz2o);
  const int32_t din = -p;  // p >= -INT32_MAX, so no overflow
  const int32_t inside = zin ? -(din < dz2i ? din : dz2i) : dz2o;
  const int32_t r = p > 0 ? outside : inside;
  return p == INT32_MAX ? INT32_MAX : r;
}

}  // namespace pcsdf
