// Device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcsdf {

// Saturating int32 addition.
__device__ __forceinline__ int32_t add_sat(int32_t a, int32_t b) {
#if defined(__clang__)
  return __builtin_elementwise_add_sat(a, b);
#else  // a host compiler building the device code for CPU tests
  const int64_t s = (int64_t)a + b;
  return s > INT32_MAX ? INT32_MAX : (s < INT32_MIN ? INT32_MIN : (int32_t)s);
#endif
}

// Correctly rounded square root of a float a that is 0 or at least 1 (here
// the magnitude of an integer squared distance).  The hardware root r is
// within one ulp for such inputs, so the rounded root is r or one of its
// neighbouring floats r- < r < r+; Tuckerman's rounding test picks it:
// r- when a <= r- r, r+ when a > r r+, else r (each residual a - r' r
// formed by one fused multiply-add, whose sign is exact).  For a = 0 the
// hardware returns 0, r- is a NaN, and both tests keep 0.  No scaling is
// needed: the inputs are never subnormal.
__device__ __forceinline__ float sqrt_rn_nonneg(float a) {
#if defined(__clang__)
  const float r = __builtin_amdgcn_sqrtf(a);
#elif defined(PCSDF_HOST_ROOT_START)  // CPU test of the rounding step
  const float r = PCSDF_HOST_ROOT_START(a);
#else  // a host compiler building the device code for CPU tests
  const float r = __builtin_sqrtf(a);
#endif
  const float rm = __builtin_bit_cast(float, __builtin_bit_cast(int32_t, r) - 1);
  const float rp = __builtin_bit_cast(float, __builtin_bit_cast(int32_t, r) + 1);
  const float em = __builtin_fmaf(-rm, r, a);
  const float ep = __builtin_fmaf(-rp, r, a);
  const float lo = em <= 0.f ? rm : r;
  return ep > 0.f ? rp : lo;
}

// Signed squared voxel distance -> signed metres:
// F(x) = sign(x) * ((float)h * sqrtf(|x|)), +-inf for +-INT32_MAX.
// The square root is correctly rounded, then one fp32 multiply.  |x| is
// below 2^22 for grids of at most 1024 voxels per axis, so its conversion
// is exact; +-INT32_MAX converts to +-2^31, which no distance reaches and
// which is replaced by infinity before the root (whose rounding test keeps
// it: both residuals are NaN), so that no lane branches.
__device__ __forceinline__ float ssq_to_metres(int32_t x, float hf) {
  const float xf = (float)x;
  const float a0 = __builtin_fabsf(xf);
  const float a = a0 == 2147483648.0f ? __builtin_inff() : a0;
  return __builtin_copysignf(hf * sqrt_rn_nonneg(a), xf);
}

// The humans' signed value at layer k is a function of the pixel's planar
// signed value p (E_D outside the disk union D, -E of its complement
// inside, +-INT32_MAX when the other set is empty) and two constants of
// the layer.  At or below the cylinders' top layer Kt: p outside the
// disks, and inside the larger (nearer to zero) of p and -(Kt+1-k)^2, the
// squared distance to the free layer above (none when Kt is the grid's
// last layer); together, max(p, lo).  Above Kt: (k-Kt)^2 plus the planar
// distance outside the disks, (k-Kt)^2 over them; together, max(p, 0) +
// add.  The addition saturates, so that p = INT32_MAX (no human voxel in
// the slice) stays INT32_MAX.
struct HumanLayer {
  int32_t lo, add;
};
__device__ __forceinline__ HumanLayer human_layer(int k, int Kt,
                                                  int has_above) {
  const int dz = k - Kt;  // > 0 above the cylinders
  const int dzp = max(dz, 0);
  const int upp = max(Kt + 1 - k, 0);  // 0 above the cylinders
  HumanLayer t;
  t.lo = has_above ? -(upp * upp) : (dz > 0 ? 0 : -INT32_MAX);
  t.add = dzp * dzp;
  return t;
}
__device__ __forceinline__ int32_t human_value(int32_t p, HumanLayer t) {
  return add_sat(max(p, t.lo), t.add);
}

}  // namespace pcsdf
