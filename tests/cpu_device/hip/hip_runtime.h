// Host stand-in for the HIP names used by the library's device helpers, so
// that tests can compile that code with g++ and run it on the CPU.  One OS
// thread plays one workgroup of a single lane.  Test infrastructure only.
#pragma once
#include <sched.h>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <algorithm>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
struct float4 { float x, y, z, w; };
inline int2 make_int2(int a, int b) { return int2{a, b}; }
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
using std::min;
using std::max;
struct Dim3 { unsigned x = 0, y = 0, z = 0; };
extern thread_local Dim3 threadIdx, blockIdx, blockDim, gridDim;
inline void __syncthreads() {}
// the 24-bit multiplier: the low 24 bits of each operand, sign-extended
inline int __mul24(int a, int b) {
  return static_cast<int>(
      static_cast<unsigned>(static_cast<int>(static_cast<unsigned>(a) << 8) >> 8) *
      static_cast<unsigned>(static_cast<int>(static_cast<unsigned>(b) << 8) >> 8));
}
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_load(p, o, s) __atomic_load_n((p), (o))
#define __hip_atomic_store(p, v, o, s) __atomic_store_n((p), (v), (o))
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
#define __builtin_amdgcn_s_sleep(n) sched_yield()
#define __builtin_amdgcn_fence(o, s) __atomic_thread_fence(o)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
