// Host stand-in for <hip/hip_ext.h>: the CPU tests use no launch helper of
// the library; only the names its declarations mention are given here.
// Test infrastructure only.
#pragma once
#include "hip_runtime.h"
#ifndef PCSDF_HOST_DIM3
#define PCSDF_HOST_DIM3
struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
#endif
