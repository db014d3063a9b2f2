// Trilinear sampling of one fp32 field at a point, in fp64: the corners of
// the point's cell are promoted to fp64, the value is the weighted sum and
// the gradient (per voxel) the weighted sum of corner differences along
// each axis.  Coordinates outside the span of voxel centres are clamped
// (status bits 1, 2, 4 for x, y, z).  Units that include this header are
// built with -ffp-contract=off so every fp64 operation rounds as written.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcsdf {

struct Trilinear {
  double D;       // interpolated value (or the infinite corner's value)
  double g[3];    // dD/dx per voxel along x, y, z (0 when inf)
  uint32_t status;
  bool inf;       // a corner is infinite: D is that corner's value
};

// The cell of point p: lower corner idx[3], fractions fr[3], clamp bits.
struct Cell {
  int idx[3];
  double fr[3];
  uint32_t status;
};

__device__ __forceinline__ Cell cell_of(int nx, int ny, int nz, double h,
                                        double ox, double oy, double oz,
                                        const float *__restrict__ p) {
  Cell C;
  C.status = 0;
  const int n[3] = {nx, ny, nz};
  const double o[3] = {ox, oy, oz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double gc = ((double)p[a] - o[a]) / h - 0.5;
    if (gc < 0.0) {
      gc = 0.0;
      C.status |= 1u << a;
    } else if (gc > (double)(n[a] - 1)) {
      gc = (double)(n[a] - 1);
      C.status |= 1u << a;
    }
    int i = (int)floor(gc);
    if (i > n[a] - 2) i = n[a] - 2;
    C.idx[a] = i;
    C.fr[a] = gc - (double)i;
  }
  return C;
}

// Value and per-voxel gradient from the eight corners c[a][b][e] (a along
// x, b along y, e along z) of a cell with fractions fr.
__device__ __forceinline__ Trilinear interpolate(const double c[2][2][2],
                                                 const double fr[3]) {
  Trilinear T;
  T.status = 0;
  T.inf = false;
  T.D = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        if (!T.inf && isinf(c[a][b][e])) {
          T.inf = true;
          T.D = c[a][b][e];
        }
  T.g[0] = T.g[1] = T.g[2] = 0.0;
  if (T.inf) return T;
  double w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a][0] = 1.0 - fr[a];
    w[a][1] = fr[a];
  }
  double D = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) D += w[0][a] * w[1][b] * w[2][e] * c[a][b][e];
  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int e = 0; e < 2; ++e)
      gx += w[1][b] * w[2][e] * (c[1][b][e] - c[0][b][e]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int e = 0; e < 2; ++e)
      gy += w[0][a] * w[2][e] * (c[a][1][e] - c[a][0][e]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      gz += w[0][a] * w[1][b] * (c[a][b][1] - c[a][b][0]);
  T.D = D;
  T.g[0] = gx;
  T.g[1] = gy;
  T.g[2] = gz;
  return T;
}

__device__ __forceinline__ Trilinear trilinear(const float *__restrict__ field,
                                               int nx, int ny, int nz,
                                               double h, double ox, double oy,
                                               double oz,
                                               const float *__restrict__ p) {
  const Cell C = cell_of(nx, ny, nz, h, ox, oy, oz, p);
  const int64_t base = ((int64_t)C.idx[2] * ny + C.idx[1]) * nx + C.idx[0];
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  double c[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        c[a][b][e] = (double)field[base + a + b * sy + e * sz];
  Trilinear T = interpolate(c, C.fr);
  T.status = C.status;
  return T;
}

}  // namespace pcsdf
