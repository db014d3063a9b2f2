// Obstacle factors of the planner (RHAP-GPMP2 section: every time-indexed
// obstacle factor reads the composite field of its time index, the last
// field past the horizon; human-trajectory section: GPMP2's hinge loss on
// the distance field penalises states close to obstacles).
//
// For support state i and collision sphere j:
//   e_ij = max(0, eps - (d_s(c_ij) - r_j)),  s = clamp(slice_i, 0, n-1),
//   J_ij = -grad d_s(c_ij) where e_ij > 0, else 0,
//   cost_i = sum_j 0.5 (e_ij / sigma)^2.
// One wave per support state: each lane samples spheres (the same fp64
// trilinear sampling as the sphere queries), writes their errors and
// Jacobians, and the wave sums the state's cost in fp64.
#include <cmath>

#include "internal.h"
#include "query_device.h"

namespace pcsdf {

struct FactorArgs {
  const float *sdf;
  int n_slices, nx, ny, nz;
  double h, ox, oy, oz, eps, inv_sigma;
  int n_states, n_spheres;
  const float *centre, *radius;
  const int32_t *slice;
  float *err, *jac;
  double *cost;
};

__global__ __launch_bounds__(256) void k_factors(FactorArgs A) {
  const int wave = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= A.n_states) return;  // uniform over the wave
  const int i = wave;
  int s = A.slice[i];
  const bool neg = s < 0;
  if (s > A.n_slices - 1) s = A.n_slices - 1;
  const int64_t V = (int64_t)A.nx * A.ny * A.nz;
  const float *field = A.sdf + (int64_t)(neg ? 0 : s) * V;
  double acc = 0.0;
  for (int j = lane; j < A.n_spheres; j += 64) {
    const int64_t q = (int64_t)i * A.n_spheres + j;
    float e, j0 = 0.f, j1 = 0.f, j2 = 0.f;
    if (neg) {
      const float nan = __builtin_nanf("");
      e = j0 = j1 = j2 = nan;
    } else {
      const Trilinear T = trilinear(field, A.nx, A.ny, A.nz, A.h, A.ox, A.oy,
                                    A.oz, A.centre + 3 * q);
      if (T.inf) {
        e = T.D > 0 ? 0.f : __builtin_inff();
      } else {
        const double dsph = T.D - (double)A.radius[j];
        const double hc = A.eps - dsph;
        e = (float)(hc > 0.0 ? hc : 0.0);
        if (e > 0.f) {
          j0 = -(float)(T.g[0] / A.h);
          j1 = -(float)(T.g[1] / A.h);
          j2 = -(float)(T.g[2] / A.h);
        }
      }
    }
    A.err[q] = e;
    A.jac[3 * q] = j0;
    A.jac[3 * q + 1] = j1;
    A.jac[3 * q + 2] = j2;
    const double r = (double)e * A.inv_sigma;
    acc += 0.5 * r * r;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) A.cost[i] = acc;
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_obstacle_factors(
    pcsdf_handle *hp, const pcsdf_grid *g, const float *sdf_dev,
    int32_t n_slices, int32_t n_states, int32_t n_spheres,
    const float *centre_dev, const float *radius_dev,
    const int32_t *state_slice_dev, double eps_m, double sigma,
    float *err_dev, float *jac_dev, double *cost_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2)
    return fail(h, PCSDF_ERR_DIMS, "factors need at least 2 voxels per axis");
  if (n_slices < 1 || n_states < 0 || n_spheres < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "need n_slices >= 1, n_states >= 0, n_spheres >= 0");
  if ((int64_t)n_states * n_spheres > INT32_MAX)
    return fail(h, PCSDF_ERR_INVALID_ARG, "too many sphere-state pairs");
  if (!std::isfinite(eps_m) || !std::isfinite(sigma) || !(sigma > 0))
    return fail(h, PCSDF_ERR_NUMERIC, "eps must be finite and sigma > 0");
  if (n_states == 0) return PCSDF_OK;
  if (!sdf_dev || !state_slice_dev || !cost_dev ||
      (n_spheres > 0 && (!centre_dev || !radius_dev || !err_dev || !jac_dev)))
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "sdf, centre, radius, slice, err, jac and cost are required");
  if (((uintptr_t)sdf_dev | (uintptr_t)centre_dev | (uintptr_t)radius_dev |
       (uintptr_t)state_slice_dev | (uintptr_t)err_dev | (uintptr_t)jac_dev) &
          3 ||
      ((uintptr_t)cost_dev & 7))
    return fail(h, PCSDF_ERR_ALIGN,
                "device buffers must be 4-byte (cost: 8-byte) aligned");
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FactorArgs A;
  A.sdf = sdf_dev;
  A.n_slices = n_slices;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.h = g->voxel_m;
  A.ox = g->origin_m[0];
  A.oy = g->origin_m[1];
  A.oz = g->origin_m[2];
  A.eps = eps_m;
  A.inv_sigma = 1.0 / sigma;
  A.n_states = n_states;
  A.n_spheres = n_spheres;
  A.centre = centre_dev;
  A.radius = radius_dev;
  A.slice = state_slice_dev;
  A.err = err_dev;
  A.jac = jac_dev;
  A.cost = cost_dev;
  const unsigned blocks = (unsigned)(((int64_t)n_states * 64 + 255) / 256);
  ProfScope ps(h, PCSDF_KERNEL_FACTORS, s);
  hipLaunchKernelGGL(k_factors, dim3(blocks), dim3(256), 0, s, A);
  return check_launch(h, "obstacle factors");
}
