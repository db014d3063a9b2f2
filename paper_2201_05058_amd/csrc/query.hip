// Sphere queries on the per-slice fields.  GPMP2's obstacle factors apply
// a hinge loss to the distance field sampled at the robot's collision
// spheres, and RHAP-GPMP2 hands every time index past the prediction
// horizon the last composite field.  Each lane answers one sphere: the
// slice is clamped, the centre mapped to fp64 grid coordinates, the eight
// fp32 corners of its cell gathered, and the trilinear value and its
// analytic gradient formed in fp64 from weighted corner differences (so no
// large interpolated values are subtracted).  This unit is built with
// -ffp-contract=off so every fp64 operation is rounded as written.
#include <cmath>

#include "internal.h"
#include "query_device.h"

namespace pcsdf {

struct QueryArgs {
  const float *sdf;  // [n_slices][V]
  int n_slices, nx, ny, nz;
  double h, ox, oy, oz, eps;
  const float *centre, *radius;
  const int32_t *slice;
  float *dist, *grad, *cost;
  uint8_t *status;
};

// Answers query q.
__device__ __forceinline__ void answer(const QueryArgs &A, int q) {
  const float *__restrict__ sdf = A.sdf;
  const float *__restrict__ centre = A.centre;
  const float *__restrict__ radius = A.radius;
  const int32_t *__restrict__ slice = A.slice;
  float *__restrict__ dist = A.dist;
  float *__restrict__ grad = A.grad;
  float *__restrict__ cost = A.cost;
  uint8_t *__restrict__ status = A.status;
  const int n_slices = A.n_slices, nx = A.nx, ny = A.ny, nz = A.nz;
  const double h = A.h, ox = A.ox, oy = A.oy, oz = A.oz, eps = A.eps;
  uint32_t st = 0;
  int s = slice[q];
  if (s < 0) {
    const float nan = __builtin_nanf("");
    dist[q] = nan;
    grad[3 * q] = nan;
    grad[3 * q + 1] = nan;
    grad[3 * q + 2] = nan;
    if (cost) cost[q] = nan;
    if (status) status[q] = (uint8_t)PCSDF_Q_SLICE_NEG;
    return;
  }
  if (s > n_slices - 1) {
    s = n_slices - 1;
    st |= PCSDF_Q_SLICE_CLAMPED;
  }
  const int64_t V = (int64_t)nx * ny * nz;
  const Trilinear T = trilinear(sdf + (int64_t)s * V, nx, ny, nz, h, ox, oy,
                                oz, centre + 3 * q);
  st |= T.status;
  if (T.inf) {
    dist[q] = (float)T.D;
    grad[3 * q] = 0.f;
    grad[3 * q + 1] = 0.f;
    grad[3 * q + 2] = 0.f;
    if (cost) cost[q] = T.D > 0 ? 0.f : __builtin_inff();
    if (status) status[q] = (uint8_t)(st | PCSDF_Q_INF_CORNER);
    return;
  }
  const double D = T.D, gx = T.g[0], gy = T.g[1], gz = T.g[2];
  const double dsph = D - (double)radius[q];
  dist[q] = (float)dsph;
  grad[3 * q] = (float)(gx / h);
  grad[3 * q + 1] = (float)(gy / h);
  grad[3 * q + 2] = (float)(gz / h);
  if (cost) {
    const double hc = eps - dsph;
    cost[q] = (float)(hc > 0.0 ? hc : 0.0);
  }
  if (status) status[q] = (uint8_t)st;
}

__global__ __launch_bounds__(256) void k_query(QueryArgs A, int n_queries) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < n_queries) answer(A, q);
}

// Queries list[0 .. *count) only.
__global__ __launch_bounds__(256) void k_query_list(
    QueryArgs A, const int32_t *__restrict__ list,
    const int32_t *__restrict__ count) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < *count) answer(A, list[t]);
}

static QueryArgs query_args(const pcsdf_grid *g, const float *sdf,
                            int n_slices, const float *centre,
                            const float *radius, const int32_t *slice,
                            double eps, float *dist, float *grad,
                            uint8_t *status, float *cost) {
  QueryArgs A;
  A.sdf = sdf;
  A.n_slices = n_slices;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.h = g->voxel_m;
  A.ox = g->origin_m[0];
  A.oy = g->origin_m[1];
  A.oz = g->origin_m[2];
  A.eps = eps;
  A.centre = centre;
  A.radius = radius;
  A.slice = slice;
  A.dist = dist;
  A.grad = grad;
  A.cost = cost;
  A.status = status;
  return A;
}

int launch_query_list(Handle *h, const pcsdf_grid *g, const float *sdf,
                      int n_slices, const int32_t *list,
                      const int32_t *count, int max_count,
                      const float *centre, const float *radius,
                      const int32_t *slice, double eps, float *dist,
                      float *grad, uint8_t *status, float *cost,
                      hipStream_t s) {
  if (max_count <= 0) return PCSDF_OK;
  const QueryArgs A = query_args(g, sdf, n_slices, centre, radius, slice, eps,
                                 dist, grad, status, cost);
  hipLaunchKernelGGL(k_query_list, dim3((unsigned)((max_count + 255) / 256)),
                     dim3(256), 0, s, A, list, count);
  return check_launch(h, "query list");
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_query_spheres(pcsdf_handle *hp, const pcsdf_grid *g,
                                   const float *sdf_dev, int32_t n_slices,
                                   int32_t n_queries, const float *centre_dev,
                                   const float *radius_dev,
                                   const int32_t *slice_dev,
                                   double hinge_eps_m, float *dist_dev,
                                   float *grad_dev, uint8_t *status_dev,
                                   float *cost_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2)
    return fail(h, PCSDF_ERR_DIMS, "queries need at least 2 voxels per axis");
  if (n_slices < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (!std::isfinite(hinge_eps_m))
    return fail(h, PCSDF_ERR_NUMERIC, "hinge_eps_m must be finite");
  if (n_queries == 0) return PCSDF_OK;
  if (!sdf_dev || !centre_dev || !radius_dev || !slice_dev || !dist_dev ||
      !grad_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "sdf, centre, radius, slice, dist and grad are required");
  if (((uintptr_t)sdf_dev | (uintptr_t)centre_dev | (uintptr_t)radius_dev |
       (uintptr_t)slice_dev | (uintptr_t)dist_dev | (uintptr_t)grad_dev |
       (uintptr_t)cost_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((n_queries + 255) / 256)), block(256);
  ProfScope ps(h, PCSDF_KERNEL_QUERY, s, true);
  const QueryArgs A =
      query_args(g, sdf_dev, n_slices, centre_dev, radius_dev, slice_dev,
                 hinge_eps_m, dist_dev, grad_dev, status_dev, cost_dev);
  launch_timed(h, k_query, grid, block, 0u, s, A, n_queries);
  return check_launch(h, "query_spheres");
}
