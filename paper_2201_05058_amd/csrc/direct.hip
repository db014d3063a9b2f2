// Exact sphere queries without building the 3-D fields.
//
// A query reads eight voxels of one slice's composite.  By the product
// structure of the humans' voxels (composite.hip), the composite at voxel
// (i, j, k) of slice s is
//   min(S(i,j,k), human_value(P_s(i, j), k)),
// where P_s is the slice's planar signed field of the humans' disk union
// (n_slices * nx * ny values, built by the planar kernels).  So a query
// needs four planar values and eight static values, and its answer is
// bit-identical to sampling the built fields (same integers, same fp32
// conversion, same fp64 interpolation).  Only the planes are built: at
// 256 x 256 x 128 they are 1/128 of the fields' voxels, and a planner's
// obstacle factors read a few thousand spheres per update.
#include <cmath>

#include "device_common.h"
#include "internal.h"
#include "query_device.h"

namespace pcsdf {

struct DirectArgs {
  const int32_t *S;  // static SSQ [V]
  const int32_t *P;  // planar fields [n_slices][ny][nx]
  const uint8_t *mask;  // answer only queries with mask[q] != 0 (nullable)
  int n_slices, nx, ny, nz, Kt, has_above;
  float hf;
  double h, ox, oy, oz, eps;
  const float *centre, *radius;
  const int32_t *slice;
  float *dist, *grad, *cost;
  uint8_t *status;
};

__device__ __forceinline__ void answer_direct(const DirectArgs &A, int q) {
  int s = A.slice[q];
  uint32_t st = 0;
  if (s < 0) {
    const float nan = __builtin_nanf("");
    A.dist[q] = nan;
    A.grad[3 * q] = nan;
    A.grad[3 * q + 1] = nan;
    A.grad[3 * q + 2] = nan;
    if (A.cost) A.cost[q] = nan;
    if (A.status) A.status[q] = (uint8_t)PCSDF_Q_SLICE_NEG;
    return;
  }
  if (s > A.n_slices - 1) {
    s = A.n_slices - 1;
    st |= PCSDF_Q_SLICE_CLAMPED;
  }
  const Cell C =
      cell_of(A.nx, A.ny, A.nz, A.h, A.ox, A.oy, A.oz, A.centre + 3 * q);
  st |= C.status;
  const int32_t *P = A.P + (int64_t)s * A.nx * A.ny;
  const HumanLayer hl[2] = {human_layer(C.idx[2], A.Kt, A.has_above),
                            human_layer(C.idx[2] + 1, A.Kt, A.has_above)};
  double c[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = C.idx[0] + a, j = C.idx[1] + b;
      const int32_t p = P[(int64_t)j * A.nx + i];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = C.idx[2] + e;
        const int32_t hv = human_value(p, hl[e]);
        const int32_t sv = A.S[((int64_t)k * A.ny + j) * A.nx + i];
        c[a][b][e] = (double)ssq_to_metres(min(sv, hv), A.hf);
      }
    }
  const Trilinear T = interpolate(c, C.fr);
  if (T.inf) {
    A.dist[q] = (float)T.D;
    A.grad[3 * q] = 0.f;
    A.grad[3 * q + 1] = 0.f;
    A.grad[3 * q + 2] = 0.f;
    if (A.cost) A.cost[q] = T.D > 0 ? 0.f : __builtin_inff();
    if (A.status) A.status[q] = (uint8_t)(st | PCSDF_Q_INF_CORNER);
    return;
  }
  const double dsph = T.D - (double)A.radius[q];
  A.dist[q] = (float)dsph;
  A.grad[3 * q] = (float)(T.g[0] / A.h);
  A.grad[3 * q + 1] = (float)(T.g[1] / A.h);
  A.grad[3 * q + 2] = (float)(T.g[2] / A.h);
  if (A.cost) {
    const double hc = A.eps - dsph;
    A.cost[q] = (float)(hc > 0.0 ? hc : 0.0);
  }
  if (A.status) A.status[q] = (uint8_t)st;
}

__global__ __launch_bounds__(256) void k_query_direct(DirectArgs A, int n) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < n && (!A.mask || A.mask[q])) answer_direct(A, q);
}

int direct_setup(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                 int32_t n_slices, int32_t n_humans, const double *xy_host,
                 double radius_m, double height_m, const int32_t *need,
                 hipStream_t s, DirectSet *out) {
  PlaneSet ps;
  int rc = planes_run(h, g, n_slices, n_humans, xy_host, radius_m, nullptr,
                      height_m, need, s, &ps);
  if (rc) return rc;
  out->P = ps.P;
  out->Kt = ps.Kt;
  out->has_above = ps.has_above;
  out->S = static_ssq;
  return PCSDF_OK;
}

int direct_from(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                const HumanSet &hs, int32_t n_slices, int32_t n_humans,
                const int32_t *need, hipStream_t s, DirectSet *out) {
  PlaneSet ps;
  int rc = planes_from(h, g, hs, n_slices, n_humans, need, s, &ps);
  if (rc) return rc;
  out->P = ps.P;
  out->Kt = ps.Kt;
  out->has_above = ps.has_above;
  out->S = static_ssq;
  return PCSDF_OK;
}

int launch_direct(Handle *h, const pcsdf_grid *g, const DirectSet &d,
                  int n_slices, int n_queries, const uint8_t *mask,
                  const float *centre, const float *radius,
                  const int32_t *slice, double eps, float *dist, float *grad,
                  uint8_t *status, float *cost, hipStream_t s) {
  if (n_queries <= 0) return PCSDF_OK;
  DirectArgs A;
  A.S = d.S;
  A.P = d.P;
  A.mask = mask;
  A.n_slices = n_slices;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.Kt = d.Kt;
  A.has_above = d.has_above;
  A.hf = (float)g->voxel_m;
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
  launch_timed(h, k_query_direct, dim3((unsigned)((n_queries + 255) / 256)),
               dim3(256), 0u, s, A, n_queries);
  return check_launch(h, "direct query");
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_query_spheres_direct(
    pcsdf_handle *hp, const pcsdf_grid *g, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t n_queries,
    const float *centre_dev, const float *radius_dev,
    const int32_t *slice_dev, double hinge_eps_m, float *dist_dev,
    float *grad_dev, uint8_t *status_dev, float *cost_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2)
    return fail(h, PCSDF_ERR_DIMS, "queries need at least 2 voxels per axis");
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (!std::isfinite(hinge_eps_m))
    return fail(h, PCSDF_ERR_NUMERIC, "hinge_eps_m must be finite");
  if (!static_ssq_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "static_ssq_dev is required");
  if (n_queries > 0 && (!centre_dev || !radius_dev || !slice_dev ||
                        !dist_dev || !grad_dev))
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "centre, radius, slice, dist and grad are required");
  if (((uintptr_t)static_ssq_dev | (uintptr_t)centre_dev |
       (uintptr_t)radius_dev | (uintptr_t)slice_dev | (uintptr_t)dist_dev |
       (uintptr_t)grad_dev | (uintptr_t)cost_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DirectSet d;
  if ((rc = direct_setup(h, g, static_ssq_dev, n_slices, n_humans,
                         human_xy_host, radius_m, height_m, nullptr, s, &d)))
    return rc;
  ProfScope pq(h, PCSDF_KERNEL_QUERY, s, true);
  return launch_direct(h, g, d, n_slices, n_queries, nullptr, centre_dev,
                       radius_dev, slice_dev, hinge_eps_m, dist_dev, grad_dev,
                       status_dev, cost_dev, s);
}
