// Exact sphere queries without building any field.
//
// A query reads eight voxels of one slice's composite.  By the product
// structure of the humans' voxels (composite.hip), the composite at voxel
// (i, j, k) of slice s is
//   min(S(i,j,k), human_value(P_s(i, j), k)),
// where P_s(i, j) is the planar signed field of the slice's disk union at
// pixel (i, j) -- a function of the slice's chords alone (plane_device.h:
// nearest chord by row search outside the disks, nearest uncovered pixel
// by row search inside).  So a query needs the planar value of four pixels
// and eight reads of the static field, and the answer is bit-identical to
// sampling the built fields (same integers, same fp32 conversion, same
// fp64 interpolation).  Only the chords of the slices are built.
//
// A planner's obstacle factors read a few thousand spheres per update,
// while the fields of all slices hold n x V voxels: answering the queries
// directly skips almost all of the composite's memory traffic.
#include <cmath>

#include "device_common.h"
#include "internal.h"
#include "plane_device.h"
#include "query_device.h"

namespace pcsdf {

struct DirectArgs {
  const int32_t *S;     // static SSQ [V]
  const int2 *chords;   // [n_slices][K][ny]
  const int64_t *xy;    // fixed-point centres [n_slices][K][2]
  const int64_t *Rs;    // fixed-point radius per slice
  int K, n_slices, nx, ny, nz, Kt, has_above;
  float hf;
  double h, ox, oy, oz, eps;
  const float *centre, *radius;
  const int32_t *slice;
  float *dist, *grad, *cost;
  uint8_t *status;
};

// Disk bounding boxes of one slice, computed when asked for.
struct BoxesOfSlice {
  const int64_t *xy;  // this slice's [K][2]
  int64_t R;
  int nx, ny;
  __device__ __forceinline__ int4 operator[](int k) const {
    return disk_box(xy[2 * k], xy[2 * k + 1], R, nx, ny);
  }
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
  const GlobalTab ch{A.chords + (int64_t)s * A.K * A.ny};
  const BoxesOfSlice box{A.xy + (int64_t)s * A.K * 2, A.Rs[s], A.nx, A.ny};
  double c[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = C.idx[0] + a, j = C.idx[1] + b;
      int32_t P = kInfP;  // no human voxel in the slice
      if (A.K > 0)
        P = plane_value_rf(ch, box,
                           RowFreeChords<GlobalTab>{ch, A.K, A.ny, A.nx, i},
                           A.K, A.nx, A.ny, i, j);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = C.idx[2] + e;
        const int dzo = k > A.Kt ? k - A.Kt : 0;
        const int32_t dz2i =
            A.has_above ? (A.Kt + 1 - k) * (A.Kt + 1 - k) : kInf;
        const int32_t hv = human_value(P, dzo * dzo, k <= A.Kt, dz2i);
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
  if (q < n) answer_direct(A, q);
}

__global__ __launch_bounds__(256) void k_query_direct_list(
    DirectArgs A, const int32_t *__restrict__ list,
    const int32_t *__restrict__ count) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < *count) answer_direct(A, list[t]);
}

int direct_setup(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                 int32_t n_slices, int32_t n_humans, const double *xy_host,
                 double radius_m, double height_m, const int32_t *need,
                 hipStream_t s, DirectSet *out) {
  HumanSet hs;
  int rc = humans_upload(h, g, n_slices, n_humans, xy_host, radius_m, nullptr,
                         height_m, s, &hs);
  if (rc) return rc;
  ProfScope pp(h, PCSDF_KERNEL_PLANES, s);
  if ((rc = launch_chords(h, hs.xy, hs.K, hs.Rs, hs.chords, g->nx, g->ny,
                          n_slices, need, s)))
    return rc;
  out->hs = hs;
  out->S = static_ssq;
  return PCSDF_OK;
}

static DirectArgs direct_args(const pcsdf_grid *g, const DirectSet &d,
                              int n_slices, const float *centre,
                              const float *radius, const int32_t *slice,
                              double eps, float *dist, float *grad,
                              uint8_t *status, float *cost) {
  DirectArgs A;
  A.S = d.S;
  A.chords = d.hs.chords;
  A.xy = d.hs.xy;
  A.Rs = d.hs.Rs;
  A.K = d.hs.K;
  A.n_slices = n_slices;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.Kt = d.hs.Kt;
  A.has_above = d.hs.has_above;
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
  return A;
}

int launch_direct_list(Handle *h, const pcsdf_grid *g, const DirectSet &d,
                       int n_slices, const int32_t *list,
                       const int32_t *count, int max_count,
                       const float *centre, const float *radius,
                       const int32_t *slice, double eps, float *dist,
                       float *grad, uint8_t *status, float *cost,
                       hipStream_t s) {
  if (max_count <= 0) return PCSDF_OK;
  const DirectArgs A = direct_args(g, d, n_slices, centre, radius, slice, eps,
                                   dist, grad, status, cost);
  hipLaunchKernelGGL(k_query_direct_list,
                     dim3((unsigned)((max_count + 255) / 256)), dim3(256), 0,
                     s, A, list, count);
  return check_launch(h, "direct query list");
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
  if (n_queries == 0) return PCSDF_OK;
  const DirectArgs A =
      direct_args(g, d, n_slices, centre_dev, radius_dev, slice_dev,
                  hinge_eps_m, dist_dev, grad_dev, status_dev, cost_dev);
  ProfScope pq(h, PCSDF_KERNEL_QUERY, s);
  hipLaunchKernelGGL(k_query_direct, dim3((unsigned)((n_queries + 255) / 256)),
                     dim3(256), 0, s, A, n_queries);
  return check_launch(h, "direct query");
}
