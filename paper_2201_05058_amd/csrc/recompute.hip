// Full recompute per slice: the exact signed EDT of the union of the
// environment's occupied voxels and the humans' voxels, computed from
// scratch for every slice.  This is the baseline the paper measures its
// composite against (mapping section, Fig. 6: composite distance fields vs
// full distance-field computations per slice), done here with this
// library's own three-pass EDT instead of PBA.
//
// Per slice: the humans' voxels come from the same exact planar field as
// in the composite (a pixel is inside the disk union iff its planar value
// is negative; a voxel is a human voxel iff its pixel is and its layer is
// at most the cylinders' top layer), OR-ed into the environment's map; the
// union map then goes through the static build's x, y and z passes.
// Outside every obstacle the result equals the composite (the minimum of
// squared distances to two sets is the squared distance to their union);
// inside, it is the true depth in the union, where the composite takes the
// minimum of the two signed fields.
#include <cmath>

#include "internal.h"

namespace pcsdf {

// out[v] = occ[v] | (P[j][i] < 0 && k <= Kt), four voxels per lane.
__global__ __launch_bounds__(256) void k_union(const uint8_t *__restrict__ occ,
                                               const int32_t *__restrict__ P,
                                               uint32_t nx, uint32_t ny,
                                               int Kt, uint32_t V,
                                               uint8_t *__restrict__ out) {
  const uint32_t v0 = (blockIdx.x * 256u + threadIdx.x) * 4u;
  if (v0 >= V) return;
#pragma unroll
  for (uint32_t d = 0; d < 4; ++d) {
    const uint32_t v = v0 + d;
    if (v >= V) break;
    const uint32_t row = v / nx;
    const uint32_t i = v - row * nx;
    const uint32_t k = row / ny;
    const uint32_t j = row - k * ny;
    const bool hum = (int)k <= Kt && P[(size_t)j * nx + i] < 0;
    out[v] = (occ[v] != 0 || hum) ? 1 : 0;
  }
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_recompute_sdf(pcsdf_handle *hp, const pcsdf_grid *g,
                                   const uint8_t *static_occ_dev,
                                   int32_t n_slices, int32_t n_humans,
                                   const double *human_xy_host,
                                   double radius_m, double height_m,
                                   int32_t *out_ssq_dev, float *out_sdf_dev,
                                   void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (!static_occ_dev || !out_ssq_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "static_occ_dev and out_ssq_dev are required");
  if (((uintptr_t)out_ssq_dev & 3) || ((uintptr_t)out_sdf_dev & 3))
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  PlaneSet ps;
  if ((rc = planes_run(h, g, n_slices, n_humans, human_xy_host, radius_m,
                       nullptr, height_m, nullptr, s, &ps)))
    return rc;
  const int64_t V = (int64_t)g->nx * g->ny * g->nz;
  if ((rc = ensure_buffer(h, h->union_buf, (size_t)V, s))) return rc;
  uint8_t *un = reinterpret_cast<uint8_t *>(h->union_buf.ptr);
  const size_t plane = (size_t)g->nx * g->ny;
  ProfScope pr(h, PCSDF_KERNEL_RECOMPUTE, s);
  for (int32_t j = 0; j < n_slices; ++j) {
    hipLaunchKernelGGL(k_union, dim3((unsigned)((V + 1023) / 1024)),
                       dim3(256), 0, s, static_occ_dev, ps.P + j * plane,
                       (uint32_t)g->nx, (uint32_t)g->ny, ps.Kt, (uint32_t)V,
                       un);
    if ((rc = check_launch(h, "union"))) return rc;
    if ((rc = pcsdf_build_static_sdf(hp, g, un, out_ssq_dev + j * V,
                                     out_sdf_dev ? out_sdf_dev + j * V
                                                 : nullptr,
                                     stream)))
      return rc;
  }
  return PCSDF_OK;
}
