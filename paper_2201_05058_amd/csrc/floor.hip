// The environment collapsed to the floor plane (RHAP-GPMP2 section: for
// the human-trajectory predictor the maintained 3-D voxel grid is
// collapsed to 2-D and its EDT computed on the GPU): a pixel is occupied
// when any voxel of its column between layers z_lo and z_hi is, and the
// planar map goes through the static build's passes as a one-layer grid.
#include <cmath>

#include "internal.h"

namespace pcsdf {

__global__ __launch_bounds__(256) void k_collapse(
    const uint8_t *__restrict__ occ, int nx, int ny, int z_lo, int z_hi,
    uint8_t *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nx * ny) return;
  const size_t plane = (size_t)nx * ny;
  uint8_t any = 0;
  for (int k = z_lo; k <= z_hi; ++k) any |= occ[k * plane + p];
  out[p] = any ? 1 : 0;
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_build_floor_sdf(pcsdf_handle *hp, const pcsdf_grid *g,
                                     const uint8_t *occ_dev, int32_t z_lo,
                                     int32_t z_hi, int32_t *ssq_dev,
                                     float *sdf_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (!occ_dev || !ssq_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "occ_dev and ssq_dev are required");
  if (z_lo < 0 || z_hi >= g->nz || z_lo > z_hi)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "need 0 <= z_lo <= z_hi < nz");
  if (((uintptr_t)ssq_dev & 3) || ((uintptr_t)sdf_dev & 3))
    return fail(h, PCSDF_ERR_ALIGN, "ssq_dev/sdf_dev must be 4-byte aligned");
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t npx = (int64_t)g->nx * g->ny;
  if ((rc = ensure_buffer(h, h->union_buf, (size_t)npx, s))) return rc;
  uint8_t *flat = reinterpret_cast<uint8_t *>(h->union_buf.ptr);
  hipLaunchKernelGGL(k_collapse, dim3((unsigned)((npx + 255) / 256)),
                     dim3(256), 0, s, occ_dev, g->nx, g->ny, z_lo, z_hi,
                     flat);
  if ((rc = check_launch(h, "collapse"))) return rc;
  pcsdf_grid g2 = *g;
  g2.nz = 1;
  return pcsdf_build_static_sdf(hp, &g2, flat, ssq_dev, sdf_dev, stream);
}
