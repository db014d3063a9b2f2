// Compute-once-and-shift composite: the paper's own way of placing the
// humans (mapping section: each moving obstacle's field is a cylinder
// primitive's field computed once, and every composite is a parallel min
// of the environment field and the humans' fields at their predicted
// positions).
//
// Per human, its cylinder's exact signed field is computed once, at the
// sub-voxel phase of its first-slice position, in a window of
// (2 A_x + 1) x (2 A_y + 1) pixels around it (A = n + m, m = R/2^16 + 2):
// a planar signed EDT of the single disk (the same planar kernels as the
// per-slice path, with the window as the plane), the vertical part in
// closed form as in the composite.  At slice s the template is shifted by
// the whole number of voxels nearest to the human's displacement since the
// first slice, and the composite is
//   min(static, min over humans of the shifted templates),
// a human contributing nothing where its window does not reach.  Per
// slice the shifted templates are reduced to one plane (a min over humans
// per pixel), and the voxels stream through the composite's epilogue; no
// per-slice EDT runs.
//
// With whole-voxel motion, humans apart from each other and cylinders
// inside the grid, this equals the exact per-slice composite; otherwise it
// differs by the sub-voxel shift, the re-voxelisation at the first slice's
// phase, the unclipped template of a human straddling the grid's edge, and
// (inside overlapping humans) the min of separate signed fields.
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace pcsdf {

// P[s][j][i] = min over humans q of T_q[j - b_y][i - b_x] (INT32_MAX where
// no window reaches), with T [K][Wy][Wx] the planar templates and base
// [n_slices][K] = (b_x, b_y) the shifted windows.  The humans' value of a
// voxel is non-decreasing in its planar value, so the min over humans of
// their 3-D values is the 3-D value of this planar min, and the composite
// then streams exactly as for the per-slice planes.
__global__ __launch_bounds__(256) void k_template_planes(
    const int32_t *__restrict__ T, const int2 *__restrict__ base, int K,
    int Wx, int Wy, int nx, int ny, int64_t total, int32_t *__restrict__ P) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int64_t row = t / nx;  // s*ny + j
  const int i = (int)(t - row * nx);
  const int s = (int)(row / ny);
  const int j = (int)(row - (int64_t)s * ny);
  const size_t wplane = (size_t)Wx * Wy;
  int32_t m = kInf;
  for (int q = 0; q < K; ++q) {
    const int2 b = base[s * K + q];
    const int tu = i - b.x, tv = j - b.y;
    if (tu < 0 || tu >= Wx || tv < 0 || tv >= Wy) continue;
    m = min(m, T[q * wplane + (size_t)tv * Wx + tu]);
  }
  P[t] = m;
}

static bool to_fixed_t(double p, double o, double h, int64_t *out) {
  double t = p - o;
  t = t / h;
  t = t * 65536.0;
  if (!std::isfinite(t) || std::fabs(t) >= 4611686018427387904.0) return false;
  *out = (int64_t)std::nearbyint(t);
  return true;
}

static __int128 floor_div(__int128 a, int64_t b) {  // b > 0
  __int128 q = a / b;
  if ((a % b) != 0 && a < 0) --q;
  return q;
}

static int64_t clamp30(__int128 v) {  // beyond +-2^30 no window reaches
  const __int128 lim = (__int128)1 << 30;
  return (int64_t)(v < -lim ? -lim : (v > lim ? lim : v));
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_template_composite_sdf(
    pcsdf_handle *hp, const pcsdf_grid *g, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (!static_ssq_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "static_ssq_dev is required");
  if (!out_ssq_dev && !out_sdf_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "at least one of out_ssq_dev / out_sdf_dev is required");
  if (((uintptr_t)static_ssq_dev & 3) || ((uintptr_t)out_ssq_dev & 3) ||
      ((uintptr_t)out_sdf_dev & 3))
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  if (n_slices < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (n_humans < 0 || n_humans > kMaxHumans)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_humans must be in [0, 256]");
  if (n_humans > 0 && !human_xy_host)
    return fail(h, PCSDF_ERR_INVALID_ARG, "human_xy_host is required");
  const double hv = g->voxel_m;
  if (!std::isfinite(radius_m) || radius_m < 0 || !std::isfinite(height_m) ||
      height_m < 0)
    return fail(h, PCSDF_ERR_NUMERIC, "radius_m/height_m must be finite, >= 0");
  int64_t R, Hq;
  if (!to_fixed_t(radius_m, 0.0, hv, &R) || !to_fixed_t(height_m, 0.0, hv, &Hq))
    return fail(h, PCSDF_ERR_NUMERIC, "radius/height out of range");
  if (R >= (1LL << 31))
    return fail(h, PCSDF_ERR_NUMERIC, "radius_m/voxel_m must be < 32768");
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t V = (int64_t)nx * ny * nz;
  const int Kt =
      Hq >= 32768 ? (int)std::min<int64_t>((Hq - 32768) / 65536, nz - 1) : -1;
  const int K = Kt < 0 ? 0 : n_humans;
  const int has_above = Kt + 1 <= nz - 1;
  const int64_t m = (R >> 16) + 2;
  const int64_t Ax = nx + m, Ay = ny + m;
  const int Wx = (int)(2 * Ax + 1), Wy = (int)(2 * Ay + 1);

  // Host parameter block: window centres [K][2] int64, radii [K] int64,
  // shifts [n_slices][K] int2.
  const size_t nb = (size_t)n_slices * (K > 0 ? K : 1);
  std::vector<int64_t> blk(3 * (size_t)(K > 0 ? K : 1) + nb);
  int64_t *tx = blk.data();
  int64_t *rs = tx + 2 * (K > 0 ? K : 1);
  int2 *bases = reinterpret_cast<int2 *>(rs + (K > 0 ? K : 1));
  for (size_t t = 0; t < (size_t)n_slices * n_humans; ++t) {
    int64_t X, Y;
    if (!to_fixed_t(human_xy_host[2 * t], g->origin_m[0], hv, &X) ||
        !to_fixed_t(human_xy_host[2 * t + 1], g->origin_m[1], hv, &Y))
      return fail(h, PCSDF_ERR_NUMERIC,
                  "human position non-finite or out of range at index " +
                      std::to_string(t));
  }
  for (int k = 0; k < K; ++k) {
    int64_t X0, Y0;
    if (!to_fixed_t(human_xy_host[2 * k], g->origin_m[0], hv, &X0) ||
        !to_fixed_t(human_xy_host[2 * k + 1], g->origin_m[1], hv, &Y0))
      return fail(h, PCSDF_ERR_NUMERIC, "human position non-finite or out of "
                                        "range");
    const int64_t ax = (int64_t)floor_div(X0, 65536);
    const int64_t ay = (int64_t)floor_div(Y0, 65536);
    tx[2 * k] = X0 - 65536 * (ax - Ax);
    tx[2 * k + 1] = Y0 - 65536 * (ay - Ay);
    rs[k] = R;
    for (int s = 0; s < n_slices; ++s) {
      int64_t X, Y;
      const size_t t = (size_t)s * n_humans + k;
      if (!to_fixed_t(human_xy_host[2 * t], g->origin_m[0], hv, &X) ||
          !to_fixed_t(human_xy_host[2 * t + 1], g->origin_m[1], hv, &Y))
        return fail(h, PCSDF_ERR_NUMERIC,
                    "human position non-finite or out of range at index " +
                        std::to_string(t));
      const __int128 bx =
          (__int128)ax + floor_div((__int128)X - X0 + 32768, 65536) - Ax;
      const __int128 by =
          (__int128)ay + floor_div((__int128)Y - Y0 + 32768, 65536) - Ay;
      bases[(size_t)s * K + k] = make_int2((int)clamp30(bx), (int)clamp30(by));
    }
  }
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t blk_bytes = blk.size() * sizeof(int64_t);
  const size_t tbytes = (size_t)(K > 0 ? K : 1) * Wx * Wy * sizeof(int32_t);
  if ((rc = ensure_buffer(h, h->param_buf, blk_bytes, s))) return rc;
  if ((rc = ensure_buffer(h, h->tmpl_buf, 2 * tbytes, s))) return rc;
  if ((rc = ensure_buffer(h, h->chord_buf,
                          (size_t)(K > 0 ? K : 1) * Wy * sizeof(int2), s)))
    return rc;
  int64_t *dev = reinterpret_cast<int64_t *>(h->param_buf.ptr);
  if ((rc = acquire_staging(h, blk_bytes))) return rc;
  std::memcpy(h->pinned, blk.data(), blk_bytes);
  if (hipMemcpyAsync(dev, h->pinned, blk_bytes, hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return fail(h, PCSDF_ERR_HIP, "upload of the template parameters failed");
  if ((rc = release_staging(h, s))) return rc;
  int32_t *T = reinterpret_cast<int32_t *>(h->tmpl_buf.ptr);
  const int2 *bases_dev = reinterpret_cast<const int2 *>(dev + 3 * K);
  const size_t plane_bytes = (size_t)n_slices * nx * ny * sizeof(int32_t);
  if ((rc = ensure_buffer(h, h->plane_buf, plane_bytes, s))) return rc;
  int32_t *P = reinterpret_cast<int32_t *>(h->plane_buf.ptr);
  {
    ProfScope pp(h, PCSDF_KERNEL_PLANES, s);
    if (K > 0) {
      // one "slice" per human: its single disk in its window
      Centres C;
      C.xy = dev;
      C.Rs = dev + 2 * K;
      if ((rc = launch_planes(h, C, 1, false,
                              reinterpret_cast<int2 *>(h->chord_buf.ptr), T,
                              Wx, Wy, K, nullptr, s)))
        return rc;
    }
    const int64_t total = (int64_t)n_slices * nx * ny;
    hipLaunchKernelGGL(k_template_planes,
                       dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       T, bases_dev, K, Wx, Wy, nx, ny, total, P);
    if ((rc = check_launch(h, "template planes"))) return rc;
  }
  ProfScope ps(h, PCSDF_KERNEL_TEMPLATE, s);
  return launch_composite(h, g, static_ssq_dev, P, nullptr, Kt, has_above,
                          n_slices, out_ssq_dev, out_sdf_dev, s);
}
