// Predicted composite fields: one exact signed field of the humans per
// time slice, min-composited with the environment field (mapping section:
// a parallel min between the environment field and the humans' fields at
// their predicted positions; RHAP-GPMP2 section: a sequence of n such
// fields, one per slice).
//
// The humans are vertical cylinders sharing one radius and height, all
// standing on the grid's floor, so a slice's human voxels form a product
// set O_h = D x Z: D is the union of voxelised disks in the xy plane and
// Z = {0..Kt} the voxel layers whose centres lie under the cylinder top.
// The squared distance to a product set splits into one term per factor,
// so for every voxel (i, j, k):
//   outside:  E_{O_h}(i,j,k)    = E_D(i,j) + max(0, k - Kt)^2
//   inside:   E_{G\O_h}(i,j,k)  = min(E_{Gxy\D}(i,j), (Kt + 1 - k)^2)
// (the complement of D x Z in the grid is (Gxy\D) x Gz  union  Gxy x (Gz\Z),
// and the second term is absent when Z reaches the grid top).  This is
// the z pass of the separable EDT done in closed form: the column input
// is constant on 0..Kt and empty elsewhere, and its lower envelope is that
// constant plus the squared distance to the interval.  So the exact 3-D
// field of the humans needs only a 2-D signed EDT per slice (planes.hip:
// each disk's chord per row from an exact integer square root of the
// voxelisation predicate, a row pass giving every pixel's distance to the
// nearest pixel outside the disks, and a bounded per-pixel search over
// rows for both signs), and the per-voxel work is a streaming epilogue:
//   read the static field once, then for every slice compute the humans'
//   value from the slice's plane, take the signed min, convert to metres
//   and write both outputs.
// The epilogue moves the compulsory bytes only: 4 B of static field per
// voxel (read once for all slices) and 8 B per voxel-slice of output; the
// planes (nx*ny*4 B per slice) stay in cache.  When V is odd a pack of one
// slice's voxels would start at a different alignment in every slice, so
// k_composite_flat walks the flattened outputs [n][V] in aligned packs
// instead, reading the static field per voxel-slice.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "composite_device.h"
#include "device_common.h"
#include "internal.h"

namespace pcsdf {

// The 16-bit copy of the static field: S16[v] = S[v] where |S[v]| <=
// 32767, else kS16Far.  Thread t converts voxels 4t .. 4t+3 (S16 is
// 256-byte aligned; S is read in 16-byte packs when it is so aligned).
__global__ __launch_bounds__(256) void k_static16(
    const int32_t *__restrict__ S, int16_t *__restrict__ S16, uint32_t V) {
  const uint32_t v = (blockIdx.x * 256u + threadIdx.x) * 4u;
  if (v >= V) return;
  auto c16 = [](int32_t x) -> uint32_t {
    return (uint32_t)(uint16_t)(x >= -32767 && x <= 32767 ? x : kS16Far);
  };
  if (v + 3 < V && !((uintptr_t)S & 15)) {
    const pk_i32x4 x = ld_global(reinterpret_cast<const pk_i32x4 *>(S + v));
    pk_i32x2 w;
    w[0] = (int32_t)(c16(x[0]) | c16(x[1]) << 16);
    w[1] = (int32_t)(c16(x[2]) | c16(x[3]) << 16);
    *reinterpret_cast<pk_i32x2 *>(S16 + v) = w;
  } else {
    for (uint32_t e = v; e < V && e < v + 4; ++e) S16[e] = (int16_t)c16(S[e]);
  }
}

// Slices with need[sl] == 0 are skipped when `need` is non-null.  Thread g
// handles voxels VEC g .. VEC g + VEC - 1 (VEC divides V); kGather reads
// their planar values one by one (VEC does not divide nx ny); with S16
// the static values come from the 16-bit copy.
template <int VEC, bool kGather, bool kSsq, bool kSdf>
__global__ __launch_bounds__(256) void k_composite(
    const int32_t *__restrict__ S, const int32_t *__restrict__ P,
    const int32_t *__restrict__ need,
    int32_t *__restrict__ oc, float *__restrict__ of, uint32_t plane,
    int n_slices, int G, int Kt, int has_above, float hf, uint32_t V,
    int order, const int16_t *__restrict__ S16) {
  // order 0: block (chunk, group) = (blockIdx.x, blockIdx.y), so the
  // blocks in flight write the same few slices over consecutive chunks.
  // order 1 (one-dimensional grid): blocks 8 apart take chunks x, x + 8,
  // ... (x = block mod 8) and, for each, its slice groups one after the
  // other.  The dispatcher places block b on XCD b mod 8, so the groups of
  // a chunk run on one XCD in close succession and re-read the chunk's
  // static field from that XCD's L2 rather than from HBM; in exchange the
  // blocks in flight write every slice at once.
  uint32_t chunk, grp;
  if (order) {
    const uint32_t ng = (uint32_t)((n_slices + G - 1) / G);
    const uint32_t j = blockIdx.x >> 3, cj = j / ng;
    grp = j - cj * ng;
    chunk = cj * 8 + (blockIdx.x & 7);
  } else {
    chunk = blockIdx.x;
    grp = blockIdx.y;
  }
  const uint32_t g = chunk * 256u + threadIdx.x;
  const uint32_t v0 = g * VEC;
  if (v0 >= V) return;
  const int s_begin = (int)grp * G;
  const int s_end = min(n_slices, s_begin + G);
  if (need) {  // skip the static read when none of the block's slices is due
    bool any = false;
    for (int sl = s_begin; sl < s_end; ++sl) any = any || need[sl] != 0;
    if (!any) return;
  }
  if (need)
    composite_pack<VEC, kGather, kSsq, kSdf, true>(
        S, P, need, oc, of, plane, V, v0, s_begin, s_end, Kt, has_above, hf);
  else
    composite_pack<VEC, kGather, kSsq, kSdf, false>(
        S, P, need, oc, of, plane, V, v0, s_begin, s_end, Kt, has_above, hf,
        S16);
}

template <int VEC, bool kGather>
static void launch_comp(Handle *h, const int32_t *S, const int32_t *P,
                        const int32_t *need, int32_t *oc, float *of,
                        uint32_t plane, int n, int G, int Kt, int has_above,
                        float hf, uint32_t V, const int16_t *S16,
                        hipStream_t s) {
  const uint32_t nthreads = V / VEC;
  const uint64_t chunks = (nthreads + 255) / 256, ng = (n + G - 1) / G;
  const uint64_t flat = (chunks + 7) / 8 * 8 * ng;
  const int order = h->tuning.composite_order == 1 && flat < (1ull << 31);
  const dim3 grid = order ? dim3((unsigned)flat) : dim3((unsigned)chunks,
                                                        (unsigned)ng);
  const dim3 block(256);
  if (oc && of)
    launch_timed(h, k_composite<VEC, kGather, true, true>, grid, block, 0u,
                 s, S, P, need, oc, of, plane, n, G, Kt, has_above, hf, V,
                 order, S16);
  else if (oc)
    launch_timed(h, k_composite<VEC, kGather, true, false>, grid, block, 0u,
                 s, S, P, need, oc, of, plane, n, G, Kt, has_above, hf, V,
                 order, S16);
  else
    launch_timed(h, k_composite<VEC, kGather, false, true>, grid, block, 0u,
                 s, S, P, need, oc, of, plane, n, G, Kt, has_above, hf, V,
                 order, S16);
}

// The same composite over the flattened outputs [n][V] in aligned packs of
// four, for grids whose V is odd (so that a pack of one slice's voxels
// would start at a different alignment in every slice).
// Pack t holds flat positions 4t .. 4t+3, each its own (slice, voxel): the
// static field is read per voxel-slice (from the caches for the slices
// after the first) so that every store is one aligned 16-byte pack.  The
// output bases are 16-byte aligned; a last partial pack is stored element
// by element.  N = n V < 2^32 - 4.
template <bool kSsq, bool kSdf>
__global__ __launch_bounds__(256) void k_composite_flat(
    const int32_t *__restrict__ S, const int32_t *__restrict__ P,
    int32_t *__restrict__ oc, float *__restrict__ of, uint32_t plane,
    uint32_t V, uint64_t N, int Kt, int has_above, float hf) {
  typedef uint32_t U;
  const U t = (U)blockIdx.x * 256u + threadIdx.x;
  const U f0 = t * 4u;
  if ((uint64_t)f0 >= N) return;
  U sl = f0 / V;
  uint32_t v = (uint32_t)(f0 - sl * V);
  uint32_t k = v / plane;
  uint32_t pix = v - k * plane;
  pk_i32x4 c;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if ((uint64_t)f0 + e < N) {
      const int32_t p = P[(size_t)sl * plane + pix];
      c[e] = min(S[v], human_value(p, human_layer((int)k, Kt, has_above)));
    } else {
      c[e] = 0;
    }
    // next flat position (V may be below four: a pack may span slices)
    ++v;
    if (++pix == plane) {
      pix = 0;
      ++k;
    }
    while (v >= V) {
      v -= V;
      ++sl;
      k = v / plane;
      pix = v - k * plane;
    }
  }
  pk_f32x4 fv;
#pragma unroll
  for (int e = 0; e < 4; ++e) fv[e] = ssq_to_metres(c[e], hf);
  if ((uint64_t)f0 + 4 <= N) {
    if (kSsq) store_i32<4>(oc + f0, c);
    if (kSdf) store_f32<4>(of + f0, fv);
  } else {
    for (int e = 0; (uint64_t)f0 + e < N; ++e) {
      if (kSsq) oc[f0 + e] = c[e];
      if (kSdf) of[f0 + e] = fv[e];
    }
  }
}

static void launch_comp_flat(Handle *h, const int32_t *S, const int32_t *P,
                             int32_t *oc, float *of, uint32_t plane,
                             uint32_t V, uint64_t N, int Kt, int has_above,
                             float hf, hipStream_t s) {
  const uint64_t packs = (N + 3) / 4;
  const dim3 grid((unsigned)((packs + 255) / 256)), block(256);
  if (oc && of)
    launch_timed(h, k_composite_flat<true, true>, grid, block, 0u, s,
                 S, P, oc, of, plane, V, N, Kt, has_above, hf);
  else if (oc)
    launch_timed(h, k_composite_flat<true, false>, grid, block, 0u,
                 s, S, P, oc, of, plane, V, N, Kt, has_above, hf);
  else
    launch_timed(h, k_composite_flat<false, true>, grid, block, 0u,
                 s, S, P, oc, of, plane, V, N, Kt, has_above, hf);
}

// Fixed-point conversion of a coordinate to the 2^-16 voxel lattice:
// rint(((p - o)/h) * 2^16), each step an IEEE fp64 operation.
static bool to_fixed(double p, double o, double h, int64_t *out) {
  double t = p - o;
  t = t / h;
  t = t * 65536.0;
  if (!std::isfinite(t) || std::fabs(t) >= 4611686018427387904.0) return false;
  *out = (int64_t)std::nearbyint(t);
  return true;
}

// Validates the humans of every slice and converts them to the fixed-point
// lattice: words [0, 2 n_slices n_humans) are the centres, then one radius
// per slice.  `w` must hold humans_words() values.
static size_t humans_words(int32_t n_slices, int32_t n_humans) {
  return 2 * (size_t)n_slices * (size_t)n_humans + (size_t)n_slices;
}

static int humans_fixed(Handle *h, const pcsdf_grid *g, int32_t n_slices,
                        int32_t n_humans, const double *human_xy_host,
                        double radius_m, const double *radius_per_slice,
                        double height_m, int64_t *w, int *Kt_out) {
  const double hv = g->voxel_m;
  if (!std::isfinite(height_m) || height_m < 0)
    return fail(h, PCSDF_ERR_NUMERIC, "height_m must be finite, >= 0");
  int64_t Hq;
  if (!to_fixed(height_m, 0.0, hv, &Hq))
    return fail(h, PCSDF_ERR_NUMERIC, "height out of range");
  const size_t ncent = (size_t)n_slices * n_humans;
  // Fixed-point radius of every slice.
  for (int32_t j = 0; j < n_slices; ++j) {
    const double r = radius_per_slice ? radius_per_slice[j] : radius_m;
    if (!std::isfinite(r) || r < 0)
      return fail(h, PCSDF_ERR_NUMERIC, "radius must be finite, >= 0");
    int64_t R;
    if (!to_fixed(r, 0.0, hv, &R))
      return fail(h, PCSDF_ERR_NUMERIC, "radius out of range");
    if (R >= (1LL << 31))
      return fail(h, PCSDF_ERR_NUMERIC, "radius/voxel_m must be < 32768");
    w[2 * ncent + j] = R;
  }
  // Highest layer whose centre lies at or under the cylinder top.
  *Kt_out = Hq >= 32768
                ? (int)std::min<int64_t>((Hq - 32768) / 65536, g->nz - 1)
                : -1;
  // Fixed-point centres, validated on the host before anything is queued.
  for (size_t t = 0; t < ncent; ++t) {
    if (!to_fixed(human_xy_host[2 * t], g->origin_m[0], hv, &w[2 * t]) ||
        !to_fixed(human_xy_host[2 * t + 1], g->origin_m[1], hv,
                  &w[2 * t + 1]))
      return fail(h, PCSDF_ERR_NUMERIC,
                  "human position non-finite or out of range at index " +
                      std::to_string(t));
  }
  return PCSDF_OK;
}

static int check_human_args(Handle *h, int32_t n_slices, int32_t n_humans,
                            const double *human_xy_host) {
  if (n_slices < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (n_humans < 0 || n_humans > kMaxHumans)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_humans must be in [0, 256]");
  if (n_humans > 0 && !human_xy_host)
    return fail(h, PCSDF_ERR_INVALID_ARG, "human_xy_host is required");
  return PCSDF_OK;
}

int humans_upload(Handle *h, const pcsdf_grid *g, int32_t n_slices,
                  int32_t n_humans, const double *human_xy_host,
                  double radius_m, const double *radius_per_slice,
                  double height_m, hipStream_t s, HumanSet *out) {
  int rc = check_human_args(h, n_slices, n_humans, human_xy_host);
  if (rc) return rc;
  const int ny = g->ny;
  const size_t ncent = (size_t)n_slices * n_humans;
  std::vector<int64_t> &xy = h->host_xy;
  xy.resize(humans_words(n_slices, n_humans));
  int Kt;
  if ((rc = humans_fixed(h, g, n_slices, n_humans, human_xy_host, radius_m,
                         radius_per_slice, height_m, xy.data(), &Kt)))
    return rc;
  const bool empty = Kt < 0 || n_humans == 0;
  if ((rc = bind_device(h))) return rc;
  const size_t xy_bytes = xy.size() * sizeof(int64_t);
  const size_t chord_bytes =
      (size_t)n_slices * (n_humans > 0 ? n_humans : 1) * ny * sizeof(int2);
  if ((rc = ensure_buffer(h, h->chord_buf, chord_bytes, s))) return rc;
  if (xy.size() <= (size_t)kCentresInArgs) {
    // small sets travel in the planar kernels' arguments
    out->C.xy = nullptr;
    out->C.Rs = nullptr;
    out->C.rs_off = (int32_t)(2 * ncent);
    std::memcpy(out->C.w, xy.data(), xy_bytes);
  } else {
    if ((rc = ensure_buffer(h, h->param_buf, xy_bytes, s))) return rc;
    int64_t *xy_dev = reinterpret_cast<int64_t *>(h->param_buf.ptr);
    if ((rc = acquire_staging(h, xy_bytes))) return rc;
    std::memcpy(h->pinned, xy.data(), xy_bytes);
    if (hipMemcpyAsync(xy_dev, h->pinned, xy_bytes, hipMemcpyHostToDevice,
                       s) != hipSuccess)
      return fail(h, PCSDF_ERR_HIP, "upload of human positions failed");
    if ((rc = release_staging(h, s))) return rc;
    out->C.xy = xy_dev;
    out->C.Rs = xy_dev + 2 * ncent;
  }
  out->chords = reinterpret_cast<int2 *>(h->chord_buf.ptr);
  out->K = empty ? 0 : n_humans;
  out->Kt = empty ? -1 : Kt;
  out->has_above = out->Kt + 1 <= g->nz - 1;
  return PCSDF_OK;
}

int planes_from(Handle *h, const pcsdf_grid *g, const HumanSet &hs,
                int32_t n_slices, int32_t n_humans, const int32_t *need,
                hipStream_t s, PlaneSet *out) {
  const int nx = g->nx, ny = g->ny;
  const size_t plane_bytes = (size_t)n_slices * nx * ny * sizeof(int32_t);
  int rc;
  if ((rc = ensure_buffer(h, h->plane_buf, 2 * plane_bytes, s))) return rc;
  int32_t *p2 = reinterpret_cast<int32_t *>(h->plane_buf.ptr);
  // Planar signed field of the disk union, per slice.
  ProfScope pp(h, PCSDF_KERNEL_PLANES, s, true);
  if ((rc = launch_planes(h, hs.C, n_humans, hs.K == 0, hs.chords, p2,
                          nx, ny, n_slices, need, s)))
    return rc;
  out->P = p2;
  out->Kt = hs.Kt;
  out->has_above = hs.has_above;
  return PCSDF_OK;
}

int planes_run(Handle *h, const pcsdf_grid *g, int32_t n_slices,
               int32_t n_humans, const double *human_xy_host, double radius_m,
               const double *radius_per_slice, double height_m,
               const int32_t *need, hipStream_t s, PlaneSet *out) {
  HumanSet hs;
  int rc = humans_upload(h, g, n_slices, n_humans, human_xy_host, radius_m,
                         radius_per_slice, height_m, s, &hs);
  if (rc) return rc;
  return planes_from(h, g, hs, n_slices, n_humans, need, s, out);
}

int composite_run(Handle *h, const pcsdf_grid *g,
                  const int32_t *static_ssq_dev, int32_t n_slices,
                  int32_t n_humans, const double *human_xy_host,
                  double radius_m, const double *radius_per_slice,
                  double height_m, int32_t *out_ssq_dev, float *out_sdf_dev,
                  const int32_t *need, hipStream_t s) {
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
  PlaneSet ps_;
  if ((rc = planes_run(h, g, n_slices, n_humans, human_xy_host, radius_m,
                       radius_per_slice, height_m, need, s, &ps_)))
    return rc;
  ProfScope ps(h, PCSDF_KERNEL_COMPOSITE, s, true);
  return launch_composite(h, g, static_ssq_dev, ps_.P, need, ps_.Kt,
                          ps_.has_above, n_slices, out_ssq_dev, out_sdf_dev,
                          s, true);
}

// Whether the per-slice packs read the 16-bit static copy: the tuning's
// choice, else when they read a static field of at least kStatic16Voxels
// voxels for at least kStatic16Groups slice groups (the copy costs 6 B per
// voxel once and saves 2 B per voxel and group; a smaller field is
// re-read from the caches, where the copy was measured to gain nothing:
// 256x256x128 x 20 slices).
constexpr int kStatic16Groups = 4;
constexpr int64_t kStatic16Voxels = 1LL << 25;
static bool use_static16(const Handle *h, int64_t V, int groups) {
  const int t = h->tuning.composite_static16;
  return t == 2 ||
         (t == 0 && V >= kStatic16Voxels && groups >= kStatic16Groups);
}

int launch_composite(Handle *h, const pcsdf_grid *g,
                     const int32_t *static_ssq_dev, const int32_t *P,
                     const int32_t *need, int Kt, int has_above,
                     int32_t n_slices, int32_t *out_ssq_dev,
                     float *out_sdf_dev, hipStream_t s, bool static_copy) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t V = (int64_t)nx * ny * nz;
  // Streaming epilogue over all voxels and slices.
  const float hf = (float)g->voxel_m;
  const PackShape ps = composite_shape((int64_t)nx * ny, V, static_ssq_dev,
                                       out_ssq_dev, out_sdf_dev);
  // Slices per block row: consecutive blocks write the same slices, which
  // keeps the concurrent write streams few and contiguous.
  int G = h->tuning.composite_slices_per_block > 0
              ? h->tuning.composite_slices_per_block
              : 2;
  if (G > n_slices) G = n_slices;
  while ((n_slices + G - 1) / G > 65535) ++G;
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const uint32_t Vu = (uint32_t)V;
  const uintptr_t out_bits =
      (uintptr_t)out_ssq_dev | (uintptr_t)out_sdf_dev;
  const uint64_t N = (uint64_t)n_slices * (uint64_t)V;
  if (V % 2 != 0 && !need && !(out_bits & 15) && N + 4 <= 0xFFFFFFFFull) {
    // aligned packs of the flattened outputs (see k_composite_flat): for
    // odd V they beat one voxel per lane (255x255x127 x 20: 0.39 -> 0.34
    // ms); for V = 2 mod 4 two-voxel packs that read the static field once
    // stay faster.  Larger outputs take the per-slice packs below.
    launch_comp_flat(h, static_ssq_dev, P, out_ssq_dev, out_sdf_dev,
                            plane, Vu, N, Kt, has_above, hf, s);
    return check_launch(h, "composite");
  }
  const int16_t *S16 = nullptr;
  if (static_copy && !need && use_static16(h, V, (n_slices + G - 1) / G)) {
    // the copy lives in the static build's intermediate buffer, which is
    // free between builds
    int rc = ensure_buffer(h, h->tmp_buf, (size_t)V * 2, s);
    if (rc) return rc;
    int16_t *c = reinterpret_cast<int16_t *>(h->tmp_buf.ptr);
    launch_timed(h, k_static16, dim3((unsigned)(((Vu + 3) / 4 + 255) / 256)),
                 dim3(256), 0u, s, static_ssq_dev, c, Vu);
    if ((rc = check_launch(h, "static16"))) return rc;
    S16 = c;
  }
  if (ps.vec == 4 && !ps.gather)
    launch_comp<4, false>(h, static_ssq_dev, P, need, out_ssq_dev, out_sdf_dev,
                          plane, n_slices, G, Kt, has_above, hf, Vu, S16,
                          s);
  else if (ps.vec == 4)
    launch_comp<4, true>(h, static_ssq_dev, P, need, out_ssq_dev, out_sdf_dev,
                         plane, n_slices, G, Kt, has_above, hf, Vu, S16,
                          s);
  else if (ps.vec == 2 && !ps.gather)
    launch_comp<2, false>(h, static_ssq_dev, P, need, out_ssq_dev, out_sdf_dev,
                          plane, n_slices, G, Kt, has_above, hf, Vu, S16,
                          s);
  else if (ps.vec == 2)
    launch_comp<2, true>(h, static_ssq_dev, P, need, out_ssq_dev, out_sdf_dev,
                         plane, n_slices, G, Kt, has_above, hf, Vu, S16,
                          s);
  else
    launch_comp<1, false>(h, static_ssq_dev, P, need, out_ssq_dev, out_sdf_dev,
                          plane, n_slices, G, Kt, has_above, hf, Vu, S16,
                          s);
  return check_launch(h, "composite");
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_predicted_composite_sdf(
    pcsdf_handle *hp, const pcsdf_grid *g, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  return composite_run(h, g, static_ssq_dev, n_slices, n_humans,
                       human_xy_host, radius_m, nullptr, height_m,
                       out_ssq_dev, out_sdf_dev, nullptr,
                       reinterpret_cast<hipStream_t>(stream));
}

extern "C" int pcsdf_predicted_composite_sdf_growing(
    pcsdf_handle *hp, const pcsdf_grid *g, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    const double *radius_per_slice_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!radius_per_slice_m)
    return fail(h, PCSDF_ERR_INVALID_ARG, "radius_per_slice_m is required");
  return composite_run(h, g, static_ssq_dev, n_slices, n_humans,
                       human_xy_host, 0.0, radius_per_slice_m, height_m,
                       out_ssq_dev, out_sdf_dev, nullptr,
                       reinterpret_cast<hipStream_t>(stream));
}

// ---- The composite without allocation -----------------------------------
// One call's planar fields, row passes and chords live in a file-scope
// device array instead of the handle's workspace, for callers that cannot
// allocate device memory (graph capture, serving loops).  Each device the
// library runs on holds its own copy of the array until the process ends;
// every call on a device shares it, so calls that overlap on one device
// race.  Nothing in it needs to start at zero: each call writes every
// chord, row-pass value and plane pixel before it reads them.
namespace pcsdf {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];

// The device address of `scratch` on the handle's (current) device, taken
// once per device: in host code the array's name is not a device address.
static int scratch_address(Handle *h, unsigned char **out) {
  if (h->device < 0 || h->device >= kNoAllocMaxDevices)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "device index beyond the no-allocation entry point's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  void *&p = g_scratch_ptr[h->device];
  if (!p) {
    void *q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !q) {
      (void)hipGetLastError();
      return fail(h, PCSDF_ERR_HIP,
                  std::string("hipGetSymbolAddress(scratch): ") +
                      hipGetErrorString(e));
    }
    p = q;
  }
  *out = static_cast<unsigned char *>(p);
  return PCSDF_OK;
}

}  // namespace pcsdf

extern "C" int pcsdf_predicted_composite_sdf_noalloc(
    pcsdf_handle *hp, const pcsdf_grid *g, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
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
  if ((rc = check_human_args(h, n_slices, n_humans, human_xy_host))) return rc;
  const size_t words = humans_words(n_slices, n_humans);
  if (words > (size_t)kCentresInArgs)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "no-allocation composite: 2*n_slices*n_humans + n_slices = " +
                    std::to_string(words) + " exceeds " +
                    std::to_string(kCentresInArgs));
  const int nx = g->nx, ny = g->ny;
  const size_t plane_bytes = (size_t)n_slices * nx * ny * sizeof(int32_t);
  const size_t chord_off = align_up(2 * plane_bytes, 256);
  const size_t chord_bytes =
      (size_t)n_slices * (n_humans > 0 ? n_humans : 1) * ny * sizeof(int2);
  if (chord_off + chord_bytes > kNoAllocScratchBytes)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "no-allocation composite: needs " +
                    std::to_string(chord_off + chord_bytes) +
                    " bytes of scratch (8*n_slices*nx*ny, then "
                    "8*n_slices*max(n_humans,1)*ny), the maximum is " +
                    std::to_string(kNoAllocScratchBytes));
  Centres C;
  C.xy = nullptr;
  C.Rs = nullptr;
  C.rs_off = (int32_t)(2 * (size_t)n_slices * n_humans);
  int Kt;
  if ((rc = humans_fixed(h, g, n_slices, n_humans, human_xy_host, radius_m,
                         nullptr, height_m, C.w, &Kt)))
    return rc;
  if ((rc = bind_device(h))) return rc;
  unsigned char *base;
  if ((rc = scratch_address(h, &base))) return rc;
  const bool empty = Kt < 0 || n_humans == 0;
  int32_t *P = reinterpret_cast<int32_t *>(base);
  int2 *chords = reinterpret_cast<int2 *>(base + chord_off);
  if ((rc = launch_planes(h, C, n_humans, empty, chords, P, nx, ny, n_slices,
                          nullptr, s)))
    return rc;
  const int Kt_eff = empty ? -1 : Kt;
  return launch_composite(h, g, static_ssq_dev, P, nullptr, Kt_eff,
                          Kt_eff + 1 <= g->nz - 1, n_slices, out_ssq_dev,
                          out_sdf_dev, s);
}
