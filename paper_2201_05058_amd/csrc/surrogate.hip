// Surrogate sphere queries with an exact fallback.
//
// The learned network answers a sphere query from the sphere's centre, the
// slice time and the humans' current state (positions and velocities) --
// without building any per-slice field.  It either predicts the composite
// distance itself, or (when the environment's fp32 field is passed) only
// the humans' part, the answer then being the smaller of the network's
// value and the environment field sampled exactly at the centre: the
// environment field is built once per room, not per slice, and a network
// that need not memorise the room is far more accurate.  Where the answer
// cannot be trusted the exact path answers instead: a query falls back when
// the predicted sphere distance d(c) - r is below a safety margin (near an
// obstacle the planner needs exact values), when the value or gradient is
// not finite, or when the centre lies outside the span of voxel centres
// (the network was trained there only; the exact path clamps and flags such
// centres).
//
// One call runs, all on the caller's stream and without host round trips:
//   1. features:  x = [c_x, c_y, c_z, t, state...] per query, t = dt * slice
//                 (slice clamped to the horizon as for exact queries);
//   2. network:   value and input gradient (mlp.hip);
//   3. decide:    surrogate answers are written out; fallback queries are
//                 flagged and their slices marked as needed;
//   4. planes:    the humans' planar fields of the marked slices only;
//   5. exact:     the flagged queries answered exactly from the planes and
//                 the static field (direct.hip), without building a field.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "query_device.h"

namespace pcsdf {

constexpr int kNetIn = PCSDF_MLP_IN;
constexpr int kState = PCSDF_MLP_IN - 4;

struct NetState {
  float v[kState];
};

// x[q][0..21] for queries [0, n): one lane per query, constant indices only.
// The network's 22 features of one query (fp32, no contraction: this
// file is built with -ffp-contract=off): the centre, t, then per human k
// its horizontal offset from the centre to its axis at t, the distance to
// that axis (correctly rounded sqrtf) and its velocity:
//   [c, t, (dx_k, dy_k, rho_k, vx_k, vy_k, 0) for k = 0, 1, 2],
//   dx_k = c_x - (px_k + vx_k t), dy_k = c_y - (py_k + vy_k t),
// from the 18-float state (per human: px, py, 0, vx, vy, 0).  A fixed
// transform of the query and the state: the distance to a human is a
// simple function of its offset, which a small network fits far better
// than the products v t it would otherwise have to learn.
__device__ __forceinline__ void fill_features(float *row, float cx, float cy,
                                              float cz, float t,
                                              const float *st) {
  row[0] = cx;
  row[1] = cy;
  row[2] = cz;
  row[3] = t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float *h = st + 6 * k;
    const float qx = h[0] + h[3] * t;
    const float qy = h[1] + h[4] * t;
    const float dx = cx - qx;
    const float dy = cy - qy;
    float *f = row + 4 + 6 * k;
    f[0] = dx;
    f[1] = dy;
    f[2] = sqrtf(dx * dx + dy * dy);
    f[3] = h[3];
    f[4] = h[4];
    f[5] = 0.f;
  }
}

__global__ __launch_bounds__(256) void k_features(
    const float *__restrict__ centre, const int32_t *__restrict__ slice,
    int n_slices, float dt, NetState st, int n, float *__restrict__ x) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  int s = slice[q];
  s = s < 0 ? 0 : (s > n_slices - 1 ? n_slices - 1 : s);
  fill_features(x + (int64_t)q * kNetIn, centre[3 * q], centre[3 * q + 1],
                centre[3 * q + 2], (float)s * dt, st.v);
}

// Pool variant: query q belongs to human configuration c = slice[q] /
// n_slices (its state is states[c]) and slice slice[q] % n_slices.
__global__ __launch_bounds__(256) void k_features_pool(
    const float *__restrict__ centre, const int32_t *__restrict__ slice,
    int n_slices, int n_configs, float dt, const float *__restrict__ states,
    int n, float *__restrict__ x) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  int g = slice[q];
  const int total = n_slices * n_configs;
  g = g < 0 ? 0 : (g > total - 1 ? total - 1 : g);
  const int c = g / n_slices, s = g - c * n_slices;
  fill_features(x + (int64_t)q * kNetIn, centre[3 * q], centre[3 * q + 1],
                centre[3 * q + 2], (float)s * dt,
                states + (int64_t)c * kState);
}

// dy/dc from the network's feature gradient G (22) through the transform
// above: g_x = G0 + sum_k (G[4+6k] + G[6+6k] dx_k / rho_k), likewise g_y
// with dy_k, g_z = G2; the ratios are 0 on an axis (rho_k = 0).
__device__ __forceinline__ void centre_gradient(const float *x,
                                                const float *G, float *g0,
                                                float *g1, float *g2) {
  float gx = G[0], gy = G[1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int b = 4 + 6 * k;
    // read and divided unconditionally (the result is selected), so that
    // no read waits behind a branch on another
    const float dx = x[b], dy = x[b + 1], rho = x[b + 2];
    const float den = rho > 0.f ? rho : 1.f;
    const float qx = dx / den, qy = dy / den;
    const float ux = rho > 0.f ? qx : 0.f;
    const float uy = rho > 0.f ? qy : 0.f;
    gx = gx + G[b];
    gx = gx + G[b + 2] * ux;
    gy = gy + G[b + 1];
    gy = gy + G[b + 2] * uy;
  }
  *g0 = gx;
  *g1 = gy;
  *g2 = G[2];
}

__global__ void k_clear(int32_t *__restrict__ p, int n) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = 0;
}

struct DecideArgs {
  const float *y, *gx, *x, *centre, *radius;
  const float *static_sdf;  // [V] or null (network answers alone)
  const int32_t *slice;
  int n, n_slices, nx, ny, nz;
  double h, ox, oy, oz, eps;
  float margin;
  float *dist, *grad, *cost;
  uint8_t *status, *used;
  int32_t *need;
};

// Slices a workgroup marks in LDS before marking them in global memory.
constexpr int kNeedBits = 1024;

// Decides every query: writes the network's answers, marks fallback
// queries in `used` and their slices in `need` (through an LDS bitmap, so
// that each workgroup writes each needed slice once; no atomics on global
// memory).
__global__ __launch_bounds__(256) void k_decide(DecideArgs A) {
  __shared__ uint32_t bits[kNeedBits / 32];
  for (int t = threadIdx.x; t < kNeedBits / 32; t += 256) bits[t] = 0u;
  __syncthreads();
  const int q = blockIdx.x * 256 + threadIdx.x;
  bool fb = false;
  if (q < A.n) {
    // Every read that does not depend on another is issued here, before
    // any branch, so that they share one wait.
    const int s = A.slice[q];
    const float c3[3] = {A.centre[3 * q], A.centre[3 * q + 1],
                         A.centre[3 * q + 2]};
    const float yq = A.y[q], rq = A.radius[q];
    float g0, g1, g2;
    centre_gradient(A.x + (int64_t)q * kNetIn, A.gx + (int64_t)q * kNetIn,
                    &g0, &g1, &g2);
    if (s < 0) {  // same answer as the exact path
      const float nan = __builtin_nanf("");
      A.dist[q] = nan;
      A.grad[3 * q] = nan;
      A.grad[3 * q + 1] = nan;
      A.grad[3 * q + 2] = nan;
      if (A.cost) A.cost[q] = nan;
      if (A.status) A.status[q] = (uint8_t)PCSDF_Q_SLICE_NEG;
      if (A.used) A.used[q] = 0;
    } else {
      const int sc = s > A.n_slices - 1 ? A.n_slices - 1 : s;
      const int n3[3] = {A.nx, A.ny, A.nz};
      const double o3[3] = {A.ox, A.oy, A.oz};
      bool inside = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double g = ((double)c3[a] - o3[a]) / A.h - 0.5;
        inside = inside && g >= 0.0 && g <= (double)(n3[a] - 1);
      }
      float v = yq;
      if (A.static_sdf && inside) {
        // the network predicts the humans' part: the answer is the smaller
        // of it and the environment field (exact, sampled as the exact
        // query does; the environment wins ties)
        const Trilinear T = trilinear(A.static_sdf, A.nx, A.ny, A.nz, A.h,
                                      A.ox, A.oy, A.oz, A.centre + 3 * q);
        const float sv = (float)T.D;
        if (sv <= v) {
          v = sv;
          g0 = (float)(T.g[0] / A.h);
          g1 = (float)(T.g[1] / A.h);
          g2 = (float)(T.g[2] / A.h);
        }
      }
      const float ds = v - rq;
      const bool ok = inside && isfinite(ds) && ds >= A.margin &&
                      isfinite(g0) && isfinite(g1) && isfinite(g2);
      if (ok) {
        A.dist[q] = ds;
        A.grad[3 * q] = g0;
        A.grad[3 * q + 1] = g1;
        A.grad[3 * q + 2] = g2;
        if (A.cost) {
          const double hc = A.eps - (double)ds;
          A.cost[q] = (float)(hc > 0.0 ? hc : 0.0);
        }
        if (A.status)
          A.status[q] = (uint8_t)(s != sc ? PCSDF_Q_SLICE_CLAMPED : 0);
      } else {
        fb = true;
        if (sc < kNeedBits)
          atomicOr(&bits[sc >> 5], 1u << (sc & 31));
        else
          A.need[sc] = 1;
      }
      A.used[q] = fb ? 1 : 0;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kNeedBits && t < A.n_slices; t += 256)
    if (bits[t >> 5] & (1u << (t & 31))) A.need[t] = 1;
}

static unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_surrogate_features(pcsdf_handle *hp, int32_t n_queries,
                                        const float *centre_dev,
                                        const int32_t *slice_dev,
                                        int32_t n_slices, double dt_s,
                                        const float *state_host,
                                        float *x_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (n_slices < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (!state_host)
    return fail(h, PCSDF_ERR_INVALID_ARG, "state_host is required");
  if (!std::isfinite(dt_s) || dt_s < 0)
    return fail(h, PCSDF_ERR_NUMERIC, "dt_s must be finite and >= 0");
  NetState st;
  for (int c = 0; c < kState; ++c) {
    if (!std::isfinite(state_host[c]))
      return fail(h, PCSDF_ERR_NUMERIC, "non-finite state entry");
    st.v[c] = state_host[c];
  }
  if (n_queries == 0) return PCSDF_OK;
  if (!centre_dev || !slice_dev || !x_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "centre, slice and x are required");
  if (((uintptr_t)centre_dev | (uintptr_t)slice_dev | (uintptr_t)x_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  int rc;
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_features, dim3(nblocks(n_queries)), dim3(256), 0, s,
                     centre_dev, slice_dev, n_slices, (float)dt_s, st,
                     n_queries, x_dev);
  return check_launch(h, "surrogate features");
}

extern "C" int pcsdf_surrogate_features_pool(
    pcsdf_handle *hp, int32_t n_queries, const float *centre_dev,
    const int32_t *slice_dev, int32_t n_slices, int32_t n_configs,
    double dt_s, const float *states_dev, float *x_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (n_queries < 0 || n_slices < 1 || n_configs < 1 ||
      (int64_t)n_slices * n_configs > INT32_MAX)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "need n_queries >= 0, n_slices >= 1, n_configs >= 1");
  if (!std::isfinite(dt_s) || dt_s < 0)
    return fail(h, PCSDF_ERR_NUMERIC, "dt_s must be finite and >= 0");
  if (n_queries == 0) return PCSDF_OK;
  if (!centre_dev || !slice_dev || !states_dev || !x_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "centre, slice, states and x are required");
  if (((uintptr_t)centre_dev | (uintptr_t)slice_dev | (uintptr_t)states_dev |
       (uintptr_t)x_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  int rc;
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_features_pool, dim3(nblocks(n_queries)), dim3(256), 0,
                     s, centre_dev, slice_dev, n_slices, n_configs,
                     (float)dt_s, states_dev, n_queries, x_dev);
  return check_launch(h, "surrogate features (pool)");
}

extern "C" int pcsdf_query_spheres_surrogate(
    pcsdf_handle *hp, pcsdf_mlp *m, const pcsdf_grid *g,
    const int32_t *static_ssq_dev, const float *static_sdf_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, const float *state_host, double dt_s,
    double fallback_margin_m,
    int32_t n_queries, const float *centre_dev, const float *radius_dev,
    const int32_t *slice_dev, double hinge_eps_m, float *dist_dev,
    float *grad_dev, uint8_t *status_dev, float *cost_dev,
    uint8_t *used_fallback_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!m) return fail(h, PCSDF_ERR_INVALID_ARG, "network is NULL");
  if (mlp_handle(m) != h)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "the network was created on another handle");
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2)
    return fail(h, PCSDF_ERR_DIMS, "queries need at least 2 voxels per axis");
  if (n_slices < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (n_humans < 0 || n_humans > kMaxHumans)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_humans must be in [0, 256]");
  if (n_humans > 0 && !human_xy_host)
    return fail(h, PCSDF_ERR_INVALID_ARG, "human_xy_host is required");
  if (!static_ssq_dev || !state_host)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "static_ssq_dev and state_host are required");
  if (!std::isfinite(fallback_margin_m) || !std::isfinite(hinge_eps_m) ||
      !std::isfinite(dt_s) || dt_s < 0 || !std::isfinite(radius_m) ||
      !std::isfinite(height_m))
    return fail(h, PCSDF_ERR_NUMERIC,
                "margin, hinge, dt, radius and height must be finite");
  for (int c = 0; c < kState; ++c)
    if (!std::isfinite(state_host[c]))
      return fail(h, PCSDF_ERR_NUMERIC, "non-finite state entry");
  if (n_queries == 0) return PCSDF_OK;
  if (!centre_dev || !radius_dev || !slice_dev || !dist_dev || !grad_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "centre, radius, slice, dist and grad are required");
  if (((uintptr_t)centre_dev | (uintptr_t)radius_dev |
       (uintptr_t)slice_dev | (uintptr_t)dist_dev | (uintptr_t)grad_dev |
       (uintptr_t)cost_dev | (uintptr_t)static_ssq_dev |
       (uintptr_t)static_sdf_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  // workspace: x [n][22], gx [n][22], y [n], used [n], need [n_slices]
  const size_t n = (size_t)n_queries;
  const size_t bx = align_up(n * kNetIn * 4, 256);
  const size_t by = align_up(n * 4, 256);
  const size_t bu = align_up(n, 256);
  const size_t bneed = align_up((size_t)n_slices * 4, 256);
  if ((rc = ensure_buffer(h, h->sur_buf, 2 * bx + by + bu + bneed, s)))
    return rc;
  char *base = reinterpret_cast<char *>(h->sur_buf.ptr);
  float *x = reinterpret_cast<float *>(base);
  float *gx = reinterpret_cast<float *>(base + bx);
  float *y = reinterpret_cast<float *>(base + 2 * bx);
  uint8_t *used = used_fallback_dev
                      ? used_fallback_dev
                      : reinterpret_cast<uint8_t *>(base + 2 * bx + by);
  int32_t *need = reinterpret_cast<int32_t *>(base + 2 * bx + by + bu);

  if ((rc = pcsdf_surrogate_features(hp, n_queries, centre_dev, slice_dev,
                                     n_slices, dt_s, state_host, x, stream)))
    return rc;
  if ((rc = pcsdf_mlp_forward(m, n_queries, x, y, gx, stream))) return rc;
  hipLaunchKernelGGL(k_clear, dim3(nblocks(n_slices)), dim3(256), 0, s, need,
                     n_slices);
  DecideArgs A;
  A.y = y;
  A.gx = gx;
  A.x = x;
  A.centre = centre_dev;
  A.radius = radius_dev;
  A.static_sdf = static_sdf_dev;
  A.slice = slice_dev;
  A.n = n_queries;
  A.n_slices = n_slices;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.h = g->voxel_m;
  A.ox = g->origin_m[0];
  A.oy = g->origin_m[1];
  A.oz = g->origin_m[2];
  A.eps = hinge_eps_m;
  A.margin = (float)fallback_margin_m;
  A.dist = dist_dev;
  A.grad = grad_dev;
  A.cost = cost_dev;
  A.status = status_dev;
  A.used = used;
  A.need = need;
  {
    ProfScope ps(h, PCSDF_KERNEL_SURROGATE_DECIDE, s);
    hipLaunchKernelGGL(k_decide, dim3(nblocks(n_queries)), dim3(256), 0, s, A);
    if ((rc = check_launch(h, "surrogate decide"))) return rc;
  }
  // The exact answers of the fallback queries, from the planes of the
  // slices they read and the static field.
  DirectSet d;
  if ((rc = direct_setup(h, g, static_ssq_dev, n_slices, n_humans,
                         human_xy_host, radius_m, height_m, need, s, &d)))
    return rc;
  ProfScope pq(h, PCSDF_KERNEL_QUERY, s, true);
  return launch_direct(h, g, d, n_slices, n_queries, used, centre_dev,
                       radius_dev, slice_dev, hinge_eps_m, dist_dev, grad_dev,
                       status_dev, cost_dev, s);
}
