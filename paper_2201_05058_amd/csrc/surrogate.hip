// Surrogate sphere queries with an exact fallback: one small network per
// human.
//
// The composite is the min of the environment field and the humans' field
// (mapping section), and outside the humans the field of their union is
// the min of the single humans' fields: E_D = min_k E_{D_k} per pixel, and
// the 3-D value adds the same layer term for every human.  So the learned
// part is one network evaluated per (query, human): it predicts the exact
// single-human field at the query as d, the distance to the continuous
// cylinder (closed form), plus a learned residual that carries the voxel
// pattern (in [0, 1) voxel for the exact field, clamped to [-1/2, 3/2]).
// The answer is the min over the environment field, sampled exactly from
// the static fp32 field, and the humans' predictions.  No per-slice field
// is built.  A query falls back to the exact path when the network's
// answer cannot be trusted:
//   - its predicted sphere distance is below the margin (near an obstacle
//     the planner needs exact values), or a value or gradient is not
//     finite, or its centre lies outside the span of voxel centres;
//   - the two smallest candidates are within `band` of each other: the
//     exact query interpolates the min of the candidates at the cell's
//     corners, which differs from the min of interpolated candidates only
//     where the order changes inside the cell (at most 2 sqrt(3) voxels of
//     difference at the query, the fields being 1-Lipschitz per voxel);
//   - a human whose voxelised disk may reach beyond the grid (the network
//     is trained on whole disks; the clipped disk is farther) comes within
//     `band` of the winner.
//
// One call, all on the caller's stream and without host round trips:
//   1. prep:    per query the environment value, the humans that can still
//               matter (bounds from the residual's clamp prune the rest
//               exactly), their count and a prefix sum over the workgroup;
//   2. scan:    the workgroups' totals (one workgroup);
//   3. rows:    the 16 features of every (query, relevant human) row;
//   4. network: value and input gradient of every row (mlp.hip), the row
//               count read on the device;
//   5. decide:  the min, the rules above, answers written out; fallback
//               queries flagged and their slices marked as needed;
//   6. planes:  the humans' planar fields of the marked slices only;
//   7. exact:   the flagged queries answered exactly from the planes and
//               the static field (direct.hip), without building a field.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "query_device.h"

namespace pcsdf {

constexpr int kSurIn = PCSDF_SURROGATE_IN;  // features per row
constexpr double kResLo = -0.5, kResHi = 1.5;  // residual clamp (voxels)
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Geometry of one human seen from one query, in voxel units (fp64).
struct HumanGeo {
  double ux, uy, rho, a, w, d;
  double phx, phy;  // the axis' phase on the voxel lattice, [0, 1)
  bool present, clipped;
};

__device__ __forceinline__ HumanGeo human_geo(const Centres &C, int K, int s,
                                              int k, double gx, double gy,
                                              double gz, int Kt, int nx,
                                              int ny) {
  HumanGeo G;
  const int64_t X = centre_word(C, 2 * ((int64_t)s * K + k));
  const int64_t Y = centre_word(C, 2 * ((int64_t)s * K + k) + 1);
  const double Rv = (double)radius_of(C, s) / 65536.0;
  const double cx = (double)X / 65536.0 - 0.5;
  const double cy = (double)Y / 65536.0 - 0.5;
  G.present = !(cx + Rv < 0.0 || cx - Rv > (double)(nx - 1) ||
                cy + Rv < 0.0 || cy - Rv > (double)(ny - 1));
  G.clipped = G.present && (cx - Rv <= -1.0 || cx + Rv >= (double)nx ||
                            cy - Rv <= -1.0 || cy + Rv >= (double)ny);
  G.ux = gx - cx;
  G.uy = gy - cy;
  G.rho = sqrt(G.ux * G.ux + G.uy * G.uy);
  G.a = G.rho - Rv;
  G.w = gz - (double)Kt;
  const double ap = G.a > 0.0 ? G.a : 0.0, wp = G.w > 0.0 ? G.w : 0.0;
  G.d = sqrt(ap * ap + wp * wp);
  G.phx = (double)((X - 32768) & 0xFFFF) / 65536.0;
  G.phy = (double)((Y - 32768) & 0xFFFF) / 65536.0;
  return G;
}

// The query's position on the voxel lattice: g = (c - o)/h - 1/2 (fp64).
struct QueryPos {
  double g[3];
  bool inside;  // within the span of voxel centres on every axis
};

__device__ __forceinline__ QueryPos query_pos(const float *c, double h,
                                              double ox, double oy, double oz,
                                              int nx, int ny, int nz) {
  QueryPos P;
  const double o3[3] = {ox, oy, oz};
  const int n3[3] = {nx, ny, nz};
  P.inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.g[a] = ((double)c[a] - o3[a]) / h - 0.5;
    P.inside = P.inside && P.g[a] >= 0.0 && P.g[a] <= (double)(n3[a] - 1);
  }
  return P;
}

// The 16 features of one row (fp64 values rounded to fp32):
//   [ux/rho, uy/rho, a, w, d, 1/(1+d), sin/cos 2pi phx, sin/cos 2pi phy,
//    sin/cos 2pi f_x, sin/cos 2pi f_y, sin/cos 2pi f_z], f = g - floor(g).
__device__ __forceinline__ void row_features(const HumanGeo &G,
                                             const double g[3], float *x) {
  const bool r0 = G.rho > 0.0;
  x[0] = (float)(r0 ? G.ux / G.rho : 0.0);
  x[1] = (float)(r0 ? G.uy / G.rho : 0.0);
  x[2] = (float)G.a;
  x[3] = (float)G.w;
  x[4] = (float)G.d;
  x[5] = (float)(1.0 / (1.0 + G.d));
  x[6] = (float)sinpi(2.0 * G.phx);
  x[7] = (float)cospi(2.0 * G.phx);
  x[8] = (float)sinpi(2.0 * G.phy);
  x[9] = (float)cospi(2.0 * G.phy);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = g[a] - floor(g[a]);
    x[10 + 2 * a] = (float)sinpi(2.0 * f);
    x[11 + 2 * a] = (float)cospi(2.0 * f);
  }
}

// A human's prediction y = fp32(h (d + clamp(delta))) in metres and its
// gradient dy/dc (fp32, metres per metre): the closed-form gradient of d
// plus, when delta is not clamped, the network's feature gradient G
// through the features' closed-form derivatives.
__device__ __forceinline__ float human_value(const HumanGeo &Gm,
                                             const double g[3], float delta,
                                             const float *Gf, double h,
                                             float grad[3]) {
  const double dl = (double)delta;
  const bool clamped = !(dl >= kResLo && dl <= kResHi);
  const double dc = dl < kResLo ? kResLo : (dl > kResHi ? kResHi : dl);
  const double y = h * (Gm.d + (isnan(dl) ? dl : dc));
  const bool r0 = Gm.rho > 0.0;
  const double ex = r0 ? Gm.ux / Gm.rho : 0.0, ey = r0 ? Gm.uy / Gm.rho : 0.0;
  const double ap = Gm.a > 0.0 ? Gm.a : 0.0, wp = Gm.w > 0.0 ? Gm.w : 0.0;
  double dd[3] = {0.0, 0.0, 0.0};
  if (Gm.d > 0.0) {
    dd[0] = ap * ex / Gm.d;
    dd[1] = ap * ey / Gm.d;
    dd[2] = wp / Gm.d;
  }
  double t[3] = {dd[0], dd[1], dd[2]};
  if (!clamped) {
    const double r3 = Gm.rho * Gm.rho * Gm.rho;
    const double q00 = r0 ? Gm.uy * Gm.uy / r3 : 0.0;
    const double q01 = r0 ? -Gm.ux * Gm.uy / r3 : 0.0;
    const double q11 = r0 ? Gm.ux * Gm.ux / r3 : 0.0;
    const double G0 = Gf[0], G1 = Gf[1], G2 = Gf[2], G3 = Gf[3];
    const double G4 = Gf[4], G5 = Gf[5];
    const double s5 = -1.0 / ((1.0 + Gm.d) * (1.0 + Gm.d));
    t[0] += G0 * q00 + G1 * q01 + G2 * ex + (G4 + G5 * s5) * dd[0];
    t[1] += G0 * q01 + G1 * q11 + G2 * ey + (G4 + G5 * s5) * dd[1];
    t[2] += G3 + (G4 + G5 * s5) * dd[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double f = g[a] - floor(g[a]);
      t[a] += kTwoPi * ((double)Gf[10 + 2 * a] * cospi(2.0 * f) -
                        (double)Gf[11 + 2 * a] * sinpi(2.0 * f));
    }
  }
  // y = h (d + delta) and dg/dc = 1/h: the metres cancel
#pragma unroll
  for (int a = 0; a < 3; ++a) grad[a] = (float)t[a];
  return (float)y;
}

// Lower and upper bounds of a human's prediction (the residual's clamp).
__device__ __forceinline__ float human_lo(const HumanGeo &G, double h) {
  return (float)(h * (G.d + kResLo));
}
__device__ __forceinline__ float human_hi(const HumanGeo &G, double h) {
  return (float)(h * (G.d + kResHi));
}

struct SurArgs {
  Centres C;
  const float *centre, *radius, *static_sdf;
  const int32_t *slice;
  int n, n_slices, K, Kt, nx, ny, nz;
  double h, ox, oy, oz, eps, band;
  float margin;
  int64_t cap;  // rows of the workspace
  // per query
  float *env;      // [n][4]: e, de/dc
  int8_t *state;   // 0 pending, 1 fallback, 2 answered (slice < 0)
  int32_t *count;  // relevant humans
  int32_t *loc;    // exclusive prefix within the workgroup
  int32_t *bsum;   // per workgroup: its total, then its exclusive offset
  int32_t *total;  // [1] rows
  // rows
  float *x, *y, *gx;
  // outputs
  float *dist, *grad, *cost;
  uint8_t *status, *used;
  int32_t *need;
};

__device__ __forceinline__ int clamp_slice(int s, int n) {
  return s < 0 ? 0 : (s > n - 1 ? n - 1 : s);
}

// Is human k relevant to a pending query: present and not provably above
// the best upper bound m_hi by more than the band?
__device__ __forceinline__ bool relevant(const HumanGeo &G, float m_hi,
                                         double h, double band) {
  return G.present && !((double)human_lo(G, h) > (double)m_hi + band);
}

__global__ __launch_bounds__(256) void k_sur_prep(SurArgs A) {
  __shared__ int32_t wsum[4];
  const int q = blockIdx.x * 256 + threadIdx.x;
  int cnt = 0;
  if (q < A.n) {
    const int s = A.slice[q];
    const float c3[3] = {A.centre[3 * q], A.centre[3 * q + 1],
                         A.centre[3 * q + 2]};
    const float rq = A.radius[q];
    int8_t st = 0;
    if (s < 0) {  // same answer as the exact path
      const float nan = __builtin_nanf("");
      A.dist[q] = nan;
      A.grad[3 * q] = nan;
      A.grad[3 * q + 1] = nan;
      A.grad[3 * q + 2] = nan;
      if (A.cost) A.cost[q] = nan;
      if (A.status) A.status[q] = (uint8_t)PCSDF_Q_SLICE_NEG;
      st = 2;
    } else {
      const QueryPos P = query_pos(c3, A.h, A.ox, A.oy, A.oz, A.nx, A.ny,
                                   A.nz);
      if (!P.inside) {
        st = 1;
      } else {
        const Trilinear T = trilinear(A.static_sdf, A.nx, A.ny, A.nz, A.h,
                                      A.ox, A.oy, A.oz, c3);
        const float e = (float)T.D;
        A.env[4 * q] = e;
        A.env[4 * q + 1] = (float)(T.g[0] / A.h);
        A.env[4 * q + 2] = (float)(T.g[1] / A.h);
        A.env[4 * q + 3] = (float)(T.g[2] / A.h);
        const int sc = clamp_slice(s, A.n_slices);
        float m_hi = e;
        for (int k = 0; k < A.K; ++k) {
          const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1],
                                       P.g[2], A.Kt, A.nx, A.ny);
          if (G.present) m_hi = fminf(m_hi, human_hi(G, A.h));
        }
        // the answer is at most m_hi: below the margin it falls back
        // whatever the network says
        if (!(m_hi - rq >= A.margin)) {
          st = 1;
        } else {
          for (int k = 0; k < A.K; ++k) {
            const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1],
                                         P.g[2], A.Kt, A.nx, A.ny);
            cnt += relevant(G, m_hi, A.h, A.band) ? 1 : 0;
          }
        }
      }
    }
    A.state[q] = st;
    A.count[q] = cnt;
  }
  // exclusive prefix of cnt over the workgroup
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  if (q < A.n) A.loc[q] = before + incl - cnt;
  if (threadIdx.x == 255)
    A.bsum[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Exclusive scan of the workgroups' totals in place (one workgroup).
__global__ __launch_bounds__(1024) void k_sur_scan(int32_t *bsum, int nb,
                                                   int32_t *total) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < nb) bsum[i] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = carry;
}

__device__ __forceinline__ int64_t row_offset(const SurArgs &A, int q) {
  return (int64_t)A.bsum[q >> 8] + A.loc[q];
}

__global__ __launch_bounds__(256) void k_sur_rows(SurArgs A) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= A.n || A.state[q] != 0 || A.count[q] == 0) return;
  const int64_t off = row_offset(A, q);
  if (off + A.count[q] > A.cap) return;  // the query falls back
  const float c3[3] = {A.centre[3 * q], A.centre[3 * q + 1],
                       A.centre[3 * q + 2]};
  const QueryPos P = query_pos(c3, A.h, A.ox, A.oy, A.oz, A.nx, A.ny, A.nz);
  const int sc = clamp_slice(A.slice[q], A.n_slices);
  const float rq = A.radius[q];
  (void)rq;
  float m_hi = A.env[4 * q];
  for (int k = 0; k < A.K; ++k) {
    const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1], P.g[2],
                                 A.Kt, A.nx, A.ny);
    if (G.present) m_hi = fminf(m_hi, human_hi(G, A.h));
  }
  int64_t r = off;
  for (int k = 0; k < A.K; ++k) {
    const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1], P.g[2],
                                 A.Kt, A.nx, A.ny);
    if (!relevant(G, m_hi, A.h, A.band)) continue;
    row_features(G, P.g, A.x + r * kSurIn);
    ++r;
  }
}

// Slices a workgroup marks in LDS before marking them in global memory.
constexpr int kNeedBits = 1024;

__global__ __launch_bounds__(256) void k_sur_decide(SurArgs A) {
  __shared__ uint32_t bits[kNeedBits / 32];
  for (int t = threadIdx.x; t < kNeedBits / 32; t += 256) bits[t] = 0u;
  __syncthreads();
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < A.n && A.state[q] != 2) {
    const int s = A.slice[q];
    const int sc = clamp_slice(s, A.n_slices);
    bool fb = A.state[q] == 1;
    if (!fb) {
      const float c3[3] = {A.centre[3 * q], A.centre[3 * q + 1],
                           A.centre[3 * q + 2]};
      const QueryPos P = query_pos(c3, A.h, A.ox, A.oy, A.oz, A.nx, A.ny,
                                   A.nz);
      const float rq = A.radius[q];
      const int cnt = A.count[q];
      const int64_t off = row_offset(A, q);
      fb = cnt > 0 && off + cnt > A.cap;
      float y = A.env[4 * q];
      float g[3] = {A.env[4 * q + 1], A.env[4 * q + 2], A.env[4 * q + 3]};
      float m2 = __builtin_inff(), cmin = __builtin_inff();
      if (!fb && cnt > 0) {
        float m_hi = y;
        for (int k = 0; k < A.K; ++k) {
          const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1],
                                       P.g[2], A.Kt, A.nx, A.ny);
          if (G.present) m_hi = fminf(m_hi, human_hi(G, A.h));
        }
        int64_t r = off;
        for (int k = 0; k < A.K; ++k) {
          const HumanGeo G = human_geo(A.C, A.K, sc, k, P.g[0], P.g[1],
                                       P.g[2], A.Kt, A.nx, A.ny);
          if (!relevant(G, m_hi, A.h, A.band)) continue;
          float gk[3];
          const float yk = human_value(G, P.g, A.y[r], A.gx + r * kSurIn,
                                       A.h, gk);
          ++r;
          if (G.clipped) cmin = fminf(cmin, yk);
          if (yk < y) {
            m2 = y;
            y = yk;
            g[0] = gk[0];
            g[1] = gk[1];
            g[2] = gk[2];
          } else if (yk < m2) {
            m2 = yk;
          }
        }
      }
      const float ds = y - rq;
      const bool ok = !fb && isfinite(ds) && ds >= A.margin &&
                      isfinite(g[0]) && isfinite(g[1]) && isfinite(g[2]) &&
                      !((double)m2 - (double)y < A.band) &&
                      !((double)cmin <= (double)y + A.band);
      if (ok) {
        A.dist[q] = ds;
        A.grad[3 * q] = g[0];
        A.grad[3 * q + 1] = g[1];
        A.grad[3 * q + 2] = g[2];
        if (A.cost) {
          const double hc = A.eps - (double)ds;
          A.cost[q] = (float)(hc > 0.0 ? hc : 0.0);
        }
        if (A.status)
          A.status[q] = (uint8_t)(s != sc ? PCSDF_Q_SLICE_CLAMPED : 0);
      }
      fb = !ok;
    }
    if (fb) {
      if (sc < kNeedBits)
        atomicOr(&bits[sc >> 5], 1u << (sc & 31));
      else
        A.need[sc] = 1;
    }
    A.used[q] = fb ? 1 : 0;
  } else if (q < A.n) {
    A.used[q] = 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kNeedBits && t < A.n_slices; t += 256)
    if (bits[t >> 5] & (1u << (t & 31))) A.need[t] = 1;
}

// The rows the network evaluated: min(total, cap).
__global__ void k_rows_out(const int32_t *__restrict__ total, int64_t cap,
                           int32_t *__restrict__ out) {
  if (threadIdx.x == 0)
    out[0] = (int32_t)((int64_t)total[0] < cap ? (int64_t)total[0] : cap);
}

__global__ void k_clear(int32_t *__restrict__ p, int n) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = 0;
}

// Training features: query q's row for human hidx[q] (0 when null) of its
// slice, the base distance d (voxels) and, with labels (metres), the
// residual target label/h - d.
__global__ __launch_bounds__(256) void k_sur_features(
    Centres C, int K, int Kt, int n_slices, int nx, int ny, int nz, double h,
    double ox, double oy, double oz, int n, const float *__restrict__ centre,
    const int32_t *__restrict__ slice, const int32_t *__restrict__ hidx,
    const float *__restrict__ label, float *__restrict__ x,
    float *__restrict__ base, float *__restrict__ target) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const float c3[3] = {centre[3 * q], centre[3 * q + 1], centre[3 * q + 2]};
  const QueryPos P = query_pos(c3, h, ox, oy, oz, nx, ny, nz);
  const int sc = clamp_slice(slice[q], n_slices);
  int k = hidx ? hidx[q] : 0;
  k = k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
  const HumanGeo G = human_geo(C, K, sc, k, P.g[0], P.g[1], P.g[2], Kt, nx,
                               ny);
  row_features(G, P.g, x + (int64_t)q * kSurIn);
  if (base) base[q] = (float)G.d;
  if (target && label) target[q] = (float)((double)label[q] / h - G.d);
}

static unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_surrogate_human_features(
    pcsdf_handle *hp, const pcsdf_grid *g, int32_t n_slices, int32_t n_humans,
    const double *human_xy_host, double radius_m, double height_m,
    int32_t n_queries, const float *centre_dev, const int32_t *slice_dev,
    const int32_t *human_dev, const float *label_dev, float *x_dev,
    float *base_dev, float *target_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (n_humans < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_humans must be >= 1");
  if (target_dev && !label_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "a target needs labels");
  if (n_queries > 0 && (!centre_dev || !slice_dev || !x_dev))
    return fail(h, PCSDF_ERR_INVALID_ARG, "centre, slice and x are required");
  if (((uintptr_t)centre_dev | (uintptr_t)slice_dev | (uintptr_t)human_dev |
       (uintptr_t)label_dev | (uintptr_t)x_dev | (uintptr_t)base_dev |
       (uintptr_t)target_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  if (n_queries == 0) return PCSDF_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HumanSet hs;
  if ((rc = humans_upload(h, g, n_slices, n_humans, human_xy_host, radius_m,
                          nullptr, height_m, s, &hs)))
    return rc;
  hipLaunchKernelGGL(k_sur_features, dim3(nblocks(n_queries)), dim3(256), 0,
                     s, hs.C, n_humans, hs.Kt, n_slices, g->nx, g->ny, g->nz,
                     g->voxel_m, g->origin_m[0], g->origin_m[1],
                     g->origin_m[2], n_queries, centre_dev, slice_dev,
                     human_dev, label_dev, x_dev, base_dev, target_dev);
  return check_launch(h, "surrogate features");
}

extern "C" int pcsdf_query_spheres_surrogate(
    pcsdf_handle *hp, pcsdf_mlp *m, const pcsdf_grid *g,
    const int32_t *static_ssq_dev, const float *static_sdf_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, double fallback_margin_m,
    double band_m, int32_t n_queries, const float *centre_dev,
    const float *radius_dev, const int32_t *slice_dev, double hinge_eps_m,
    float *dist_dev, float *grad_dev, uint8_t *status_dev, float *cost_dev,
    uint8_t *used_fallback_dev, int32_t *rows_dev, void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!m) return fail(h, PCSDF_ERR_INVALID_ARG, "network is NULL");
  if (mlp_handle(m) != h)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "the network was created on another handle");
  if (mlp_inputs(m) != kSurIn)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "the network must take " + std::to_string(kSurIn) +
                    " inputs");
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2)
    return fail(h, PCSDF_ERR_DIMS, "queries need at least 2 voxels per axis");
  if (n_queries < 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_queries must be >= 0");
  if (!static_ssq_dev || !static_sdf_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "static_ssq_dev and static_sdf_dev are required");
  if (!std::isfinite(fallback_margin_m) || !std::isfinite(hinge_eps_m) ||
      !std::isfinite(band_m) || band_m < 0)
    return fail(h, PCSDF_ERR_NUMERIC,
                "margin and hinge must be finite, band finite and >= 0");
  if (n_queries > 0 && (!centre_dev || !radius_dev || !slice_dev ||
                        !dist_dev || !grad_dev))
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "centre, radius, slice, dist and grad are required");
  if (((uintptr_t)centre_dev | (uintptr_t)radius_dev |
       (uintptr_t)slice_dev | (uintptr_t)dist_dev | (uintptr_t)grad_dev |
       (uintptr_t)cost_dev | (uintptr_t)static_ssq_dev |
       (uintptr_t)static_sdf_dev | (uintptr_t)rows_dev) & 3)
    return fail(h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n_queries == 0) {
    if (rows_dev) {
      if ((rc = bind_device(h))) return rc;
      hipLaunchKernelGGL(k_clear, dim3(1), dim3(256), 0, s, rows_dev, 1);
      return check_launch(h, "surrogate rows");
    }
    return PCSDF_OK;
  }
  HumanSet hs;
  if ((rc = humans_upload(h, g, n_slices, n_humans, human_xy_host, radius_m,
                          nullptr, height_m, s, &hs)))
    return rc;

  // workspace: per query env [4], state, count, loc, used; per workgroup
  // bsum; total; need [n_slices]; rows x [cap][16], y [cap], gx [cap][16]
  const int64_t n = n_queries;
  const int nb = (int)nblocks(n);
  const int64_t K = hs.K;
  int64_t cap = n * K;
  const int64_t cap_max = std::max<int64_t>(4 * n, 1 << 20);
  if (cap > cap_max) cap = cap_max;
  const size_t b_env = align_up((size_t)n * 16, 256);
  const size_t b_q4 = align_up((size_t)n * 4, 256);
  const size_t b_q1 = align_up((size_t)n, 256);
  const size_t b_bs = align_up((size_t)nb * 4 + 256, 256);
  const size_t b_need = align_up((size_t)n_slices * 4, 256);
  const size_t b_x = align_up((size_t)cap * kSurIn * 4 + 4, 256);
  const size_t b_y = align_up((size_t)cap * 4 + 4, 256);
  const size_t bytes = b_env + 2 * b_q4 + 2 * b_q1 + b_bs + b_need + 2 * b_x +
                       b_y;
  if ((rc = ensure_buffer(h, h->sur_buf, bytes, s))) return rc;
  char *p = reinterpret_cast<char *>(h->sur_buf.ptr);
  SurArgs A;
  A.env = reinterpret_cast<float *>(p);
  p += b_env;
  A.count = reinterpret_cast<int32_t *>(p);
  p += b_q4;
  A.loc = reinterpret_cast<int32_t *>(p);
  p += b_q4;
  A.state = reinterpret_cast<int8_t *>(p);
  p += b_q1;
  uint8_t *used_ws = reinterpret_cast<uint8_t *>(p);
  p += b_q1;
  A.bsum = reinterpret_cast<int32_t *>(p);
  A.total = A.bsum + nb;
  p += b_bs;
  A.need = reinterpret_cast<int32_t *>(p);
  p += b_need;
  A.x = reinterpret_cast<float *>(p);
  p += b_x;
  A.gx = reinterpret_cast<float *>(p);
  p += b_x;
  A.y = reinterpret_cast<float *>(p);
  A.C = hs.C;
  A.centre = centre_dev;
  A.radius = radius_dev;
  A.static_sdf = static_sdf_dev;
  A.slice = slice_dev;
  A.n = n_queries;
  A.n_slices = n_slices;
  A.K = hs.K;
  A.Kt = hs.Kt;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.h = g->voxel_m;
  A.ox = g->origin_m[0];
  A.oy = g->origin_m[1];
  A.oz = g->origin_m[2];
  A.eps = hinge_eps_m;
  A.band = band_m;
  A.margin = (float)fallback_margin_m;
  A.cap = cap;
  A.dist = dist_dev;
  A.grad = grad_dev;
  A.cost = cost_dev;
  A.status = status_dev;
  A.used = used_fallback_dev ? used_fallback_dev : used_ws;
  {
    ProfScope ps(h, PCSDF_KERNEL_SURROGATE_DECIDE, s);
    hipLaunchKernelGGL(k_clear, dim3(nblocks(n_slices)), dim3(256), 0, s,
                       A.need, n_slices);
    hipLaunchKernelGGL(k_sur_prep, dim3(nb), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_sur_scan, dim3(1), dim3(1024), 0, s, A.bsum, nb,
                       A.total);
    hipLaunchKernelGGL(k_sur_rows, dim3(nb), dim3(256), 0, s, A);
    if ((rc = check_launch(h, "surrogate rows"))) return rc;
  }
  if (cap > 0) {
    ProfScope ps(h, PCSDF_KERNEL_MLP, s);
    if ((rc = mlp_rows(m, (int)cap, A.total, A.x, A.y, A.gx, s))) return rc;
  }
  {
    ProfScope ps(h, PCSDF_KERNEL_SURROGATE_DECIDE, s);
    hipLaunchKernelGGL(k_sur_decide, dim3(nb), dim3(256), 0, s, A);
    if ((rc = check_launch(h, "surrogate decide"))) return rc;
  }
  if (rows_dev)
    hipLaunchKernelGGL(k_rows_out, dim3(1), dim3(64), 0, s, A.total, cap,
                       rows_dev);
  // The exact answers of the fallback queries, from the planes of the
  // slices they read and the static field.
  DirectSet d;
  if ((rc = direct_from(h, g, static_ssq_dev, hs, n_slices, n_humans,
                        A.need, s, &d)))
    return rc;
  ProfScope pq(h, PCSDF_KERNEL_QUERY, s, true);
  return launch_direct(h, g, d, n_slices, n_queries, A.used, centre_dev,
                       radius_dev, slice_dev, hinge_eps_m, dist_dev, grad_dev,
                       status_dev, cost_dev, s);
}
