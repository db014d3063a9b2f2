/*
 * CPU oracle for predicted composite signed distance fields.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow C that restates
 * what the method computes so that the GPU library can be checked against
 * it.  Only the test suite, the smoke check and the CPU baseline leg of the
 * benchmark load it; the GPU library never does, and the two share no
 * code, header or table.  Built plainly it is single-threaded; built with
 * -fopenmp (a separate library, for the CPU baseline's all-core timing) the
 * independent lines of each pass and the voxel loops run on all threads,
 * computing the same values in the same order per element.
 *
 * What is computed (Finean et al. 2022, section "Mapping - Predicted
 * Composite Distance Fields", and the RHAP-GPMP2 section):
 *   - an environment distance field, computed once for the static map;
 *   - a distance field of the humans, modelled as vertical cylinders, at
 *     their predicted positions for each future time slice;
 *   - the composite of the two by an elementwise min, one field per slice;
 *   - sampling of a slice's field (distance and gradient) at collision
 *     spheres, as consumed by GPMP2's hinge-loss obstacle factors, with
 *     time indices past the last slice using the last slice.
 * Fields are signed (the preliminary work this section builds on is titled
 * "predicted composite signed-distance fields").
 *
 * Conventions (the paper is silent on them; these are the readings used):
 *   grid x fastest, idx = (k*ny + j)*nx + i; voxel centres at
 *   origin + h*(i+1/2, j+1/2, k+1/2); voxels outside the grid do not exist.
 *   E_S(v) = min over u in S of |v-u|^2 in voxel units, INF if S is empty.
 *   SSQ_S(v) = E_S(v) for v not in S, -E_{G\S}(v) for v in S; INF is
 *   INT32_MAX and -INF is -INT32_MAX.
 *   F(x) = sign(x) * ((float)h * sqrtf((float)|x|)), F(+-INF) = +-inf.
 *
 * Each function below cites the passage or definition it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF32 INT32_MAX
#define OR_INF64 INT64_MAX
#define OR_Q 65536.0

/* ---------------------------------------------------------------------
 * Exact squared EDT.
 *
 * Definition: E_S(v) = min_{u in S} |v - u|^2.  Because |v-u|^2 is a sum
 * of one term per axis, the minimum can be taken one axis at a time:
 *   g_x(v) = min_{i'} f0(i', j, k) + (i - i')^2,  f0 = 0 on S, INF off S,
 *   g_y(v) = min_{j'} g_x(i, j', k) + (j - j')^2,
 *   E_S(v) = min_{k'} g_y(i, j, k') + (k - k')^2.
 * Each 1-D minimum is the lower envelope of parabolas of Felzenszwalb and
 * Huttenlocher ("Distance transforms of sampled functions", 2012), written
 * here in their notation: v[] holds the sites of the envelope, z[] the
 * boundaries between consecutive parabolas.  Sites whose value is INF are
 * not parabolas and are skipped.  Intersections are computed in double; the
 * integer numerators are exact in double and two distinct intersections of
 * this problem differ by at least 1/(2048^2), far above rounding, so the
 * comparisons are exact.
 * ------------------------------------------------------------------- */
static void or_envelope(const int64_t *f, int n, int64_t *d, int *v,
                        double *z) {
  int k = -1;
  for (int q = 0; q < n; q++) {
    if (f[q] == OR_INF64) continue;
    if (k < 0) {
      k = 0;
      v[0] = q;
      z[0] = -HUGE_VAL;
      z[1] = HUGE_VAL;
      continue;
    }
    double s;
    for (;;) {
      int p = v[k];
      double num = (double)(f[q] + (int64_t)q * q) -
                   (double)(f[p] + (int64_t)p * p);
      s = num / (2.0 * (double)(q - p));
      if (s <= z[k]) {
        k--; /* z[0] = -inf stops this at k = 0 */
        continue;
      }
      break;
    }
    k++;
    v[k] = q;
    z[k] = s;
    z[k + 1] = HUGE_VAL;
  }
  if (k < 0) {
    for (int q = 0; q < n; q++) d[q] = OR_INF64;
    return;
  }
  int j = 0;
  for (int q = 0; q < n; q++) {
    while (z[j + 1] < (double)q) j++;
    int64_t dq = (int64_t)(q - v[j]);
    d[q] = dq * dq + f[v[j]];
  }
}

/* One 1-D pass along `axis` (0 = x, 1 = y, 2 = z) of a full grid.  The
 * lines are independent; each thread has its own envelope buffers.
 * Returns -1 if they cannot be allocated. */
static int or_pass(int64_t *a, int nx, int ny, int nz, int axis) {
  int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
  int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx : (int64_t)nx * ny);
  int n1 = axis == 0 ? ny : nx;
  int n2 = axis == 2 ? ny : nz;
  int failed = 0;
#pragma omp parallel
  {
    int64_t *fbuf = malloc(sizeof(int64_t) * n);
    int64_t *dbuf = malloc(sizeof(int64_t) * n);
    int *vbuf = malloc(sizeof(int) * n);
    double *zbuf = malloc(sizeof(double) * (n + 1));
    int ok = fbuf && dbuf && vbuf && zbuf;
    if (!ok) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for collapse(2) schedule(static)
    for (int b = 0; b < n2; b++) {
      for (int c = 0; c < n1; c++) {
        if (!ok) continue;
        int64_t base;
        if (axis == 0) base = ((int64_t)b * ny + c) * nx;
        else if (axis == 1) base = (int64_t)b * nx * ny + c;
        else base = (int64_t)b * nx + c;
        for (int q = 0; q < n; q++) fbuf[q] = a[base + q * stride];
        or_envelope(fbuf, n, dbuf, vbuf, zbuf);
        for (int q = 0; q < n; q++) a[base + q * stride] = dbuf[q];
      }
    }
    free(fbuf); free(dbuf); free(vbuf); free(zbuf);
  }
  return failed ? -1 : 0;
}

/* E_S for the set of voxels where set[v] != 0 (want = 1) or == 0
 * (want = 0).  out: int64 [V], OR_INF64 where S is empty. */
static int or_edt_sq_sel(const uint8_t *set, int want, int nx, int ny,
                         int nz, int64_t *out) {
  int64_t V = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < V; i++)
    out[i] = ((set[i] != 0) == (want != 0)) ? 0 : OR_INF64;
  for (int axis = 0; axis < 3; axis++)
    if (or_pass(out, nx, ny, nz, axis)) return -1;
  return 0;
}

int or_edt_sq(const uint8_t *set, int nx, int ny, int nz, int64_t *out) {
  return or_edt_sq_sel(set, 1, nx, ny, nz, out);
}

/* Pass order variant used by the order-invariance check: axes applied in
 * the order given by `order` (a permutation of 0,1,2). */
int or_edt_sq_order(const uint8_t *set, int nx, int ny, int nz,
                    const int *order, int64_t *out) {
  int64_t V = (int64_t)nx * ny * nz;
  for (int64_t i = 0; i < V; i++) out[i] = set[i] ? 0 : OR_INF64;
  for (int p = 0; p < 3; p++)
    if (or_pass(out, nx, ny, nz, order[p])) return -1;
  return 0;
}

/* 1-D lower envelope exposed for direct checks against a brute-force min. */
int or_envelope_1d(const int64_t *f, int n, int64_t *out) {
  int *v = malloc(sizeof(int) * (n > 0 ? n : 1));
  double *z = malloc(sizeof(double) * (n + 1));
  if (!v || !z) { free(v); free(z); return -1; }
  or_envelope(f, n, out, v, z);
  free(v); free(z);
  return 0;
}

/* ---------------------------------------------------------------------
 * Signed-squared field of a set: E_S outside S, -E_{G\S} inside S.
 * ------------------------------------------------------------------- */
int or_signed_sq(const uint8_t *set, int nx, int ny, int nz, int32_t *out) {
  int64_t V = (int64_t)nx * ny * nz;
  int64_t *eo = malloc(sizeof(int64_t) * V);
  int64_t *ef = malloc(sizeof(int64_t) * V);
  if (!eo || !ef) { free(eo); free(ef); return -1; }
  if (or_edt_sq_sel(set, 1, nx, ny, nz, eo) ||
      or_edt_sq_sel(set, 0, nx, ny, nz, ef)) {
    free(eo); free(ef);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < V; i++) {
    if (set[i]) {
      out[i] = ef[i] == OR_INF64 ? -OR_INF32 : -(int32_t)ef[i];
    } else {
      out[i] = eo[i] == OR_INF64 ? OR_INF32 : (int32_t)eo[i];
    }
  }
  free(eo); free(ef);
  return 0;
}

/* ---------------------------------------------------------------------
 * F: signed squared voxel distance -> signed metres, fp32.
 * The square root is taken first, then one fp32 multiply by (float)h.
 * ------------------------------------------------------------------- */
float or_F(int32_t x, double h) {
  if (x == OR_INF32) return HUGE_VALF;
  if (x == -OR_INF32) return -HUGE_VALF;
  float hf = (float)h;
  if (x >= 0) return hf * sqrtf((float)x);
  return -(hf * sqrtf((float)(-(int64_t)x)));
}

void or_to_float(const int32_t *x, int64_t n, double h, float *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) out[i] = or_F(x[i], h);
}

/* Threads the loops above may use (1 unless built with OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int or_threads(void) { return omp_get_max_threads(); }
#else
int or_threads(void) { return 1; }
#endif

/* ---------------------------------------------------------------------
 * Voxelised vertical cylinders (the human primitive of the mapping
 * section), evaluated exactly in integers on a 2^-16 voxel lattice:
 *   X = rint(((p_x - o_x)/h) * 2^16), Y likewise, R = rint((r/h) * 2^16),
 *   Hq = rint((H/h) * 2^16);
 *   voxel (i,j,k) is in cylinder c iff
 *     (2^15*(2i+1) - X)^2 + (2^15*(2j+1) - Y)^2 <= R^2   and
 *     2^15*(2k+1) <= Hq          (base of the cylinder at z = o_z).
 * The squares are evaluated in 128-bit integers, literally.
 * Returns -1 for non-finite or out-of-range inputs.
 * ------------------------------------------------------------------- */
static int or_fixed(double p, double o, double h, int64_t *out) {
  double t = p - o;
  t = t / h;
  t = t * OR_Q;
  if (!isfinite(t) || fabs(t) >= 4611686018427387904.0 /* 2^62 */)
    return -1;
  *out = (int64_t)rint(t);
  return 0;
}

int or_human_occupancy(int nx, int ny, int nz, double h, double ox,
                       double oy, double oz, int n_humans,
                       const double *xy, double radius, double height,
                       uint8_t *out) {
  (void)oz;
  int64_t R, Hq;
  if (or_fixed(radius, 0.0, h, &R) || or_fixed(height, 0.0, h, &Hq))
    return -1;
  int64_t *X = malloc(sizeof(int64_t) * (n_humans > 0 ? n_humans : 1));
  int64_t *Y = malloc(sizeof(int64_t) * (n_humans > 0 ? n_humans : 1));
  if (!X || !Y) { free(X); free(Y); return -1; }
  for (int c = 0; c < n_humans; c++) {
    if (or_fixed(xy[2 * c], ox, h, &X[c]) ||
        or_fixed(xy[2 * c + 1], oy, h, &Y[c])) {
      free(X); free(Y);
      return -1;
    }
  }
  const int64_t half = 32768;
  __int128 R2 = (__int128)R * R;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++) {
    int zin = half * (2 * (int64_t)k + 1) <= Hq;
    for (int j = 0; j < ny; j++) {
      for (int i = 0; i < nx; i++) {
        int in = 0;
        if (zin) {
          for (int c = 0; c < n_humans && !in; c++) {
            __int128 dx = (__int128)(half * (2 * (int64_t)i + 1)) - X[c];
            __int128 dy = (__int128)(half * (2 * (int64_t)j + 1)) - Y[c];
            if (dx * dx + dy * dy <= R2) in = 1;
          }
        }
        out[((int64_t)k * ny + j) * nx + i] = (uint8_t)in;
      }
    }
  }
  free(X); free(Y);
  return 0;
}

/* ---------------------------------------------------------------------
 * Composite: elementwise min of the environment field and the humans'
 * field (the "parallel min" of the mapping section), on signed-squared
 * int32 values.
 * ------------------------------------------------------------------- */
void or_composite(const int32_t *a, const int32_t *b, int64_t n,
                  int32_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) out[i] = a[i] < b[i] ? a[i] : b[i];
}

/* Static field: SSQ of the caller's occupancy, and optionally F of it. */
int or_build_static(const uint8_t *occ, int nx, int ny, int nz, double h,
                    int32_t *ssq, float *sdf) {
  if (or_signed_sq(occ, nx, ny, nz, ssq)) return -1;
  if (sdf) or_to_float(ssq, (int64_t)nx * ny * nz, h, sdf);
  return 0;
}

/* The full per-slice composite: for each slice j, voxelise the humans at
 * their predicted positions, take the signed-squared field of that set
 * with two full-grid EDTs, min it with the static field, convert.
 * xy: [n_slices][n_humans][2].  Outputs [n_slices][V] (either may be NULL).
 */
int or_predicted_composite(const int32_t *static_ssq, int nx, int ny, int nz,
                           double h, double ox, double oy, double oz,
                           int n_slices, int n_humans, const double *xy,
                           double radius, double height, int32_t *out_ssq,
                           float *out_sdf) {
  int64_t V = (int64_t)nx * ny * nz;
  uint8_t *hocc = malloc(V);
  int32_t *hssq = malloc(sizeof(int32_t) * V);
  int32_t *c = malloc(sizeof(int32_t) * V);
  if (!hocc || !hssq || !c) { free(hocc); free(hssq); free(c); return -1; }
  int rc = 0;
  for (int s = 0; s < n_slices && !rc; s++) {
    rc = or_human_occupancy(nx, ny, nz, h, ox, oy, oz, n_humans,
                            xy + (int64_t)s * n_humans * 2, radius, height,
                            hocc);
    if (rc) break;
    rc = or_signed_sq(hocc, nx, ny, nz, hssq);
    if (rc) break;
    or_composite(static_ssq, hssq, V, c);
    if (out_ssq) memcpy(out_ssq + (int64_t)s * V, c, sizeof(int32_t) * V);
    if (out_sdf) or_to_float(c, V, h, out_sdf + (int64_t)s * V);
  }
  free(hocc); free(hssq); free(c);
  return rc;
}

/* ---------------------------------------------------------------------
 * Brute force, straight from the definition: nearest voxel of a set by
 * exhaustive search.  Used to pin the separable EDT on tiny grids and to
 * check sampled voxels at full size.
 * ------------------------------------------------------------------- */
int64_t or_edt_at(const uint8_t *set, int want, int nx, int ny, int nz,
                  int i, int j, int k) {
  int64_t best = OR_INF64;
  for (int kk = 0; kk < nz; kk++) {
    int64_t dz = kk - k;
    int64_t dz2 = dz * dz;
    if (dz2 >= best) continue;
    for (int jj = 0; jj < ny; jj++) {
      int64_t dy = jj - j;
      int64_t dzy = dz2 + dy * dy;
      if (dzy >= best) continue;
      const uint8_t *row = set + ((int64_t)kk * ny + jj) * nx;
      for (int ii = 0; ii < nx; ii++) {
        if ((row[ii] != 0) != (want != 0)) continue;
        int64_t dx = ii - i;
        int64_t d = dzy + dx * dx;
        if (d < best) best = d;
      }
    }
  }
  return best;
}

/* Signed-squared value of one voxel by brute force. */
int32_t or_ssq_at(const uint8_t *set, int nx, int ny, int nz, int i, int j,
                  int k) {
  int inside = set[((int64_t)k * ny + j) * nx + i] != 0;
  int64_t e = or_edt_at(set, inside ? 0 : 1, nx, ny, nz, i, j, k);
  if (e == OR_INF64) return inside ? -OR_INF32 : OR_INF32;
  return inside ? -(int32_t)e : (int32_t)e;
}

/* ---------------------------------------------------------------------
 * Sphere query on a slice field (GPMP2 obstacle factors sample the
 * distance field and its gradient; RHAP-GPMP2 assigns slice n-1 to every
 * time index past the horizon).
 *
 * Trilinear interpolation of the fp32 field between voxel centres, in
 * fp64:  g_a = (c_a - o_a)/h - 1/2; out-of-range g is clamped and flagged;
 * i_a = min(floor(g_a), n_a - 2); f_a = g_a - i_a;
 * D = sum_{abc} w_a w_b w_c q_abc;  dD/dg_x = sum_{bc} w_b w_c (q_1bc -
 * q_0bc) and likewise for y, z;  gradient = dD/dg / h.
 * Outputs: dist = fp32(D - r), grad = fp32(gradient), optional hinge cost
 * max(0, eps - (D - r)) as fp32.
 * Status bits: 1,2,4 = x,y,z out of range; 8 = slice clamped to n-1;
 * 16 = an infinite corner (then dist = +-inf, grad = 0); 32 = negative
 * slice (then dist, grad and cost are NaN).
 * Requires every n_a >= 2.
 * ------------------------------------------------------------------- */
#define OR_OOR_X 1
#define OR_OOR_Y 2
#define OR_OOR_Z 4
#define OR_SLICE_CLAMPED 8
#define OR_INF_CORNER 16
#define OR_SLICE_NEG 32

void or_query(const float *sdf, int n_slices, int nx, int ny, int nz,
              double h, double ox, double oy, double oz, int n_queries,
              const float *centre, const float *radius, const int32_t *slice,
              double hinge_eps, float *dist, float *grad, uint8_t *status,
              float *cost) {
  const int64_t V = (int64_t)nx * ny * nz;
  const int n[3] = {nx, ny, nz};
  const double o[3] = {ox, oy, oz};
  for (int q = 0; q < n_queries; q++) {
    uint8_t st = 0;
    int s = slice[q];
    if (s < 0) {
      st |= OR_SLICE_NEG;
      dist[q] = NAN;
      grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = NAN;
      if (cost) cost[q] = NAN;
      if (status) status[q] = st;
      continue;
    }
    if (s > n_slices - 1) {
      s = n_slices - 1;
      st |= OR_SLICE_CLAMPED;
    }
    const float *field = sdf + (int64_t)s * V;
    int idx[3];
    double fr[3];
    for (int a = 0; a < 3; a++) {
      double g = ((double)centre[3 * q + a] - o[a]) / h - 0.5;
      if (g < 0.0) {
        g = 0.0;
        st |= (uint8_t)(1 << a);
      } else if (g > (double)(n[a] - 1)) {
        g = (double)(n[a] - 1);
        st |= (uint8_t)(1 << a);
      }
      int i = (int)floor(g);
      if (i > n[a] - 2) i = n[a] - 2;
      idx[a] = i;
      fr[a] = g - (double)i;
    }
    double c[2][2][2];
    int infc = 0;
    double infval = 0.0;
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++)
        for (int e = 0; e < 2; e++) {
          int64_t v = ((int64_t)(idx[2] + e) * ny + (idx[1] + b)) * nx +
                      (idx[0] + a);
          c[a][b][e] = (double)field[v];
          if (isinf(c[a][b][e]) && !infc) {
            infc = 1;
            infval = c[a][b][e];
          }
        }
    if (infc) {
      st |= OR_INF_CORNER;
      dist[q] = (float)infval;
      grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = 0.0f;
      if (cost) cost[q] = infval > 0 ? 0.0f : HUGE_VALF;
      if (status) status[q] = st;
      continue;
    }
    double w[3][2];
    for (int a = 0; a < 3; a++) {
      w[a][0] = 1.0 - fr[a];
      w[a][1] = fr[a];
    }
    double D = 0.0;
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++)
        for (int e = 0; e < 2; e++)
          D += w[0][a] * w[1][b] * w[2][e] * c[a][b][e];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int b = 0; b < 2; b++)
      for (int e = 0; e < 2; e++)
        gx += w[1][b] * w[2][e] * (c[1][b][e] - c[0][b][e]);
    for (int a = 0; a < 2; a++)
      for (int e = 0; e < 2; e++)
        gy += w[0][a] * w[2][e] * (c[a][1][e] - c[a][0][e]);
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++)
        gz += w[0][a] * w[1][b] * (c[a][b][1] - c[a][b][0]);
    double dsph = D - (double)radius[q];
    dist[q] = (float)dsph;
    grad[3 * q] = (float)(gx / h);
    grad[3 * q + 1] = (float)(gy / h);
    grad[3 * q + 2] = (float)(gz / h);
    if (cost) {
      double hc = hinge_eps - dsph;
      cost[q] = (float)(hc > 0.0 ? hc : 0.0);
    }
    if (status) status[q] = st;
  }
}
