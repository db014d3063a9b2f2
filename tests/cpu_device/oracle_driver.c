/* Drives the C oracle from a binary scene file so that it can be built
 * and run under the address and undefined-behaviour sanitizers (a test
 * build only: the oracle itself is loaded by Python without them).
 *
 * Input: int32 nx, ny, nz, n_slices, n_humans, n_queries; fp64 h, ox, oy,
 * oz, radius, height; uint8 occ[V]; fp64 xy[n_slices][n_humans][2];
 * fp32 centre[Q][3], radius[Q]; int32 slice[Q].
 * Output: int32 static[V], composite[n][V]; fp32 sdf[n][V], dist[Q],
 * grad[Q][3], cost[Q]; uint8 status[Q]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_build_static(const uint8_t *occ, int nx, int ny, int nz, double h,
                    int32_t *ssq, float *sdf);
int or_predicted_composite(const int32_t *static_ssq, int nx, int ny, int nz,
                           double h, double ox, double oy, double oz,
                           int n_slices, int n_humans, const double *xy,
                           double radius, double height, int32_t *out_ssq,
                           float *out_sdf);
void or_query(const float *sdf, int n_slices, int nx, int ny, int nz,
              double h, double ox, double oy, double oz, int n_queries,
              const float *centre, const float *radius, const int32_t *slice,
              double hinge_eps, float *dist, float *grad, uint8_t *status,
              float *cost);

static void *take(FILE *f, size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t *d = take(f, 6 * sizeof(int32_t));
  double *r = take(f, 6 * sizeof(double));
  const int nx = d[0], ny = d[1], nz = d[2], n = d[3], K = d[4], Q = d[5];
  const size_t V = (size_t)nx * ny * nz;
  uint8_t *occ = take(f, V);
  double *xy = take(f, sizeof(double) * 2 * (size_t)n * K);
  float *centre = take(f, sizeof(float) * 3 * (size_t)Q);
  float *rad = take(f, sizeof(float) * (size_t)Q);
  int32_t *slice = take(f, sizeof(int32_t) * (size_t)Q);
  fclose(f);
  int32_t *st = malloc(sizeof(int32_t) * V);
  int32_t *c = malloc(sizeof(int32_t) * V * n);
  float *cf = malloc(sizeof(float) * V * n);
  float *dist = malloc(sizeof(float) * (Q + 1));
  float *grad = malloc(sizeof(float) * 3 * (Q + 1));
  float *cost = malloc(sizeof(float) * (Q + 1));
  uint8_t *status = malloc(Q + 1);
  if (!st || !c || !cf || !dist || !grad || !cost || !status) return 3;
  if (or_build_static(occ, nx, ny, nz, r[0], st, NULL)) return 4;
  if (or_predicted_composite(st, nx, ny, nz, r[0], r[1], r[2], r[3], n, K, xy,
                             r[4], r[5], c, cf))
    return 5;
  or_query(cf, n, nx, ny, nz, r[0], r[1], r[2], r[3], Q, centre, rad, slice,
           0.3, dist, grad, status, cost);
  FILE *o = fopen(argv[2], "wb");
  if (!o) return 6;
  fwrite(st, sizeof(int32_t), V, o);
  fwrite(c, sizeof(int32_t), V * n, o);
  fwrite(cf, sizeof(float), V * n, o);
  fwrite(dist, sizeof(float), Q, o);
  fwrite(grad, sizeof(float), 3 * (size_t)Q, o);
  fwrite(cost, sizeof(float), Q, o);
  fwrite(status, 1, Q, o);
  fclose(o);
  free(d); free(r); free(occ); free(xy); free(centre); free(rad); free(slice);
  free(st); free(c); free(cf); free(dist); free(grad); free(cost);
  free(status);
  return 0;
}
