// Planar signed EDT of the humans' disk union, one plane per slice.
//
// A slice's human voxels are D x Z (see composite.hip), with D the union of
// the voxelised disks.  Each disk is convex, so its voxels in grid row j
// form one integer interval, a chord [a, b] of the closed predicate
//   (2^15(2i+1) - X)^2 + (2^15(2j+1) - Y)^2 <= R^2:
// with dy = 2^15(2j+1) - Y and W = floor(sqrt(R^2 - dy^2)), a voxel is in
// the chord iff |2^15(2i+1) - X| <= W, i.e. 2i+1 lies in
// [ceil((X-W)/2^15), floor((X+W)/2^15)].  All of this is exact integer
// arithmetic (divisions by powers of two are arithmetic shifts).
//
// With the chords in hand every pixel is independent, so the plane is
// computed one pixel per lane instead of by sequential column sweeps:
//   outside D:  E_D(i,j) = min over disks, over the disk's rows jj, of
//               (j-jj)^2 + (distance from i to the chord)^2,
//               pruned by each disk's bounding box and by (j-jj)^2 >= best;
//   inside D:   E_{Gxy\D}(i,j) = min over rows jj of
//               (j-jj)^2 + (distance from i to the nearest uncovered pixel
//               of row jj)^2, searching rows outward from j and stopping
//               once (j-jj)^2 reaches the best value; in a row the covered
//               run through i is the union of the chords that overlap or
//               touch it.
// Both are the definition of the squared distance written row by row
// (the x term of the nearest voxel in row jj is the distance to the
// nearest chord end), so the result is exact.
#include <type_traits>

#include "internal.h"

namespace pcsdf {

__device__ __forceinline__ int64_t floor_pow2(int64_t a, int sh) {
  return a >> sh;  // arithmetic shift: floor division by 2^sh
}
__device__ __forceinline__ int64_t ceil_pow2(int64_t a, int sh) {
  return -((-a) >> sh);
}

// Voxel indices i whose centres satisfy |2^15(2i+1) - C| <= W.
__device__ __forceinline__ void index_range(int64_t C, int64_t W, int n,
                                            int *lo, int *hi) {
  const int64_t lt = ceil_pow2(C - W, 15);   // smallest admissible 2i+1
  const int64_t ht = floor_pow2(C + W, 15);  // largest admissible 2i+1
  int64_t a = ceil_pow2(lt - 1, 1);
  int64_t b = floor_pow2(ht - 1, 1);
  if (a < 0) a = 0;
  if (b > n - 1) b = n - 1;
  if (a > b) {
    *lo = 1;
    *hi = 0;
  } else {
    *lo = (int)a;
    *hi = (int)b;
  }
}

__device__ __forceinline__ int64_t isqrt64(int64_t v) {
  int64_t r = (int64_t)sqrt((double)v);
  while (r > 0 && r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// chords[s][k][j] = (a, b), empty when a > b.
__global__ __launch_bounds__(256) void k_chords(const int64_t *__restrict__ xy,
                                                int K, int64_t R, int nx,
                                                int ny, int64_t total,
                                                int2 *__restrict__ chords) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int j = (int)(t % ny);
  const int64_t sk = t / ny;  // s*K + k
  const int64_t X = xy[2 * sk], Y = xy[2 * sk + 1];
  const int64_t dy = 32768LL * (2LL * j + 1) - Y;
  int2 c = make_int2(1, 0);
  if (dy <= R && dy >= -R) {
    const int64_t W = isqrt64(R * R - dy * dy);
    index_range(X, W, nx, &c.x, &c.y);
  }
  chords[t] = c;
}

__device__ __forceinline__ bool covers(int2 c, int i) {
  return c.x <= i && i <= c.y;
}

// Squared distance along row jj from pixel i to the nearest uncovered
// pixel of that row: 0 if i is uncovered, kInf if the row is covered.
// `ch` is the slice's chord table [K][ny].
template <class Tab>
__device__ __forceinline__ int32_t row_free_dist(const Tab &ch, int K, int ny,
                                                 int nx, int jj, int i) {
  bool cov = false;
  for (int k = 0; k < K; ++k) cov |= covers(ch[k * ny + jj], i);
  if (!cov) return 0;
  int lo = i, hi = i;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int k = 0; k < K; ++k) {
      const int2 c = ch[k * ny + jj];
      if (c.x <= c.y && c.x <= hi + 1 && c.y >= lo - 1) {
        if (c.x < lo) {
          lo = c.x;
          changed = true;
        }
        if (c.y > hi) {
          hi = c.y;
          changed = true;
        }
      }
    }
  }
  const int dl = lo >= 1 ? i - lo + 1 : kInf;
  const int dr = hi <= nx - 2 ? hi + 1 - i : kInf;
  const int d = dl < dr ? dl : dr;
  return d == kInf ? kInf : d * d;
}

// Chord table views: LDS (ds_read) or global memory through the cache.
struct LdsTab {
  const int2 *p;  // points into __shared__ memory
  __device__ __forceinline__ int2 operator[](int t) const { return p[t]; }
};
struct GlobalTab {
  const int2 *__restrict__ p;
  __device__ __forceinline__ int2 operator[](int t) const { return p[t]; }
};

// Row pass of the free-set channel for every pixel of every slice:
// F1[s][j][i] = squared distance along row j to the nearest uncovered
// pixel (0 when (i, j) is uncovered, kInf when the whole row is covered).
__global__ __launch_bounds__(256) void k_rowfree(
    const int2 *__restrict__ chords, int K, int nx, int ny, int64_t total,
    int32_t *__restrict__ F1) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int64_t row = t / nx;  // s*ny + j
  const int i = (int)(t - row * nx);
  const int64_t s = row / ny;
  const int j = (int)(row - s * ny);
  const GlobalTab ch{chords + s * K * ny};
  F1[t] = row_free_dist(ch, K, ny, nx, j, i);
}

// Squared distance from pixel (i, j) to the chords of rows [lo, hi] of one
// disk, visiting rows in order of growing |jj - j| from row j0 in `dir`,
// four rows per step so their loads overlap.
template <class Tab>
__device__ __forceinline__ int32_t scan_rows(const Tab &ch, int base, int i,
                                             int j, int j0, int end, int dir,
                                             int dxb2, int32_t best) {
  for (int jj = j0; dir > 0 ? jj <= end : jj >= end; jj += 4 * dir) {
    const int dy0 = jj - j;
    // every remaining row is at least this far: (dy)^2 plus the squared
    // distance to the disk's x extent
    if (dy0 * dy0 + dxb2 >= best) break;
    int2 c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = jj + u * dir;
      const bool in = dir > 0 ? r <= end : r >= end;
      c[u] = in ? ch[base + r] : make_int2(1, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int dy = dy0 + u * dir;
      if (c[u].x > c[u].y) continue;
      const int dx = i < c[u].x ? c[u].x - i : (i > c[u].y ? i - c[u].y : 0);
      best = min(best, dy * dy + dx * dx);
    }
  }
  return best;
}

// Squared distance from (i, j) to disk k's chords, or `best` if the disk
// cannot improve on it.
template <class Tab>
__device__ __forceinline__ int32_t scan_disk(const Tab &ch, int4 b, int k,
                                             int ny, int i, int j,
                                             int32_t best) {
  if (b.x > b.y || b.z > b.w) return best;
  const int dxb = max(0, max(b.x - i, i - b.y));
  const int dyb = max(0, max(b.z - j, j - b.w));
  const int dxb2 = dxb * dxb;
  if (dxb2 + dyb * dyb >= best) return best;
  const int j0 = min(max(j, b.z), b.w);
  best = scan_rows(ch, k * ny, i, j, j0, b.w, +1, dxb2, best);
  return scan_rows(ch, k * ny, i, j, j0 - 1, b.z, -1, dxb2, best);
}

// One block per (tile, slice).  The slice's chords (K*ny pairs) are staged
// in LDS when they fit (kLds), else read through the cache from global
// memory; the disks' bounding boxes always live in LDS.
template <bool kLds>
__global__ __launch_bounds__(256) void k_planes(
    const int2 *__restrict__ chords, const int64_t *__restrict__ xy, int K,
    int64_t R, int nx, int ny, int tiles, const int32_t *__restrict__ F1,
    int32_t *__restrict__ P) {
  extern __shared__ int4 sh4[];
  const int s = blockIdx.x / tiles;
  const int tile = blockIdx.x - s * tiles;
  const int2 *gch = chords + (int64_t)s * K * ny;
  int4 *box = sh4;                                   // K boxes
  int2 *lch = reinterpret_cast<int2 *>(sh4 + K);     // K*ny chords
  if (kLds)
    for (int t = threadIdx.x; t < K * ny; t += 256) lch[t] = gch[t];
  for (int k = threadIdx.x; k < K; k += 256) {
    const int64_t X = xy[2 * ((int64_t)s * K + k)];
    const int64_t Y = xy[2 * ((int64_t)s * K + k) + 1];
    int4 b;
    index_range(X, R, nx, &b.x, &b.y);  // superset of every chord
    index_range(Y, R, ny, &b.z, &b.w);  // exact row span
    box[k] = b;
  }
  __syncthreads();
  typename std::conditional<kLds, LdsTab, GlobalTab>::type ch{kLds ? lch
                                                                   : gch};

  const int npx = nx * ny;
  for (int p = tile * 256 + threadIdx.x; p < npx; p += tiles * 256) {
    const int j = p / nx;
    const int i = p - j * nx;
    bool inside = false;
    for (int k = 0; k < K; ++k) inside |= covers(ch[k * ny + j], i);
    int32_t out;
    if (!inside) {
      // The disk with the smallest bounding-box bound first, so the
      // others are mostly pruned.
      int kbest = -1;
      int lbmin = kInf;
      for (int k = 0; k < K; ++k) {
        const int4 b = box[k];
        if (b.x > b.y || b.z > b.w) continue;
        const int dxb = max(0, max(b.x - i, i - b.y));
        const int dyb = max(0, max(b.z - j, j - b.w));
        const int lb = dxb * dxb + dyb * dyb;
        if (lb < lbmin) {
          lbmin = lb;
          kbest = k;
        }
      }
      int32_t best = kInf;
      if (kbest >= 0) best = scan_disk(ch, box[kbest], kbest, ny, i, j, best);
      for (int k = 0; k < K; ++k)
        if (k != kbest) best = scan_disk(ch, box[k], k, ny, i, j, best);
      out = best;
    } else {
      // Rows outward from j, eight rows (four distances) per step so the
      // loads of the precomputed row distances overlap.
      const int32_t *f1 = F1 + (int64_t)s * npx + i;
      int32_t best = f1[(int64_t)j * nx];
      const int dmax = max(j, ny - 1 - j);
      for (int d0 = 1; d0 <= dmax; d0 += 4) {
        if (d0 * d0 >= best) break;
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int d = d0 + u;
          v[2 * u] = (d <= dmax && j - d >= 0) ? f1[(int64_t)(j - d) * nx]
                                               : kInf;
          v[2 * u + 1] = (d <= dmax && j + d < ny)
                             ? f1[(int64_t)(j + d) * nx]
                             : kInf;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int d2 = (d0 + u) * (d0 + u);
          if (v[2 * u] != kInf) best = min(best, d2 + v[2 * u]);
          if (v[2 * u + 1] != kInf) best = min(best, d2 + v[2 * u + 1]);
        }
      }
      out = best == kInf ? -kInf : -best;
    }
    P[(int64_t)s * npx + p] = out;
  }
}

int launch_planes(Handle *h, const int64_t *xy, int K, int64_t R, bool empty,
                  int2 *chords, int32_t *P, int nx, int ny, int n_slices,
                  hipStream_t s) {
  const int Keff = empty ? 0 : K;
  const int64_t total = (int64_t)n_slices * Keff * ny;
  if (total > 0) {
    hipLaunchKernelGGL(k_chords, dim3((unsigned)((total + 255) / 256)),
                       dim3(256), 0, s, xy, Keff, R, nx, ny, total, chords);
    int rc = check_launch(h, "chords");
    if (rc) return rc;
  }
  const int npx = nx * ny;
  int32_t *F1 = P + (int64_t)n_slices * npx;
  const int64_t npix = (int64_t)n_slices * npx;
  if (Keff > 0) {
    hipLaunchKernelGGL(k_rowfree, dim3((unsigned)((npix + 255) / 256)),
                       dim3(256), 0, s, chords, Keff, nx, ny, npix, F1);
    int rc = check_launch(h, "rowfree");
    if (rc) return rc;
  }
  int tiles = (2048 + n_slices - 1) / n_slices;
  const int maxt = (npx + 255) / 256;
  if (tiles > maxt) tiles = maxt;
  if (tiles < 1) tiles = 1;
  const size_t box_bytes = (size_t)Keff * sizeof(int4);
  const size_t ch_bytes = (size_t)Keff * ny * sizeof(int2);
  const bool use_lds = box_bytes + ch_bytes <= 48 * 1024;
  const dim3 grid((unsigned)((int64_t)tiles * n_slices)), block(256);
  if (use_lds)
    hipLaunchKernelGGL(k_planes<true>, grid, block, box_bytes + ch_bytes, s,
                       chords, xy, Keff, R, nx, ny, tiles, F1, P);
  else
    hipLaunchKernelGGL(k_planes<false>, grid, block, box_bytes, s, chords, xy,
                       Keff, R, nx, ny, tiles, F1, P);
  return check_launch(h, "planes");
}

}  // namespace pcsdf
