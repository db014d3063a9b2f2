// Device helpers of the humans' planar field, shared by the per-call
// kernels (planes.hip) and the batch's planar workers (batch.hip).
// See planes.hip for the method: exact integer chords of the voxelised
// disks, a row pass of the free set, and bounded row searches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcsdf {

constexpr int32_t kInfP = INT32_MAX;

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

// Chord of disk (X, Y, R) in row j, clipped to [0, nx): (a, b), a > b if
// empty.
__device__ __forceinline__ int2 disk_chord(int64_t X, int64_t Y, int64_t R,
                                           int nx, int j) {
  const int64_t dy = 32768LL * (2LL * j + 1) - Y;
  int2 c = make_int2(1, 0);
  if (dy <= R && dy >= -R) {
    const int64_t W = isqrt64(R * R - dy * dy);
    index_range(X, W, nx, &c.x, &c.y);
  }
  return c;
}

// Bounding box (i range superset, exact j range) of disk (X, Y, R).
__device__ __forceinline__ int4 disk_box(int64_t X, int64_t Y, int64_t R,
                                         int nx, int ny) {
  int4 b;
  index_range(X, R, nx, &b.x, &b.y);
  index_range(Y, R, ny, &b.z, &b.w);
  return b;
}

// v^2 on the full-rate 24-bit multiplier: pixel offsets are below 2^11.
__device__ __forceinline__ int32_t sq24(int v) { return __mul24(v, v); }

__device__ __forceinline__ bool covers(int2 c, int i) {
  return c.x <= i && i <= c.y;
}

// Squared distance along row jj from pixel i to the nearest uncovered
// pixel of that row: 0 if i is uncovered, kInfP if the row is covered.
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
  const int dl = lo >= 1 ? i - lo + 1 : kInfP;
  const int dr = hi <= nx - 2 ? hi + 1 - i : kInfP;
  const int d = dl < dr ? dl : dr;
  return d == kInfP ? kInfP : sq24(d);
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
    if (sq24(dy0) + dxb2 >= best) break;
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
      best = min(best, sq24(dy) + sq24(dx));
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
  const int dxb2 = sq24(dxb);
  if (dxb2 + sq24(dyb) >= best) return best;
  const int j0 = min(max(j, b.z), b.w);
  best = scan_rows(ch, k * ny, i, j, j0, b.w, +1, dxb2, best);
  return scan_rows(ch, k * ny, i, j, j0 - 1, b.z, -1, dxb2, best);
}

// Row-pass values of the free set at column i: precomputed (f1[j*nx] is
// row j) or computed from the chords on demand.
struct RowFreeTable {
  const int32_t *f1;
  int nx;
  __device__ __forceinline__ int32_t operator()(int jr) const {
    return f1[__mul24(jr, nx)];  // jr nx < 2^20
  }
};
template <class Tab>
struct RowFreeChords {
  const Tab &ch;
  int K, ny, nx, i;
  __device__ __forceinline__ int32_t operator()(int jr) const {
    return row_free_dist(ch, K, ny, nx, jr, i);
  }
};

// Planar signed value of pixel (i, j): E_D outside the disk union, -E of
// its complement inside (+-kInfP when the other set is empty).  `ch` is the
// slice's chord table [K][ny], `box` its K boxes, rf the row pass of the
// free set at column i.
template <class Tab, class BoxTab, class RowFree>
__device__ __forceinline__ int32_t plane_value_rf(const Tab &ch,
                                                  const BoxTab &box,
                                                  const RowFree &rf, int K,
                                                  int nx, int ny, int i,
                                                  int j) {
  bool inside = false;
  for (int k = 0; k < K; ++k) inside |= covers(ch[k * ny + j], i);
  int32_t out;
  if (!inside) {
    // The disk with the smallest bounding-box bound first, so the
    // others are mostly pruned.
    int kbest = -1;
    int lbmin = kInfP;
    for (int k = 0; k < K; ++k) {
      const int4 b = box[k];
      if (b.x > b.y || b.z > b.w) continue;
      const int dxb = max(0, max(b.x - i, i - b.y));
      const int dyb = max(0, max(b.z - j, j - b.w));
      const int lb = sq24(dxb) + sq24(dyb);
      if (lb < lbmin) {
        lbmin = lb;
        kbest = k;
      }
    }
    int32_t best = kInfP;
    if (kbest >= 0) best = scan_disk(ch, box[kbest], kbest, ny, i, j, best);
    for (int k = 0; k < K; ++k)
      if (k != kbest) best = scan_disk(ch, box[k], k, ny, i, j, best);
    out = best;
  } else {
    // Rows outward from j, eight rows (four distances) per step so the
    // loads of the precomputed row distances overlap.
    int32_t best = rf(j);
    const int dmax = max(j, ny - 1 - j);
    for (int d0 = 1; d0 <= dmax; d0 += 4) {
      if (sq24(d0) >= best) break;
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int d = d0 + u;
        v[2 * u] = (d <= dmax && j - d >= 0) ? rf(j - d) : kInfP;
        v[2 * u + 1] = (d <= dmax && j + d < ny) ? rf(j + d) : kInfP;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int d2 = sq24(d0 + u);
        if (v[2 * u] != kInfP) best = min(best, d2 + v[2 * u]);
        if (v[2 * u + 1] != kInfP) best = min(best, d2 + v[2 * u + 1]);
      }
    }
    out = best == kInfP ? -kInfP : -best;
  }
  return out;
}

// The same with the row pass precomputed: f1 offset to column i.
template <class Tab, class BoxTab>
__device__ __forceinline__ int32_t plane_value(const Tab &ch, const BoxTab &box,
                                               const int32_t *f1, int K,
                                               int nx, int ny, int i, int j) {
  return plane_value_rf(ch, box, RowFreeTable{f1, nx}, K, nx, ny, i, j);
}

}  // namespace pcsdf
