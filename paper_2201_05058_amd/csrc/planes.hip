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
#include "plane_device.h"

namespace pcsdf {

// chords[s][k][j] = (a, b), empty when a > b.
// Slices whose entry in `need` is zero are skipped (all slices when `need`
// is null) by this kernel and the two below.
// Rs[s] is slice s's fixed-point disk radius.
__global__ __launch_bounds__(256) void k_chords(Centres C, int K, int nx,
                                                int ny, int64_t total,
                                                const int32_t *__restrict__ need,
                                                int2 *__restrict__ chords) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int j = (int)(t % ny);
  const int64_t sk = t / ny;  // s*K + k
  if (need && need[sk / K] == 0) return;
  const int64_t X = centre_word(C, 2 * sk), Y = centre_word(C, 2 * sk + 1);
  const int2 c = disk_chord(X, Y, radius_of(C, sk / K), nx, j);
  chords[t] = c;
}

// Row pass of the free-set channel for every pixel of every slice:
// F1[s][j][i] = squared distance along row j to the nearest uncovered
// pixel (0 when (i, j) is uncovered, kInf when the whole row is covered).
// Block b takes pixels 256 (b mod bpr) + 0..255 of row b / bpr of all
// slices' rows: the row, and so its chords, is uniform over the block.
__global__ __launch_bounds__(256) void k_rowfree(
    const int2 *__restrict__ chords, int K, int nx, int ny, int bpr,
    const int32_t *__restrict__ need, int32_t *__restrict__ F1) {
  const int row = (int)(blockIdx.x / (unsigned)bpr);  // s*ny + j
  const int i = (int)(blockIdx.x - (unsigned)row * bpr) * 256 + threadIdx.x;
  const int s = row / ny;
  if (i >= nx || (need && need[s] == 0)) return;
  const int j = row - s * ny;
  const GlobalTab ch{chords + (int64_t)s * K * ny};
  F1[(int64_t)row * nx + i] = row_free_dist(ch, K, ny, nx, j, i);
}

// Coverage of every pixel of every slice by the disks, one byte per pixel
// (1: covered): the map whose 2-D signed EDT is the planar field.  One
// block per row of one slice (nx <= 1024): the row's K chords are staged
// in LDS, and each lane marks 4 adjacent pixels, stored as one word when
// the row allows it.
__global__ __launch_bounds__(256) void k_cover(
    const int2 *__restrict__ chords, int K, int nx, int ny,
    uint8_t *__restrict__ cov) {
  __shared__ int2 rc[kMaxHumans];
  const int row = blockIdx.x;  // s*ny + j
  const int s = row / ny, j = row - s * ny;
  const int2 *ch = chords + (int64_t)s * K * ny + j;
  for (int k = threadIdx.x; k < K; k += 256) rc[k] = ch[k * ny];
  __syncthreads();
  const int i0 = 4 * threadIdx.x;
  if (i0 >= nx) return;
  uint32_t m = 0;  // bit e: pixel i0 + e is covered
  for (int k = 0; k < K; ++k) {
    const int2 c = rc[k];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      m |= (c.x <= i0 + e && i0 + e <= c.y) ? 1u << e : 0u;
  }
  uint8_t *dst = cov + (int64_t)row * nx + i0;
  if (nx % 4 == 0) {  // the word is inside the row and 4-byte aligned
    *reinterpret_cast<uint32_t *>(dst) =
        (m & 1u) | ((m & 2u) << 7) | ((m & 4u) << 14) | ((m & 8u) << 21);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < nx) dst[e] = (m >> e) & 1u;
  }
}

// One block per (tile, slice).  The slice's chords (K*ny pairs) are staged
// in LDS when they fit (kLds), else read through the cache from global
// memory; the disks' bounding boxes always live in LDS.  Blocks of 16
// waves: two share a CU's waves at 33 KB of LDS each for 8 humans x 512
// rows (blocks of 4 waves would be limited to 16 waves per CU by LDS),
// and the per-pixel row scans are chains of LDS round trips.
constexpr int kPlaneThreads = 1024;
template <bool kLds>
__global__ __launch_bounds__(kPlaneThreads) void k_planes(
    const int2 *__restrict__ chords, Centres C, int K, int nx, int ny,
    int tiles, const int32_t *__restrict__ F1,
    const int32_t *__restrict__ need, int32_t *__restrict__ P) {
  extern __shared__ int4 sh4[];
  const int s = blockIdx.x / tiles;
  const int tile = blockIdx.x - s * tiles;
  if (need && need[s] == 0) return;  // uniform over the block
  const int64_t R = radius_of(C, s);
  const int2 *gch = chords + (int64_t)s * K * ny;
  int4 *box = sh4;                                   // K boxes
  int2 *lch = reinterpret_cast<int2 *>(sh4 + K);     // K*ny chords
  if (kLds)
    for (int t = threadIdx.x; t < K * ny; t += kPlaneThreads) lch[t] = gch[t];
  for (int k = threadIdx.x; k < K; k += kPlaneThreads) {
    const int64_t X = centre_word(C, 2 * ((int64_t)s * K + k));
    const int64_t Y = centre_word(C, 2 * ((int64_t)s * K + k) + 1);
    const int4 b = disk_box(X, Y, R, nx, ny);
    box[k] = b;
  }
  __syncthreads();
  typename std::conditional<kLds, LdsTab, GlobalTab>::type ch{kLds ? lch
                                                                   : gch};

  const int npx = nx * ny;
  for (int p = tile * kPlaneThreads + threadIdx.x; p < npx;
       p += tiles * kPlaneThreads) {
    const int j = p / nx;
    const int i = p - j * nx;
    const int32_t out = plane_value(ch, box, F1 + (int64_t)s * npx + i, K, nx,
                                    ny, i, j);
    P[(int64_t)s * npx + p] = out;
  }
}

int launch_chords(Handle *h, const Centres &C, int K, int2 *chords, int nx,
                  int ny, int n_slices, const int32_t *need, hipStream_t s) {
  const int64_t total = (int64_t)n_slices * K * ny;
  if (total <= 0) return PCSDF_OK;
  launch_timed(h, k_chords, dim3((unsigned)((total + 255) / 256)), dim3(256),
               0u, s, C, K, nx, ny, total, need, chords);
  return check_launch(h, "chords");
}

int launch_planes(Handle *h, const Centres &C, int K, bool empty,
                  int2 *chords, int32_t *P, int nx, int ny, int n_slices,
                  const int32_t *need, hipStream_t s) {
  const int Keff = empty ? 0 : K;
  int rc0 = launch_chords(h, C, Keff, chords, nx, ny, n_slices, need, s);
  if (rc0) return rc0;
  const int npx = nx * ny;
  int32_t *F1 = P + (int64_t)n_slices * npx;
  const int64_t npix = (int64_t)n_slices * npx;
  if (!need && Keff > 0 && ny <= 512 && h->tuning.static_segments == 0 &&
      (int64_t)((nx + 63) / 64) * n_slices >= 256) {
    // Every slice of a large stack: the planar field is the 2-D signed EDT
    // of the disks' coverage, by the static build's row pass and y column
    // pass over the stack of slices (each slice a z layer of an
    // nx x ny x n grid).  The coverage bytes use the front of P, the row
    // pass's output the back.  With the default segment counts (a static
    // build tuning sends the planes to the per-pixel kernel) columns of at
    // most 512 pixels keep the column pass's envelopes in LDS (16-bit
    // entries), so no workspace is allocated.  Below one workgroup of
    // column segments per CU (64 columns of a slice each) the per-pixel
    // kernel is faster (512 x 512 x 50 slices: 0.20 ms against 0.47;
    // 256 x 256 x 20: 0.076 against 0.035).
    uint8_t *cov = reinterpret_cast<uint8_t *>(P);
    launch_timed(h, k_cover, dim3((unsigned)(npix / nx)), dim3(256), 0u, s,
                 chords, Keff, nx, ny, cov);
    int rc = check_launch(h, "cover");
    if (!rc) rc = launch_pass_x_u8(h, cov, F1, nx, (int64_t)n_slices * ny, s);
    if (!rc)
      rc = launch_pass_col(h, F1, P, nullptr, 1.0f, nx, n_slices, ny, nx,
                           (int64_t)npx, true, false, s);
    return rc;
  }
  if (Keff > 0) {
    const int bpr = (nx + 255) / 256;
    launch_timed(h, k_rowfree, dim3((unsigned)(npix / nx * bpr)), dim3(256),
                 0, s, chords, Keff, nx, ny, bpr, need, F1);
    int rc = check_launch(h, "rowfree");
    if (rc) return rc;
  }
  int tiles = (512 + n_slices - 1) / n_slices;
  const int maxt = (npx + kPlaneThreads - 1) / kPlaneThreads;
  if (tiles > maxt) tiles = maxt;
  if (tiles < 1) tiles = 1;
  const size_t box_bytes = (size_t)Keff * sizeof(int4);
  const size_t ch_bytes = (size_t)Keff * ny * sizeof(int2);
  const bool use_lds = box_bytes + ch_bytes <= 48 * 1024;
  const dim3 grid((unsigned)((int64_t)tiles * n_slices)),
      block(kPlaneThreads);
  if (use_lds)
    launch_timed(h, k_planes<true>, grid, block,
                 (uint32_t)(box_bytes + ch_bytes), s, chords, C, Keff, nx, ny,
                 tiles, F1, need, P);
  else
    launch_timed(h, k_planes<false>, grid, block, (uint32_t)box_bytes, s,
                 chords, C, Keff, nx, ny, tiles, F1, need, P);
  return check_launch(h, "planes");
}

}  // namespace pcsdf
