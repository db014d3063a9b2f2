// Device side of the batched composite (see batch.hip): scene table entry,
// planar-field item, composite chunk and the persistent worker loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "plane_device.h"

namespace pcsdf {

struct SceneDev {
  const int32_t *S;
  int32_t *oc;
  float *of;
  const int64_t *xy;  // [n][K][2] fixed-point centres
  int2 *chords;       // [n][K][ny] (used when the table exceeds LDS)
  int32_t *P;         // [n][ny][nx] planar fields
  int32_t *F1;        // [n][ny][nx] row pass of the free set
  int64_t R;
  uint32_t V;
  int nx, ny, nz, n, K, Kt, has_above, vec4;
  float hf;
  int pad[2];
};

constexpr int kItemPlane = 0;
constexpr int kItemComposite = 1;
// Pixels of one planar item when the slice's chords fit in LDS.
constexpr int kPlaneTile = 4096;

__host__ __device__ inline bool chords_in_lds(int K, int ny, int lds_cap) {
  return K * 16 + K * ny * 8 <= lds_cap;
}

// ------------------------------------------------------------ device side

// Planar field of slice s.  When the chords fit in LDS the slice is split
// into tiles of kPlaneTile pixels, each an item of its own: the item
// builds the slice's chords and boxes in LDS and evaluates its pixels, the
// row pass of the free set being computed from the chords where a pixel
// inside the disks needs it.  Otherwise one item does the whole slice with
// the chords and the row pass in global memory.
__device__ inline void plane_item(const SceneDev &sc, int s, int tile,
                                  int4 *lds, int lds_cap) {
  const int K = sc.K, nx = sc.nx, ny = sc.ny;
  const int64_t npx = (int64_t)nx * ny;
  const int64_t *xy = sc.xy + (int64_t)s * K * 2;
  int4 *box = lds;
  const bool in_lds = chords_in_lds(K, ny, lds_cap);
  if (in_lds) {
    int2 *lch = reinterpret_cast<int2 *>(lds + K);
    for (int t = threadIdx.x; t < K; t += blockDim.x)
      box[t] = disk_box(xy[2 * t], xy[2 * t + 1], sc.R, nx, ny);
    for (int t = threadIdx.x; t < K * ny; t += blockDim.x) {
      const int k = t / ny, j = t - k * ny;
      lch[t] = disk_chord(xy[2 * k], xy[2 * k + 1], sc.R, nx, j);
    }
    __syncthreads();
    const LdsTab ch{lch};
    int32_t *P = sc.P + (int64_t)s * npx;
    const int64_t p1 = min(npx, (int64_t)(tile + 1) * kPlaneTile);
    for (int64_t p = (int64_t)tile * kPlaneTile + threadIdx.x; p < p1;
         p += blockDim.x) {
      const int j = (int)(p / nx), i = (int)(p - (int64_t)j * nx);
      P[p] = plane_value_rf(ch, box, RowFreeChords<LdsTab>{ch, K, ny, nx, i},
                            K, nx, ny, i, j);
    }
    return;
  }
  int2 *gch = sc.chords + (int64_t)s * K * ny;
  for (int t = threadIdx.x; t < K; t += blockDim.x)
    box[t] = disk_box(xy[2 * t], xy[2 * t + 1], sc.R, nx, ny);
  for (int t = threadIdx.x; t < K * ny; t += blockDim.x) {
    const int k = t / ny, j = t - k * ny;
    gch[t] = disk_chord(xy[2 * k], xy[2 * k + 1], sc.R, nx, j);
  }
  __threadfence();
  __syncthreads();
  int32_t *f1 = sc.F1 + (int64_t)s * npx;
  int32_t *P = sc.P + (int64_t)s * npx;
  {
    const GlobalTab ch{gch};
    for (int64_t p = threadIdx.x; p < npx; p += blockDim.x) {
      const int j = (int)(p / nx), i = (int)(p - (int64_t)j * nx);
      f1[p] = row_free_dist(ch, K, ny, nx, j, i);
    }
    __threadfence();
    __syncthreads();
    for (int64_t p = threadIdx.x; p < npx; p += blockDim.x) {
      const int j = (int)(p / nx), i = (int)(p - (int64_t)j * nx);
      P[p] = plane_value(ch, box, f1 + i, K, nx, ny, i, j);
    }
  }
}

// Composite of `count` consecutive voxels from v0 (VEC voxels per lane and
// step) for slices [s0, s1).
template <int VEC>
__device__ inline void composite_chunk(const SceneDev &sc, uint32_t v0,
                                uint32_t count, int s0, int s1) {
  const uint32_t nx = sc.nx, ny = sc.ny, V = sc.V;
  const size_t plane = (size_t)nx * ny;
  const uint32_t end = min(V, v0 + count);
  for (uint32_t v = v0 + threadIdx.x * VEC; v < end; v += blockDim.x * VEC) {
    const uint32_t row = v / nx;
    const uint32_t i = v - row * nx;
    const uint32_t k = row / ny;
    const uint32_t j = row - k * ny;
    const int kk = (int)k;
    const int dzo = kk > sc.Kt ? kk - sc.Kt : 0;
    const int dz2o = dzo * dzo;
    const bool zin = kk <= sc.Kt;
    const int32_t dz2i =
        sc.has_above ? (sc.Kt + 1 - kk) * (sc.Kt + 1 - kk) : INT32_MAX;
    const int32_t *prow = sc.P + (size_t)j * nx + i;
    if constexpr (VEC == 4) {
      const int4 s4 = *reinterpret_cast<const int4 *>(sc.S + v);
      for (int sl = s0; sl < s1; ++sl) {
        const int4 p4 = *reinterpret_cast<const int4 *>(prow + sl * plane);
        int4 c;
        c.x = min(s4.x, human_value(p4.x, dz2o, zin, dz2i));
        c.y = min(s4.y, human_value(p4.y, dz2o, zin, dz2i));
        c.z = min(s4.z, human_value(p4.z, dz2o, zin, dz2i));
        c.w = min(s4.w, human_value(p4.w, dz2o, zin, dz2i));
        const size_t o = (size_t)sl * V + v;
        if (sc.oc) *reinterpret_cast<int4 *>(sc.oc + o) = c;
        if (sc.of) {
          float4 f;
          f.x = ssq_to_metres(c.x, sc.hf);
          f.y = ssq_to_metres(c.y, sc.hf);
          f.z = ssq_to_metres(c.z, sc.hf);
          f.w = ssq_to_metres(c.w, sc.hf);
          *reinterpret_cast<float4 *>(sc.of + o) = f;
        }
      }
    } else {
      const int32_t s = sc.S[v];
      for (int sl = s0; sl < s1; ++sl) {
        const int32_t c =
            min(s, human_value(prow[sl * plane], dz2o, zin, dz2i));
        const size_t o = (size_t)sl * V + v;
        if (sc.oc) sc.oc[o] = c;
        if (sc.of) sc.of[o] = ssq_to_metres(c, sc.hf);
      }
    }
  }
}

// Persistent workers.  A fixed grid strides over a list of work items;
// nothing waits on anything, so every workgroup runs a bounded number of
// bounded items.  The planar items of a batch are run by one launch and
// its composite items by the next on the same stream, so stream order is
// the only dependency between them.
__device__ inline void batch_planes(const SceneDev *__restrict__ scenes,
                                    const int4 *__restrict__ items,
                                    int n_items, int lds_cap, int4 *lds) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    plane_item(scenes[w.y], w.z, w.w, lds, lds_cap);
    __syncthreads();  // the next item reuses the LDS
  }
}

__device__ inline void batch_composites(const SceneDev *__restrict__ scenes,
                                        const int4 *__restrict__ items,
                                        int n_items, int G,
                                        uint32_t chunk_voxels) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    const SceneDev sc = scenes[w.y];
    const int s1 = min(sc.n, w.z + G);
    if (sc.vec4)
      composite_chunk<4>(sc, (uint32_t)w.w, chunk_voxels, w.z, s1);
    else
      composite_chunk<1>(sc, (uint32_t)w.w, chunk_voxels, w.z, s1);
  }
}

}  // namespace pcsdf
