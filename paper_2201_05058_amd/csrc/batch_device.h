// Device side of the batched composite (see batch.hip): scene table entry,
// planar-field item, composite chunk and the worker loops.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "composite_device.h"
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
  int nx, ny, nz, n, K, Kt, has_above;
  int vec, gather;  // pack shape of the composite (composite_shape)
  float hf;
  uint32_t item0;   // first composite item of the scene
  uint32_t items;   // its composite items: slice groups x chunks
  uint32_t chunks;  // voxel chunks per slice group
};

// Composite items are numbered scene by scene, each scene's count padded
// to a multiple of kItemGroup, so that one table entry per kItemGroup
// items names the scene (padding items do nothing).
constexpr int kItemGroupShift = 6;
constexpr int kItemGroup = 1 << kItemGroupShift;

// One scene-table entry, read field by field through the constant address
// space: the compiler takes a pointer loaded from there to be global, so
// every access through it is a global instruction rather than a flat one
// (a wait for a flat access cannot be counted in order and so waits for
// all outstanding loads and stores).  A whole-struct copy would lose the
// address space.
__device__ __forceinline__ SceneDev load_scene(const SceneDev *scenes, int q) {
#if defined(__clang__)
  typedef __attribute__((address_space(4))) const SceneDev ConstScene;
#else  // a host compiler building the device code for CPU tests
  typedef const SceneDev ConstScene;
#endif
  ConstScene *c = (ConstScene *)(scenes + q);
  SceneDev d;
  d.S = c->S;
  d.oc = c->oc;
  d.of = c->of;
  d.xy = c->xy;
  d.chords = c->chords;
  d.P = c->P;
  d.F1 = c->F1;
  d.R = c->R;
  d.V = c->V;
  d.nx = c->nx;
  d.ny = c->ny;
  d.nz = c->nz;
  d.n = c->n;
  d.K = c->K;
  d.Kt = c->Kt;
  d.has_above = c->has_above;
  d.vec = c->vec;
  d.gather = c->gather;
  d.hf = c->hf;
  d.item0 = c->item0;
  d.items = c->items;
  d.chunks = c->chunks;
  return d;
}

constexpr int kItemPlane = 0;
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

// Composite of `count` consecutive voxels from v0 (VEC voxels per lane)
// for slices [s0, s1); v0 is a multiple of the chunk size, itself a
// multiple of 4.  Each lane runs the same epilogue as the single-scene
// kernel; with the tuned chunk of 256 lanes x 4 voxels a lane handles one
// pack and exits.  (A loop that loads the next step's data ahead of the
// current stores was measured slower for these short item lengths, and
// persistent grids slower than one workgroup per item.)
template <int VEC, bool kGather, bool kSsq, bool kSdf>
__device__ inline void composite_chunk(const SceneDev &sc, uint32_t v0,
                                       uint32_t count, int s0, int s1) {
  const uint32_t plane = (uint32_t)sc.nx * (uint32_t)sc.ny;
  const uint32_t end = min(sc.V, v0 + count);
  for (uint32_t v = v0 + threadIdx.x * VEC; v < end; v += blockDim.x * VEC)
    composite_pack<VEC, kGather, kSsq, kSdf>(sc.S, sc.P, nullptr, sc.oc,
                                             sc.of, plane, sc.V, v, s0, s1,
                                             sc.Kt, sc.has_above, sc.hf);
}

template <int VEC, bool kGather>
__device__ inline void composite_chunk_any(const SceneDev &sc, uint32_t v0,
                                           uint32_t count, int s0, int s1) {
  if (sc.oc && sc.of)
    composite_chunk<VEC, kGather, true, true>(sc, v0, count, s0, s1);
  else if (sc.oc)
    composite_chunk<VEC, kGather, true, false>(sc, v0, count, s0, s1);
  else
    composite_chunk<VEC, kGather, false, true>(sc, v0, count, s0, s1);
}

// Workers.  A grid strides over a list of work items; nothing waits on
// anything, so every workgroup runs a bounded number of bounded items.
// The planar items of a batch are run by one launch and its composite
// items by the next on the same stream, so stream order is the only
// dependency between them.
__device__ inline void batch_planes(const SceneDev *__restrict__ scenes,
                                    const int4 *__restrict__ items,
                                    int n_items, int lds_cap, int4 *lds) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    plane_item(load_scene(scenes, w.y), w.z, w.w, lds, lds_cap);
    __syncthreads();  // the next item reuses the LDS
  }
}

// Composite item `it` belongs to scene q = scene_of[it / kItemGroup]; it
// is slice group (it - item0) / chunks and voxel chunk (it - item0) %
// chunks of that scene, or padding when it - item0 >= items.
__device__ inline void batch_composites(const SceneDev *__restrict__ scenes,
                                        const int32_t *__restrict__ scene_of,
                                        uint32_t total, int G,
                                        uint32_t chunk_voxels) {
  for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
    const SceneDev sc = load_scene(scenes, scene_of[it >> kItemGroupShift]);
    const uint32_t local = it - sc.item0;
    if (local >= sc.items) continue;
    const uint32_t sg = local / sc.chunks;
    const uint32_t v0 = (local - sg * sc.chunks) * chunk_voxels;
    const int s0 = (int)sg * G;
    const int s1 = min(sc.n, s0 + G);
    if (sc.vec == 4 && !sc.gather)
      composite_chunk_any<4, false>(sc, v0, chunk_voxels, s0, s1);
    else if (sc.vec == 4)
      composite_chunk_any<4, true>(sc, v0, chunk_voxels, s0, s1);
    else if (sc.vec == 2 && !sc.gather)
      composite_chunk_any<2, false>(sc, v0, chunk_voxels, s0, s1);
    else if (sc.vec == 2)
      composite_chunk_any<2, true>(sc, v0, chunk_voxels, s0, s1);
    else
      composite_chunk_any<1, false>(sc, v0, chunk_voxels, s0, s1);
  }
}

}  // namespace pcsdf
