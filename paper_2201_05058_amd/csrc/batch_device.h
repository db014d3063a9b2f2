// Device side of the batched composite (see batch.hip): scene table entry,
// planar-field item, composite chunk and the persistent worker loop.
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
  int nx, ny, nz, n, K, Kt, has_above, vec;  // vec: 4, 2 or 1 voxels
  float hf;
  int pad[2];
};

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
  d.hf = c->hf;
  d.pad[0] = d.pad[1] = 0;
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

// Composite of `count` consecutive voxels from v0 (VEC voxels per lane and
// step) for slices [s0, s1).  v0 is a multiple of the chunk size, itself a
// multiple of 4.
//
// A persistent wave runs many (voxels, slice) steps back to back, and on
// this GPU a wait for a load also waits for every store issued before it.
// So each step's loads (static and planar packs) are issued before the
// previous step's stores: the wait for them then covers only the loads.
template <int VEC>
struct CompositeStep {
  typename Pack<VEC>::I s, p;
  int32_t dz2o, dz2i;
  bool zin;
};

template <int VEC>
__device__ __forceinline__ void load_step(const SceneDev &sc, uint32_t plane,
                                          uint32_t v, int sl,
                                          CompositeStep<VEC> &st) {
  const uint32_t k = v / plane;
  const uint32_t pix = v - k * plane;
  const int kk = (int)k;
  const int dzo = kk > sc.Kt ? kk - sc.Kt : 0;
  st.dz2o = dzo * dzo;
  st.zin = kk <= sc.Kt;
  st.dz2i = sc.has_above ? (sc.Kt + 1 - kk) * (sc.Kt + 1 - kk) : INT32_MAX;
  st.s = load_i32<VEC>(sc.S + v);
  st.p = load_i32<VEC>(sc.P + (size_t)sl * plane + pix);
}

template <int VEC, bool kSsq, bool kSdf>
__device__ inline void composite_chunk(const SceneDev &sc, uint32_t v0,
                                       uint32_t count, int s0, int s1) {
  const uint32_t plane = (uint32_t)sc.nx * (uint32_t)sc.ny;
  const uint32_t end = min(sc.V, v0 + count);
  const uint32_t stride = blockDim.x * VEC;
  uint32_t v = v0 + threadIdx.x * VEC;
  if (v >= end) return;
  int sl = s0;
  CompositeStep<VEC> cur;
  load_step<VEC>(sc, plane, v, sl, cur);
  // Make the first step's loads complete here, so that inside the loop
  // the current step's data is known to be in registers and no wait there
  // covers the previous stores.
  wait_for<VEC>(cur.s);
  wait_for<VEC>(cur.p);
  for (;;) {
    uint32_t vn = v;
    int sn = sl + 1;
    if (sn == s1) {
      sn = s0;
      vn = v + stride;
    }
    const bool more = vn < end;
    // Unconditional, so that the wait for these loads is counted exactly
    // (a load on one side of a branch makes the wait for the current
    // step's data a wait for everything); past the end it re-reads the
    // current step's (valid) addresses.
    CompositeStep<VEC> nxt;
    load_step<VEC>(sc, plane, more ? vn : v, more ? sn : sl, nxt);
    typename Pack<VEC>::I c;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      c[e] = min(cur.s[e],
                 human_value(cur.p[e], cur.dz2o, cur.zin, cur.dz2i));
    const size_t o = (size_t)sl * sc.V + v;
    if (kSsq) store_i32<VEC>(sc.oc + o, c);
    if (kSdf) {
      typename Pack<VEC>::F f;
#pragma unroll
      for (int e = 0; e < VEC; ++e) f[e] = ssq_to_metres(c[e], sc.hf);
      store_f32<VEC>(sc.of + o, f);
    }
    if (!more) break;
    v = vn;
    sl = sn;
    cur = nxt;
  }
}

template <int VEC>
__device__ inline void composite_chunk_any(const SceneDev &sc, uint32_t v0,
                                           uint32_t count, int s0, int s1) {
  if (sc.oc && sc.of)
    composite_chunk<VEC, true, true>(sc, v0, count, s0, s1);
  else if (sc.oc)
    composite_chunk<VEC, true, false>(sc, v0, count, s0, s1);
  else
    composite_chunk<VEC, false, true>(sc, v0, count, s0, s1);
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

// Composite items are not listed: item `it` of scene q (tile_start[q] <= it
// < tile_start[q + 1]) is slice group (it - tile_start[q]) / chunks and
// voxel chunk (it - tile_start[q]) % chunks of that scene, chunks =
// ceil(V / chunk_voxels).  A workgroup finds the scene of its first item
// by binary search over the n_scenes + 1 prefix sums and walks forward
// from there (its items increase).
__device__ inline void batch_composites(const SceneDev *__restrict__ scenes,
                                        const uint32_t *__restrict__ tile_start,
                                        int n_scenes, int G,
                                        uint32_t chunk_voxels) {
  const uint32_t total = tile_start[n_scenes];
  uint32_t it = blockIdx.x;
  if (it >= total) return;
  int lo = 0, hi = n_scenes - 1;  // last q with tile_start[q] <= it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  int q = lo;
  for (; it < total; it += gridDim.x) {
    while (tile_start[q + 1] <= it) ++q;
    const SceneDev sc = load_scene(scenes, q);
    const uint32_t chunks = (sc.V + chunk_voxels - 1) / chunk_voxels;
    const uint32_t local = it - tile_start[q];
    const uint32_t sg = local / chunks;
    const uint32_t v0 = (local - sg * chunks) * chunk_voxels;
    const int s0 = (int)sg * G;
    const int s1 = min(sc.n, s0 + G);
    if (sc.vec == 4)
      composite_chunk_any<4>(sc, v0, chunk_voxels, s0, s1);
    else if (sc.vec == 2)
      composite_chunk_any<2>(sc, v0, chunk_voxels, s0, s1);
    else
      composite_chunk_any<1>(sc, v0, chunk_voxels, s0, s1);
  }
}

}  // namespace pcsdf
