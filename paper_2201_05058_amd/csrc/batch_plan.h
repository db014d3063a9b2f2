// Host side of the batched composite: validation of the scenes, the work
// list and the layout of the parameter block (see batch.hip).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "batch_device.h"
#include "internal.h"

namespace pcsdf {

struct BatchPlan {
  std::vector<SceneDev> scenes;
  std::vector<int4> items;          // planar items
  std::vector<int32_t> scene_of;  // scene of each group of kItemGroup items
  uint32_t composite_items = 0;   // including padding
  std::vector<int64_t> xy;
  std::vector<size_t> xy_off;  // per scene, in int64 units
  int lds_cap = 0;
  int G = 2;
  uint32_t chunk_voxels = 0;
  int blocks = 0;     // persistent grid of the planar launch
  int blocks_cu = 0;  // persistent composite grid (0: one item per block)
};

inline bool fixed(double p, double o, double h, int64_t *out) {
  double t = p - o;
  t = t / h;
  t = t * 65536.0;
  if (!std::isfinite(t) || std::fabs(t) >= 4611686018427387904.0) return false;
  *out = (int64_t)std::nearbyint(t);
  return true;
}

// Validates the scenes and fills everything but device addresses.
inline int plan_batch(Handle *h, int n_scenes, const pcsdf_scene *scenes,
                      const pcsdf_tuning &tu, int n_cu, BatchPlan *bp) {
  if (n_scenes < 1 || !scenes)
    return fail(h, PCSDF_ERR_INVALID_ARG, "need at least one scene");
  bp->G = tu.batch_slices_per_item > 0 ? tu.batch_slices_per_item : 4;
  const int quads = tu.batch_chunk_quads > 0 ? tu.batch_chunk_quads : 256;
  bp->chunk_voxels = (uint32_t)quads * 4;
  bp->blocks = n_cu * (tu.batch_blocks_per_cu > 0 ? tu.batch_blocks_per_cu
                                                   : 8);
  bp->blocks_cu = tu.batch_blocks_per_cu > 0 ? n_cu * tu.batch_blocks_per_cu
                                             : 0;
  bp->scenes.resize(n_scenes);
  bp->xy_off.resize(n_scenes);
  bp->xy.clear();
  int lds_need = 0;
  for (int q = 0; q < n_scenes; ++q) {
    const pcsdf_scene &in = scenes[q];
    const std::string tag = "scene " + std::to_string(q) + ": ";
    int rc = check_grid(h, &in.grid);
    if (rc) return fail(h, rc, tag + h->err);
    if (!in.static_ssq_dev || (!in.out_ssq_dev && !in.out_sdf_dev))
      return fail(h, PCSDF_ERR_INVALID_ARG,
                  tag + "inline field and one output are required");
    if (in.n_slices < 1 || in.n_humans < 0 || in.n_humans > kMaxHumans ||
        (in.n_humans > 0 && !in.human_xy_host))
      return fail(h, PCSDF_ERR_INVALID_ARG, tag + "bad slice/human counts");
    if (((uintptr_t)in.static_ssq_dev | (uintptr_t)in.out_ssq_dev |
         (uintptr_t)in.out_sdf_dev) & 3)
      return fail(h, PCSDF_ERR_ALIGN, tag + "buffers must be 4-byte aligned");
    const double hv = in.grid.voxel_m;
    int64_t R, Hq;
    if (!std::isfinite(in.radius_m) || in.radius_m < 0 ||
        !std::isfinite(in.height_m) || in.height_m < 0 ||
        !fixed(in.radius_m, 0.0, hv, &R) || !fixed(in.height_m, 0.0, hv, &Hq) ||
        R >= (1LL << 31))
      return fail(h, PCSDF_ERR_NUMERIC, tag + "bad radius or height");
    SceneDev &d = bp->scenes[q];
    std::memset(&d, 0, sizeof(d));
    d.nx = in.grid.nx;
    d.ny = in.grid.ny;
    d.nz = in.grid.nz;
    d.n = in.n_slices;
    d.V = (uint32_t)((int64_t)d.nx * d.ny * d.nz);
    d.R = R;
    d.Kt = Hq >= 32768 ? (int)std::min<int64_t>((Hq - 32768) / 65536, d.nz - 1)
                       : -1;
    d.has_above = d.Kt + 1 <= d.nz - 1;
    d.K = (d.Kt < 0) ? 0 : in.n_humans;
    d.hf = (float)hv;
    const PackShape ps =
        composite_shape((int64_t)d.nx * d.ny, (int64_t)d.V, in.static_ssq_dev,
                        in.out_ssq_dev, in.out_sdf_dev);
    d.vec = ps.vec;
    d.gather = ps.gather;
    bp->xy_off[q] = bp->xy.size();
    for (int64_t t = 0; t < (int64_t)in.n_slices * in.n_humans; ++t) {
      int64_t X, Y;
      if (!fixed(in.human_xy_host[2 * t], in.grid.origin_m[0], hv, &X) ||
          !fixed(in.human_xy_host[2 * t + 1], in.grid.origin_m[1], hv, &Y))
        return fail(h, PCSDF_ERR_NUMERIC,
                    tag + "human position non-finite or out of range at "
                          "index " + std::to_string(t));
      if (d.K > 0) {
        bp->xy.push_back(X);
        bp->xy.push_back(Y);
      }
    }
    lds_need = std::max(lds_need, d.K * 16 + d.K * d.ny * 8);
  }
  bp->lds_cap = std::min(lds_need, 48 * 1024);
  // planar items (tiles of a slice when its chords fit in LDS),
  // scene-major; composite items are counted per scene
  bp->items.clear();
  bp->scene_of.clear();
  int64_t next = 0;
  for (int q = 0; q < n_scenes; ++q) {
    SceneDev &d = bp->scenes[q];
    const int64_t npx = (int64_t)d.nx * d.ny;
    const int tiles = chords_in_lds(d.K, d.ny, bp->lds_cap)
                          ? (int)((npx + kPlaneTile - 1) / kPlaneTile)
                          : 1;
    for (int s = 0; s < d.n; ++s)
      for (int t = 0; t < tiles; ++t)
        bp->items.push_back(make_int4(kItemPlane, q, s, t));
    const int64_t chunks =
        ((int64_t)d.V + bp->chunk_voxels - 1) / bp->chunk_voxels;
    const int64_t ct = (int64_t)((d.n + bp->G - 1) / bp->G) * chunks;
    const int64_t padded = (ct + kItemGroup - 1) / kItemGroup * kItemGroup;
    if (next + padded > (int64_t)INT32_MAX)
      return fail(h, PCSDF_ERR_DIMS,
                  "batch has more than 2^31 - 1 composite items; raise the "
                  "chunk size or split the batch");
    d.item0 = (uint32_t)next;
    d.items = (uint32_t)ct;
    d.chunks = (uint32_t)chunks;
    bp->scene_of.insert(bp->scene_of.end(), (size_t)(padded / kItemGroup), q);
    next += padded;
  }
  bp->composite_items = (uint32_t)next;
  if (bp->items.size() > (size_t)INT32_MAX)
    return fail(h, PCSDF_ERR_DIMS, "batch has too many planar items");
  return PCSDF_OK;
}

inline size_t scratch_of(const SceneDev &d) {
  const size_t plane = (size_t)d.n * d.nx * d.ny;
  return align_up((size_t)d.n * std::max(d.K, 1) * d.ny * sizeof(int2), 256) +
         2 * align_up(plane * sizeof(int32_t), 256);
}

// Byte offsets of the parameter block: scene table, scene of each group
// of composite items, planar items, centres.
struct ParamLayout {
  size_t groups, items, xy, total;
};
inline ParamLayout param_layout(const BatchPlan &bp) {
  ParamLayout L;
  L.groups = align_up(bp.scenes.size() * sizeof(SceneDev), 256);
  L.items = align_up(L.groups + bp.scene_of.size() * 4, 256);
  L.xy = align_up(L.items + bp.items.size() * 16, 256);
  L.total = L.xy + bp.xy.size() * 8;
  return L;
}

// Assigns device addresses and serialises the parameter block into
// `host`.
inline void bind_plan(BatchPlan *bp, const pcsdf_scene *scenes, char *pbase,
                      char *sbase, std::vector<char> *host) {
  const size_t n_sc = bp->scenes.size();
  const ParamLayout L = param_layout(*bp);
  size_t soff = 0;
  for (size_t q = 0; q < n_sc; ++q) {
    SceneDev &d = bp->scenes[q];
    d.S = scenes[q].static_ssq_dev;
    d.oc = scenes[q].out_ssq_dev;
    d.of = scenes[q].out_sdf_dev;
    d.xy = reinterpret_cast<const int64_t *>(pbase + L.xy) + bp->xy_off[q];
    const size_t plane = (size_t)d.n * d.nx * d.ny;
    d.chords = reinterpret_cast<int2 *>(sbase + soff);
    soff += align_up((size_t)d.n * std::max(d.K, 1) * d.ny * sizeof(int2), 256);
    d.P = reinterpret_cast<int32_t *>(sbase + soff);
    soff += align_up(plane * sizeof(int32_t), 256);
    d.F1 = reinterpret_cast<int32_t *>(sbase + soff);
    soff += align_up(plane * sizeof(int32_t), 256);
  }
  host->assign(L.total, 0);
  std::memcpy(host->data(), bp->scenes.data(), n_sc * sizeof(SceneDev));
  std::memcpy(host->data() + L.groups, bp->scene_of.data(),
              bp->scene_of.size() * 4);
  std::memcpy(host->data() + L.items, bp->items.data(),
              bp->items.size() * 16);
  if (!bp->xy.empty())
    std::memcpy(host->data() + L.xy, bp->xy.data(), bp->xy.size() * 8);
}

inline size_t plan_scratch(const BatchPlan &bp) {
  size_t t = 0;
  for (const SceneDev &d : bp.scenes) t += scratch_of(d);
  return t;
}

}  // namespace pcsdf
