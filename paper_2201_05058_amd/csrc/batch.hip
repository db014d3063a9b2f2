// Batched predicted composite fields: many scenes of uneven grid sizes and
// slice counts in two launches, optionally captured in one hipGraph with
// the upload of their parameters.
//
// Work list.  The planar-field items (scene, slice, pixel tile) of all
// scenes are listed, scene-major, and a persistent grid strides over them.
// The composite items (scene, slice group, voxel chunk) are numbered scene
// by scene, each scene's count padded to a multiple of 64 so that one
// table entry per 64 items names the scene; the second launch covers them
// either with a persistent grid (a given number of workgroups per CU) or
// with one workgroup per item.  The only dependency (a composite item reads its
// slices' planes) is the stream order of the two launches.  No workgroup
// ever waits on another, so every workgroup runs a bounded number of
// bounded items.  The launch shape (slices per composite item, voxels per
// item, persistent workgroups per CU or none) comes from the handle's
// tuning, which the autotuner below fills by timing candidates on the
// caller's inputs.
//
// The device code lives in batch_device.h and the planning in
// batch_plan.h, so that both can also be compiled for the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch_device.h"
#include "batch_plan.h"
#include "internal.h"

namespace pcsdf {

__global__ __launch_bounds__(256) void k_batch_planes(
    const SceneDev *__restrict__ scenes, const int4 *__restrict__ items,
    int n_items, int lds_cap) {
  extern __shared__ int4 lds[];
  batch_planes(scenes, items, n_items, lds_cap, lds);
}

__global__ __launch_bounds__(256) void k_batch_composites(
    const SceneDev *__restrict__ scenes, const int32_t *__restrict__ scene_of,
    uint32_t total, int G, uint32_t chunk_voxels) {
  batch_composites(scenes, scene_of, total, G, chunk_voxels);
}

// -------------------------------------------------------------- host side

// Enqueues the planar and the composite launch (parameters already
// uploaded to pbase).
static int enqueue_batch(Handle *h, const BatchPlan &bp, char *pbase,
                         hipStream_t s) {
  const ParamLayout L = param_layout(bp);
  const SceneDev *scenes = reinterpret_cast<const SceneDev *>(pbase);
  const int32_t *scene_of =
      reinterpret_cast<const int32_t *>(pbase + L.groups);
  const int4 *items = reinterpret_cast<const int4 *>(pbase + L.items);
  const int np = (int)bp.items.size();
  const int64_t nc = bp.composite_items;
  if (np > 0) {
    hipLaunchKernelGGL(k_batch_planes, dim3(std::min(np, bp.blocks)),
                       dim3(256), (size_t)bp.lds_cap, s, scenes, items, np,
                       bp.lds_cap);
    int rc = check_launch(h, "batch_planes");
    if (rc) return rc;
  }
  if (nc > 0) {
    const int64_t grid = bp.blocks_cu > 0 ? std::min<int64_t>(nc, bp.blocks_cu)
                                          : nc;
    hipLaunchKernelGGL(k_batch_composites, dim3((unsigned)grid), dim3(256), 0,
                       s, scenes, scene_of, bp.composite_items, bp.G,
                       bp.chunk_voxels);
    return check_launch(h, "batch_composites");
  }
  return PCSDF_OK;
}

static int device_cus(Handle *h, int *n_cu) {
  int v = 0;
  hipError_t e =
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount,
                            h->device);
  if (e != hipSuccess || v <= 0)
    return fail(h, PCSDF_ERR_HIP, "cannot read the compute unit count");
  *n_cu = v;
  return PCSDF_OK;
}

// Plans, uploads and enqueues one batch through the handle's buffers.
static int run_batch(Handle *h, int n_scenes, const pcsdf_scene *scenes,
                     const pcsdf_tuning &tu, hipStream_t s) {
  int rc;
  if ((rc = bind_device(h))) return rc;
  int n_cu = 0;
  if ((rc = device_cus(h, &n_cu))) return rc;
  BatchPlan bp;
  if ((rc = plan_batch(h, n_scenes, scenes, tu, n_cu, &bp))) return rc;
  std::vector<char> &host = h->batch_host;
  if ((rc = ensure_buffer(h, h->batch_params, param_layout(bp).total, s)))
    return rc;
  if ((rc = ensure_buffer(h, h->batch_scratch, plan_scratch(bp), s)))
    return rc;
  char *pbase = reinterpret_cast<char *>(h->batch_params.ptr);
  bind_plan(&bp, scenes, pbase, reinterpret_cast<char *>(h->batch_scratch.ptr),
            &host);
  if ((rc = acquire_staging(h, host.size()))) return rc;
  std::memcpy(h->pinned, host.data(), host.size());
  if (hipMemcpyAsync(pbase, h->pinned, host.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return fail(h, PCSDF_ERR_HIP, "upload of the batch parameters failed");
  if ((rc = release_staging(h, s))) return rc;
  ProfScope ps(h, PCSDF_KERNEL_BATCH, s);
  return enqueue_batch(h, bp, pbase, s);
}

}  // namespace pcsdf

using namespace pcsdf;

struct pcsdf_batch_graph {
  Handle *h = nullptr;
  BatchPlan plan;
  std::vector<pcsdf_scene> scenes;
  DevBuf params, scratch;
  void *pinned = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
};

extern "C" int pcsdf_predicted_composite_sdf_batch(pcsdf_handle *hp,
                                                   int32_t n_scenes,
                                                   const pcsdf_scene *scenes,
                                                   void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  h->err.clear();
  return run_batch(h, n_scenes, scenes, h->tuning,
                   reinterpret_cast<hipStream_t>(stream));
}

static int graph_fail(pcsdf_batch_graph *g, int code, const std::string &m) {
  return fail(g->h, code, m);
}

extern "C" void pcsdf_batch_graph_destroy(pcsdf_batch_graph *g) {
  if (!g) return;
  if (g->pending && g->done) (void)hipEventSynchronize(g->done);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->done) (void)hipEventDestroy(g->done);
  DevBuf *bufs[] = {&g->params, &g->scratch};
  bool any = false;
  for (DevBuf *b : bufs) any = any || b->ptr;
  if (any) (void)hipDeviceSynchronize();
  for (DevBuf *b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  if (g->pinned) (void)hipHostFree(g->pinned);
  delete g;
}

extern "C" int pcsdf_batch_graph_create(pcsdf_handle *hp, int32_t n_scenes,
                                        const pcsdf_scene *scenes,
                                        void *stream,
                                        pcsdf_batch_graph **out) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!out) return fail(h, PCSDF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  h->err.clear();
  (void)stream;  // capture runs on a private stream
  int rc;
  if ((rc = bind_device(h))) return rc;
  int n_cu = 0;
  if ((rc = device_cus(h, &n_cu))) return rc;
  pcsdf_batch_graph *g = new (std::nothrow) pcsdf_batch_graph();
  if (!g) return fail(h, PCSDF_ERR_OOM, "graph object allocation failed");
  g->h = h;
  if ((rc = plan_batch(h, n_scenes, scenes, h->tuning, n_cu, &g->plan))) {
    delete g;
    return rc;
  }
  g->scenes.assign(scenes, scenes + n_scenes);
  std::vector<char> host;
  hipStream_t cap = nullptr;
  if ((rc = ensure_buffer(h, g->params, param_layout(g->plan).total,
                          nullptr)) ||
      (rc = ensure_buffer(h, g->scratch, plan_scratch(g->plan), nullptr))) {
    pcsdf_batch_graph_destroy(g);
    return rc;
  }
  char *pbase = reinterpret_cast<char *>(g->params.ptr);
  bind_plan(&g->plan, scenes, pbase, reinterpret_cast<char *>(g->scratch.ptr),
            &host);
  if (hipHostMalloc(&g->pinned, host.size(), hipHostMallocDefault) !=
      hipSuccess) {
    g->pinned = nullptr;
    pcsdf_batch_graph_destroy(g);
    return fail(h, PCSDF_ERR_OOM, "pinned staging allocation failed");
  }
  std::memcpy(g->pinned, host.data(), host.size());
  if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
    pcsdf_batch_graph_destroy(g);
    return fail(h, PCSDF_ERR_HIP, "graph stream/event creation failed");
  }
  bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) ==
            hipSuccess;
  if (ok) {
    ok = hipMemcpyAsync(pbase, g->pinned, host.size(), hipMemcpyHostToDevice,
                        cap) == hipSuccess;
    if (ok) ok = enqueue_batch(h, g->plan, pbase, cap) == PCSDF_OK;
    hipGraph_t graph = nullptr;
    const bool ended = hipStreamEndCapture(cap, &graph) == hipSuccess;
    ok = ok && ended && graph;
    g->graph = graph;
  }
  if (ok)
    ok = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) ==
         hipSuccess;
  (void)hipStreamDestroy(cap);
  if (!ok) {
    (void)hipGetLastError();
    pcsdf_batch_graph_destroy(g);
    return fail(h, PCSDF_ERR_HIP, "capturing the batch graph failed");
  }
  *out = g;
  return PCSDF_OK;
}

extern "C" int pcsdf_batch_graph_set_positions(pcsdf_batch_graph *g,
                                               int32_t scene,
                                               const double *human_xy_host) {
  if (!g) return PCSDF_ERR_INVALID_ARG;
  Handle *h = g->h;
  if (scene < 0 || scene >= (int32_t)g->scenes.size())
    return graph_fail(g, PCSDF_ERR_INVALID_ARG, "scene index out of range");
  const pcsdf_scene &sc = g->scenes[scene];
  const SceneDev &d = g->plan.scenes[scene];
  if (d.K == 0) return PCSDF_OK;
  if (!human_xy_host)
    return graph_fail(g, PCSDF_ERR_INVALID_ARG, "human_xy_host is NULL");
  std::vector<int64_t> tmp((size_t)d.n * d.K * 2);
  for (int64_t t = 0; t < (int64_t)d.n * d.K; ++t) {
    if (!fixed(human_xy_host[2 * t], sc.grid.origin_m[0], sc.grid.voxel_m,
               &tmp[2 * t]) ||
        !fixed(human_xy_host[2 * t + 1], sc.grid.origin_m[1], sc.grid.voxel_m,
               &tmp[2 * t + 1]))
      return graph_fail(g, PCSDF_ERR_NUMERIC,
                        "human position non-finite or out of range");
  }
  if (g->pending) {
    if (hipEventSynchronize(g->done) != hipSuccess)
      return graph_fail(g, PCSDF_ERR_HIP, "waiting for the graph failed");
    g->pending = false;
  }
  const size_t off_xy = param_layout(g->plan).xy;
  std::memcpy(static_cast<char *>(g->pinned) + off_xy +
                  g->plan.xy_off[scene] * 8,
              tmp.data(), tmp.size() * 8);
  (void)h;
  return PCSDF_OK;
}

extern "C" int pcsdf_batch_graph_launch(pcsdf_batch_graph *g, void *stream) {
  if (!g) return PCSDF_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(g->h, PCSDF_KERNEL_BATCH, s);
  if (hipGraphLaunch(g->exec, s) != hipSuccess)
    return graph_fail(g, PCSDF_ERR_HIP, "hipGraphLaunch failed");
  ps.stop();
  if (hipEventRecord(g->done, s) != hipSuccess)
    return graph_fail(g, PCSDF_ERR_HIP, "hipEventRecord failed");
  g->pending = true;
  return PCSDF_OK;
}

// ---------------------------------------------------------------- tuning

namespace {

// Milliseconds per call of the timed regions `id` inside `fn` (HIP events
// on the stream around the kernels alone, so that host work between calls
// does not count), over reps calls after one warm-up call; -1 on error.
// The handle's profiling state and totals are left as they were.
template <class F>
double kernel_ms(Handle *h, int id, hipStream_t s, int reps, F fn) {
  if (drain_profile(h)) return -1.0;
  const uint32_t mask = h->prof_mask;
  double ms[PCSDF_KERNEL_COUNT];
  int64_t n[PCSDF_KERNEL_COUNT];
  std::memcpy(ms, h->prof_ms, sizeof ms);
  std::memcpy(n, h->prof_n, sizeof n);
  double out = -1.0;
  h->prof_mask = 0;
  if (fn() == PCSDF_OK && hipStreamSynchronize(s) == hipSuccess) {
    h->prof_mask = 1u << id;
    const double before = h->prof_ms[id];
    int rc = PCSDF_OK;
    for (int r = 0; r < reps && rc == PCSDF_OK; ++r) rc = fn();
    if (rc == PCSDF_OK && hipStreamSynchronize(s) == hipSuccess &&
        drain_profile(h) == PCSDF_OK)
      out = (h->prof_ms[id] - before) / reps;
  }
  h->prof_mask = mask;
  std::memcpy(h->prof_ms, ms, sizeof ms);
  std::memcpy(h->prof_n, n, sizeof n);
  return out;
}

}  // namespace

extern "C" int pcsdf_autotune_batch(pcsdf_handle *hp, int32_t n_scenes,
                                    const pcsdf_scene *scenes, void *stream,
                                    int32_t reps, pcsdf_tuning *best,
                                    double *best_ms) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!best || !best_ms || reps < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "best, best_ms and reps >= 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const pcsdf_tuning base = h->tuning;
  pcsdf_tuning win = base;
  double win_ms = -1.0;
  const int Gs[] = {1, 2, 4};
  const int Cs[] = {256, 1024, 4096};
  const int Bs[] = {0, 4, 8, 16};  // 0: one workgroup per composite item
  for (int G : Gs)
    for (int C : Cs)
      for (int B : Bs) {
        pcsdf_tuning t = base;
        t.batch_slices_per_item = G;
        t.batch_chunk_quads = C;
        t.batch_blocks_per_cu = B;
        const double ms = kernel_ms(h, PCSDF_KERNEL_BATCH, s, reps, [&] {
          return run_batch(h, n_scenes, scenes, t, s);
        });
        if (ms < 0) {
          h->tuning = base;
          return h->err.empty() ? fail(h, PCSDF_ERR_HIP, "tuning run failed")
                                : PCSDF_ERR_HIP;
        }
        if (win_ms < 0 || ms < win_ms) {
          win_ms = ms;
          win = t;
        }
      }
  h->tuning = win;
  // leave the outputs as the tuned configuration writes them
  int rc = run_batch(h, n_scenes, scenes, win, s);
  if (rc) return rc;
  *best = win;
  *best_ms = win_ms;
  return PCSDF_OK;
}

extern "C" int pcsdf_autotune_composite(pcsdf_handle *hp,
                                        const pcsdf_scene *sc, void *stream,
                                        int32_t reps, pcsdf_tuning *best,
                                        double *best_ms) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!sc || !best || !best_ms || reps < 1)
    return fail(h, PCSDF_ERR_INVALID_ARG, "scene, best, best_ms, reps >= 1");
  const pcsdf_tuning base = h->tuning;
  pcsdf_tuning win = base;
  double win_ms = -1.0;
  const int n = sc->n_slices;
  // slice groups in both block orders
  constexpr int kG = 7, kCand = 2 * kG;
  const int Gs[kG] = {1, 2, 3, 4, 5, 10, n};
  double best_of[kCand];
  for (int c = 0; c < kCand; ++c) best_of[c] = -1.0;
  // Three interleaved rounds over the candidates, each keeping its fastest
  // round: the candidates neighbouring ones differ by a few per cent, less
  // than the drift of a single pass.
  for (int round = 0; round < 3; ++round)
    for (int c = 0; c < kCand; ++c) {
      const int G = Gs[c % kG];
      bool seen = false;  // n may repeat an earlier candidate
      for (int e = 0; e < c % kG; ++e) seen = seen || Gs[e] == G;
      if (G < 1 || G > n || seen) continue;
      h->tuning = base;
      h->tuning.composite_slices_per_block = G;
      h->tuning.composite_order = c / kG;
      // the composite kernel alone: the slice group and the block order
      // change nothing else, and a call's wall time can be the host's
      const double ms = kernel_ms(
          h, PCSDF_KERNEL_COMPOSITE, reinterpret_cast<hipStream_t>(stream),
          reps, [&] {
            return pcsdf_predicted_composite_sdf(
                hp, &sc->grid, sc->static_ssq_dev, sc->n_slices,
                sc->n_humans, sc->human_xy_host, sc->radius_m, sc->height_m,
                sc->out_ssq_dev, sc->out_sdf_dev, stream);
          });
      if (ms < 0) {
        h->tuning = base;
        return PCSDF_ERR_HIP;
      }
      if (best_of[c] < 0 || ms < best_of[c]) best_of[c] = ms;
    }
  for (int c = 0; c < kCand; ++c) {
    if (best_of[c] < 0) continue;
    if (win_ms < 0 || best_of[c] < win_ms) {
      win_ms = best_of[c];
      win = base;
      win.composite_slices_per_block = Gs[c % kG];
      win.composite_order = c / kG;
    }
  }
  h->tuning = win;
  int rc = pcsdf_predicted_composite_sdf(
      hp, &sc->grid, sc->static_ssq_dev, sc->n_slices, sc->n_humans,
      sc->human_xy_host, sc->radius_m, sc->height_m, sc->out_ssq_dev,
      sc->out_sdf_dev, stream);
  if (rc) return rc;
  *best = win;
  *best_ms = win_ms;
  return PCSDF_OK;
}
