// Handle, error reporting, device binding and workspace management of the
// C-ABI.  No kernels here.
#include <cmath>
#include <new>

#include "internal.h"

namespace pcsdf {

int fail(Handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

int bind_device(Handle *h) {
  int d = -1;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess)
    return fail(h, PCSDF_ERR_HIP,
                std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (h->device < 0) {
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                              d);
    if (e != hipSuccess)
      return fail(h, PCSDF_ERR_HIP,
                  std::string("hipDeviceGetAttribute: ") +
                      hipGetErrorString(e));
    for (auto &sl : h->staging) {
      e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
      if (e != hipSuccess)
        return fail(h, PCSDF_ERR_HIP,
                    std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    h->max_lds = lds;
    h->device = d;
  } else if (d != h->device) {
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "handle is bound to device " + std::to_string(h->device) +
                    " but device " + std::to_string(d) + " is current");
  }
  return PCSDF_OK;
}

int ensure_buffer(Handle *h, DevBuf &b, size_t bytes, hipStream_t stream) {
  if (b.bytes >= bytes && b.ptr) return PCSDF_OK;
  if (b.ptr) {
    // Work queued earlier (on any stream) may still read the old buffer.
    (void)stream;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
      return fail(h, PCSDF_ERR_HIP,
                  std::string("hipDeviceSynchronize: ") +
                      hipGetErrorString(e));
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  const size_t want = align_up(bytes > 0 ? bytes : 256, 1 << 21);
  hipError_t e = hipMalloc(&b.ptr, want);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    return fail(h, PCSDF_ERR_OOM,
                "workspace allocation of " + std::to_string(want) +
                    " bytes failed: " + hipGetErrorString(e));
  }
  b.bytes = want;
  return PCSDF_OK;
}

int acquire_staging(Handle *h, size_t bytes) {
  const int k = h->staging_next;
  Handle::StagingSlot &sl = h->staging[k];
  if (sl.pending) {
    hipError_t e = hipEventSynchronize(sl.done);
    if (e != hipSuccess)
      return fail(h, PCSDF_ERR_HIP,
                  std::string("hipEventSynchronize: ") +
                      hipGetErrorString(e));
    sl.pending = false;
  }
  h->staging_cur = k;
  if (!(sl.bytes >= bytes && sl.p)) {
    if (sl.p) (void)hipHostFree(sl.p);
    sl.p = nullptr;
    sl.bytes = 0;
    const size_t want = align_up(bytes > 0 ? bytes : 64, 4096);
    hipError_t e = hipHostMalloc(&sl.p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      sl.p = nullptr;
      h->pinned = nullptr;
      (void)hipGetLastError();
      return fail(h, PCSDF_ERR_OOM, "pinned staging allocation failed");
    }
    sl.bytes = want;
  }
  h->pinned = sl.p;
  return PCSDF_OK;
}

int release_staging(Handle *h, hipStream_t stream) {
  Handle::StagingSlot &sl = h->staging[h->staging_cur];
  hipError_t e = hipEventRecord(sl.done, stream);
  if (e != hipSuccess)
    return fail(h, PCSDF_ERR_HIP,
                std::string("hipEventRecord: ") + hipGetErrorString(e));
  sl.pending = true;
  h->staging_next = (h->staging_cur + 1) % Handle::kStagingSlots;
  return PCSDF_OK;
}

int check_launch(Handle *h, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(h, PCSDF_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
  return PCSDF_OK;
}

int check_grid(Handle *h, const pcsdf_grid *g) {
  if (!g) return fail(h, PCSDF_ERR_INVALID_ARG, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > kMaxDim ||
      g->ny > kMaxDim || g->nz > kMaxDim)
    return fail(h, PCSDF_ERR_DIMS,
                "grid dimensions must be in [1, 1024], got " +
                    std::to_string(g->nx) + "x" + std::to_string(g->ny) +
                    "x" + std::to_string(g->nz));
  if (g->reserved != 0)
    return fail(h, PCSDF_ERR_INVALID_ARG, "grid.reserved must be 0");
  if (!std::isfinite(g->voxel_m) || !(g->voxel_m > 0))
    return fail(h, PCSDF_ERR_NUMERIC, "voxel_m must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g->origin_m[a]))
      return fail(h, PCSDF_ERR_NUMERIC, "origin_m must be finite");
  h->err.clear();
  return PCSDF_OK;
}

static hipEvent_t take_event(Handle *h) {
  if (!h->prof_pool.empty()) {
    hipEvent_t e = h->prof_pool.back();
    h->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(Handle *h, int id, hipStream_t s, bool per_launch)
    : h_(h), id_(id), s_(s) {
  if (!((h_->prof_mask >> id_) & 1u)) return;
  if (per_launch) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s_, &st) != hipSuccess ||
        st != hipStreamCaptureStatusNone)
      return;
    active_ = true;
    prev_ = h_->prof_scope;
    h_->prof_scope = this;
    return;
  }
  a_ = take_event(h_);
  b_ = take_event(h_);
  if (a_ && b_) (void)hipEventRecord(a_, s_);
}

void ProfScope::attach(hipEvent_t *a, hipEvent_t *b) {
  *a = *b = nullptr;
  if (!active_) return;
  hipEvent_t ea = take_event(h_), eb = take_event(h_);
  if (!ea || !eb) {
    if (ea) h_->prof_pool.push_back(ea);
    if (eb) h_->prof_pool.push_back(eb);
    return;
  }
  *a = ea;
  *b = eb;
  h_->prof_pending.push_back({id_, ea, eb, counted_ ? 0 : 1});
  counted_ = true;
}

void ProfScope::stop() {
  if (active_) {
    h_->prof_scope = prev_;
    active_ = false;
    return;
  }
  if (!a_ || !b_) return;
  (void)hipEventRecord(b_, s_);
  h_->prof_pending.push_back({id_, a_, b_, 1});
  a_ = b_ = nullptr;
}

int drain_profile(Handle *h) {
  for (auto &p : h->prof_pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) {
      h->prof_pending.clear();
      return fail(h, PCSDF_ERR_HIP,
                  std::string("profile events: ") + hipGetErrorString(e));
    }
    h->prof_ms[p.id] += ms;
    h->prof_n[p.id] += p.count;
    h->prof_pool.push_back(p.a);
    h->prof_pool.push_back(p.b);
  }
  h->prof_pending.clear();
  return PCSDF_OK;
}

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_profile_enable(pcsdf_handle *hp, int on) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  h->prof_mask = on ? (1u << PCSDF_KERNEL_COUNT) - 1u : 0u;
  return PCSDF_OK;
}

extern "C" int pcsdf_profile_select(pcsdf_handle *hp, uint32_t region_mask) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (region_mask >> PCSDF_KERNEL_COUNT)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "region mask has bits beyond PCSDF_KERNEL_COUNT");
  h->prof_mask = region_mask;
  return PCSDF_OK;
}

extern "C" int pcsdf_profile_read(pcsdf_handle *hp, int id, double *total_ms,
                                  int64_t *count) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (id < 0 || id >= PCSDF_KERNEL_COUNT || !total_ms || !count)
    return fail(h, PCSDF_ERR_INVALID_ARG, "bad profile id or output pointer");
  int rc = drain_profile(h);
  if (rc) return rc;
  *total_ms = h->prof_ms[id];
  *count = h->prof_n[id];
  return PCSDF_OK;
}

extern "C" int pcsdf_profile_reset(pcsdf_handle *hp) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = drain_profile(h);
  for (int i = 0; i < PCSDF_KERNEL_COUNT; ++i) {
    h->prof_ms[i] = 0.0;
    h->prof_n[i] = 0;
  }
  return rc;
}

extern "C" int pcsdf_create(pcsdf_handle **out) {
  if (!out) return PCSDF_ERR_INVALID_ARG;
  Handle *h = new (std::nothrow) Handle();
  *out = reinterpret_cast<pcsdf_handle *>(h);
  return h ? PCSDF_OK : PCSDF_ERR_OOM;
}

extern "C" void pcsdf_destroy(pcsdf_handle *hp) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return;
  for (auto &sl : h->staging)
    if (sl.pending) (void)hipEventSynchronize(sl.done);
  DevBuf *bufs[] = {&h->tmp_buf,       &h->plane_buf,      &h->chord_buf,
                    &h->param_buf,     &h->stack_buf,      &h->batch_params,
                    &h->batch_scratch, &h->sur_buf,     &h->union_buf,
                    &h->tmpl_buf};
  bool any = false;
  for (DevBuf *b : bufs) any = any || b->ptr;
  if (any) (void)hipDeviceSynchronize();
  for (DevBuf *b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  for (auto &sl : h->staging) {
    if (sl.p) (void)hipHostFree(sl.p);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  for (auto &p : h->prof_pending) {
    (void)hipEventSynchronize(p.b);
    h->prof_pool.push_back(p.a);
    h->prof_pool.push_back(p.b);
  }
  for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  delete h;
}

extern "C" const char *pcsdf_last_error(const pcsdf_handle *hp) {
  const Handle *h = reinterpret_cast<const Handle *>(hp);
  return h ? h->err.c_str() : "null handle";
}

extern "C" int pcsdf_set_tuning(pcsdf_handle *hp, const pcsdf_tuning *t) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!t) return fail(h, PCSDF_ERR_INVALID_ARG, "tuning is NULL");
  const int sg = t->static_segments;
  if (t->composite_slices_per_block < 0 || t->batch_slices_per_item < 0 ||
      t->batch_chunk_quads < 0 || t->batch_blocks_per_cu < 0 ||
      t->batch_blocks_per_cu > 32 || t->batch_chunk_quads % 256 != 0 ||
      !(sg == 0 || sg == 1 || sg == 2 || sg == 4 || sg == 8) ||
      (t->composite_order != 0 && t->composite_order != 1) ||
      t->composite_static16 < 0 || t->composite_static16 > 2)
    return fail(h, PCSDF_ERR_INVALID_ARG,
                "tuning values must be >= 0, blocks per CU <= 32, chunk "
                "quads a multiple of 256, static segments 0, 1, 2, 4 or 8, "
                "composite order 0 or 1 and composite static16 0, 1 or 2");
  h->tuning = *t;
  return PCSDF_OK;
}

extern "C" int pcsdf_get_tuning(const pcsdf_handle *hp, pcsdf_tuning *t) {
  const Handle *h = reinterpret_cast<const Handle *>(hp);
  if (!h || !t) return PCSDF_ERR_INVALID_ARG;
  *t = h->tuning;
  return PCSDF_OK;
}

extern "C" const char *pcsdf_status_string(int status) {
  switch (status) {
    case PCSDF_OK: return "PCSDF_OK";
    case PCSDF_ERR_INVALID_ARG: return "PCSDF_ERR_INVALID_ARG";
    case PCSDF_ERR_DIMS: return "PCSDF_ERR_DIMS";
    case PCSDF_ERR_ALIGN: return "PCSDF_ERR_ALIGN";
    case PCSDF_ERR_OOM: return "PCSDF_ERR_OOM";
    case PCSDF_ERR_HIP: return "PCSDF_ERR_HIP";
    case PCSDF_ERR_NUMERIC: return "PCSDF_ERR_NUMERIC";
    default: return "PCSDF_ERR_UNKNOWN";
  }
}
