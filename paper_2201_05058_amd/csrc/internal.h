// Library-internal declarations shared by the translation units of
// libpcsdf.so: the handle, error reporting, workspace management and the
// kernel launchers each unit exports to the others.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pcsdf.h"

namespace pcsdf {

class ProfScope;

constexpr int32_t kInf = INT32_MAX;  // "no site" / empty set
constexpr int kMaxDim = 1024;
constexpr int kMaxHumans = 256;

// A device buffer owned by the handle, grown on demand.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct Handle {
  std::string err;
  int device = -1;
  int max_lds = 65536;  // bytes of LDS a workgroup may use on `device`
  DevBuf tmp_buf;       // int32 [V] intermediate of the 3-D EDT; between
                        // builds the composite's 16-bit static copy
  DevBuf plane_buf;     // int32 planar fields of the humans
  DevBuf chord_buf;     // int2 chords of the humans' disks per row
  DevBuf param_buf;     // per-call parameter blocks (fixed-point centres)
  DevBuf stack_buf;     // envelope stacks when a column exceeds LDS
  DevBuf batch_params;  // batch: scene table, work items, centres
  DevBuf batch_scratch; // batch: chords, planes and row passes per scene
  DevBuf sur_buf;       // surrogate queries: features, outputs, fallback list
  DevBuf union_buf;     // full recompute: uint8 union map of one slice
  DevBuf tmpl_buf;      // shifted-template composite: per-human windows
  std::vector<char> batch_host;  // batch parameter block before upload
  // A second stream on the handle's device, forked from and joined back to
  // the caller's stream with the two events: the static build runs the
  // free set's channel of a column pass on it, beside the envelope kernel.
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  pcsdf_tuning tuning = {};  // launch shapes; 0 = default
  // pinned host staging for small per-call parameter blocks: a ring of
  // slots, so that a call only waits for the upload made kStagingSlots
  // calls before it
  static constexpr int kStagingSlots = 4;
  struct StagingSlot {
    void *p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
  };
  StagingSlot staging[kStagingSlots];
  int staging_next = 0, staging_cur = 0;
  void *pinned = nullptr;  // the slot acquired by the current call
  std::vector<int64_t> host_xy;  // fixed-point centres before upload
  // kernel timing with HIP events on the launch stream: bit `id` set =
  // region PCSDF_KERNEL_<id> timed (none by default)
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> prof_pool;
  struct Pending {
    int id;
    hipEvent_t a, b;
    int count;  // 1 for the first timed part of a region, else 0
  };
  std::vector<Pending> prof_pending;
  ProfScope *prof_scope = nullptr;  // innermost open per-launch region
  double prof_ms[PCSDF_KERNEL_COUNT] = {};
  int64_t prof_n[PCSDF_KERNEL_COUNT] = {};
};

// Times one region of launches when the handle's profiling is on; a no-op
// otherwise.  By default the region is bracketed by two event records on
// the stream.  A per-launch region instead times each of its kernels by
// the kernel's own dispatch (hipExtLaunchKernel's start and stop events),
// which puts no marker packets between the kernels; its kernels must be
// launched with launch_timed, and its time is the sum of their durations.
// Per-launch regions are not timed while the stream is being captured.
class ProfScope {
 public:
  ProfScope(Handle *h, int id, hipStream_t s, bool per_launch = false);
  ~ProfScope() { stop(); }
  void stop();
  // Start and stop events for one kernel of an open per-launch region
  // (both nullptr when it is not timed).
  void attach(hipEvent_t *a, hipEvent_t *b);

 private:
  Handle *h_;
  int id_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool active_ = false;   // an open per-launch region
  bool counted_ = false;  // its first kernel has been attached
  ProfScope *prev_ = nullptr;
};

// Launches `kernel`, timed by its dispatch when a per-launch region is
// open on the handle.
template <class F, class... Args>
inline void launch_timed(Handle *h, F kernel, dim3 grid, dim3 block,
                         uint32_t shmem, hipStream_t s, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (h->prof_scope) h->prof_scope->attach(&a, &b);
  if (a)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Waits for the handle's pending timed regions and adds them to its
// totals.
int drain_profile(Handle *h);

// Records `msg` as the handle's last error and returns `code`.
int fail(Handle *h, int code, const std::string &msg);

// Binds the handle to the current device on first use, checks later calls
// use the same device, and reads device limits.
int bind_device(Handle *h);

// Ensures `b` holds `bytes`; waits for `stream` before freeing a smaller
// allocation that work already enqueued may still use.
int ensure_buffer(Handle *h, DevBuf &b, size_t bytes, hipStream_t stream);

// Pinned staging buffer (h->pinned) for an H2D parameter upload: the next
// slot of the ring, after the upload last made from it has completed, with
// at least `bytes`.
int acquire_staging(Handle *h, size_t bytes);
// Marks the acquired slot as in use by work enqueued on `stream`.
int release_staging(Handle *h, hipStream_t stream);

// Checks the last launch; on failure records the HIP error.
int check_launch(Handle *h, const char *what);

int check_grid(Handle *h, const pcsdf_grid *g);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- launchers implemented in edt.hip ----------------------------------

// Row pass along x of a uint8 occupancy grid of `rows` rows of nx voxels:
// out = +d^2 (free voxel, d = distance along the row to the nearest
// occupied voxel), -d^2 (occupied, nearest free), +-kInf if none.
int launch_pass_x_u8(Handle *h, const uint8_t *occ, int32_t *out, int nx,
                     int64_t rows, hipStream_t s);

// Column pass of the separable EDT along a strided axis.  Columns are
// indexed by (fast index i in [0, nfast), outer index o in [0, nouter)):
// element q of column (i, o) is at o*outer_stride + i + q*stride, q < m.
// Input and output are signed-squared partial fields (see edt.hip).
// When sdf_out is non-null the pass also writes F(out) with voxel size h.
// square_input: the inputs are perfect squares (an x pass's output).
// use_side: the free set's channel may run on the handle's side stream
// (created on first use), joined back before the call returns.
int launch_pass_col(Handle *h, const int32_t *in, int32_t *out,
                    float *sdf_out, float h_f, int nfast, int nouter, int m,
                    int64_t stride, int64_t outer_stride, bool square_input,
                    bool use_side, hipStream_t s);

// ---- implemented in planes.hip -----------------------------------------

// Fixed-point disk centres [n_slices][K][2] and radii [n_slices] of the
// humans, read by the planar kernels: in device memory, or, when they fit,
// carried in the kernel arguments themselves, so that a call needs no
// upload before its first kernel.
constexpr int kCentresInArgs = 240;  // int64 words
struct Centres {
  const int64_t *xy = nullptr;  // device centres, or null: words below
  const int64_t *Rs = nullptr;  // device radii (with xy)
  int32_t rs_off = 0;           // index of the radii in w (without xy)
  int64_t w[kCentresInArgs];    // centres, then radii (without xy)
};
__device__ __forceinline__ int64_t centre_word(const Centres &c,
                                               int64_t i) {
  return c.xy ? c.xy[i] : c.w[i];
}
__device__ __forceinline__ int64_t radius_of(const Centres &c, int64_t s) {
  return c.xy ? c.Rs[s] : c.w[c.rs_off + s];
}

// Planar signed field of the humans' disk union for every slice, into
// P [n_slices][ny][nx]: chords per (slice, human, row) into `chords`, then
// one lane per pixel.  C holds the fixed-point centres [n_slices][K][2]
// and each slice's fixed-point disk radius; no human voxel at all when
// `empty` is set.  With `need` (device int32 [n_slices]) only slices with
// a non-zero entry are computed.
int launch_planes(Handle *h, const Centres &C, int K, bool empty,
                  int2 *chords, int32_t *P, int nx, int ny, int n_slices,
                  const int32_t *need, hipStream_t s);

// Chords only (the first step of launch_planes): chords[s][k][j], K humans
// per slice (0: nothing to do).
int launch_chords(Handle *h, const Centres &C, int K, int2 *chords, int nx,
                  int ny, int n_slices, const int32_t *need, hipStream_t s);

// ---- implemented in composite.hip --------------------------------------

// The humans of every slice validated and converted to the fixed-point
// lattice: centres [n_slices][K][2] and radii [n_slices], kept for the
// kernel arguments when they fit in kCentresInArgs words, else uploaded
// (one pinned staging copy); the chords buffer sized for them.
struct HumanSet {
  Centres C;          // fixed-point centres and radii
  int2 *chords;       // device, [n_slices][K][ny] (K >= 1 rows reserved)
  int K;              // humans per slice after dropping empty cylinders
  int Kt;             // highest voxel layer of the cylinders, -1 if none
  int has_above;      // a free layer exists above Kt
};
int humans_upload(Handle *h, const pcsdf_grid *g, int32_t n_slices,
                  int32_t n_humans, const double *xy_host, double radius_m,
                  const double *radius_per_slice, double height_m,
                  hipStream_t s, HumanSet *out);

// The humans' planes of every slice (validation of the human arguments,
// fixed-point upload, chords, planar EDT) into the handle's plane buffer.
// radius_per_slice (host, nullable) overrides radius_m slice by slice.
struct PlaneSet {
  int32_t *P;     // [n_slices][ny][nx] signed squared planar field
  int Kt;         // highest voxel layer of the cylinders, -1 if none
  int has_above;  // a free layer exists above Kt
};
int planes_run(Handle *h, const pcsdf_grid *g, int32_t n_slices,
               int32_t n_humans, const double *xy_host, double radius_m,
               const double *radius_per_slice, double height_m,
               const int32_t *need, hipStream_t s, PlaneSet *out);
// The same from humans already converted and placed by humans_upload.
int planes_from(Handle *h, const pcsdf_grid *g, const HumanSet &hs,
                int32_t n_slices, int32_t n_humans, const int32_t *need,
                hipStream_t s, PlaneSet *out);

// The streaming epilogue alone: outputs of every slice (with `need`, of
// the marked slices) from the static field and the planar fields P
// [n_slices][ny][nx] of the humans (cylinder layers 0..Kt).  With
// static_copy (callers that may use the handle's workspace) it may first
// make the 16-bit copy of the static field there and read that instead.
int launch_composite(Handle *h, const pcsdf_grid *g,
                     const int32_t *static_ssq_dev, const int32_t *P,
                     const int32_t *need, int Kt, int has_above,
                     int32_t n_slices, int32_t *out_ssq_dev,
                     float *out_sdf_dev, hipStream_t s,
                     bool static_copy = false);

// The whole predicted-composite call (validation, planes, streaming
// epilogue).  With `need` (device int32 [n_slices]) only the slices whose
// entry is non-zero are computed and written; the other slices of the
// outputs are left untouched.
int composite_run(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                  int32_t n_slices, int32_t n_humans, const double *xy_host,
                  double radius_m, const double *radius_per_slice,
                  double height_m, int32_t *out_ssq, float *out_sdf,
                  const int32_t *need, hipStream_t s);

// ---- implemented in direct.hip -----------------------------------------

// Exact queries from the planar fields and the static field (no 3-D field
// is built): the planes of the slices with a non-zero `need` entry (all
// when null) are built into the handle's plane buffer.
struct DirectSet {
  const int32_t *P;  // planar fields [n_slices][ny][nx]
  const int32_t *S;  // static SSQ
  int Kt, has_above;
};
int direct_setup(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                 int32_t n_slices, int32_t n_humans, const double *xy_host,
                 double radius_m, double height_m, const int32_t *need,
                 hipStream_t s, DirectSet *out);
int direct_from(Handle *h, const pcsdf_grid *g, const int32_t *static_ssq,
                const HumanSet &hs, int32_t n_slices, int32_t n_humans,
                const int32_t *need, hipStream_t s, DirectSet *out);
// Exact queries [0, n_queries), only those with mask[q] != 0 when a mask
// is given (device uint8 [n_queries]).
int launch_direct(Handle *h, const pcsdf_grid *g, const DirectSet &d,
                  int n_slices, int n_queries, const uint8_t *mask,
                  const float *centre, const float *radius,
                  const int32_t *slice, double eps, float *dist, float *grad,
                  uint8_t *status, float *cost, hipStream_t s);

// ---- implemented in query.hip ------------------------------------------

// Sphere queries for the indices list[0 .. *count) only (count on the
// device; the grid is sized for at most `max_count` entries).
int launch_query_list(Handle *h, const pcsdf_grid *g, const float *sdf,
                      int n_slices, const int32_t *list,
                      const int32_t *count, int max_count,
                      const float *centre, const float *radius,
                      const int32_t *slice, double eps, float *dist,
                      float *grad, uint8_t *status, float *cost,
                      hipStream_t s);

// ---- implemented in mlp.hip --------------------------------------------

// The handle a network was created on.
Handle *mlp_handle(pcsdf_mlp *m);
// Inputs per row of the network.
int mlp_inputs(const pcsdf_mlp *m);
// Value and input gradient of rows [0, min(n, *n_dev)) (fused inference).
int mlp_rows(pcsdf_mlp *m, int n, const int32_t *n_dev, const float *x,
             float *y, float *gx, hipStream_t s);

}  // namespace pcsdf
