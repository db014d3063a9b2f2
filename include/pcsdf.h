/*
 * pcsdf — predicted composite signed distance fields on MI355X (gfx950).
 *
 * C-ABI of the GPU library.  The operations follow the mapping section of
 * Finean et al., "Motion Planning in Dynamic Environments Using
 * Context-Aware Human Trajectory Prediction" (2022), section "Mapping -
 * Predicted Composite Distance Fields", and its RHAP-GPMP2 section:
 *   - an environment distance field, computed once for the static map;
 *   - one composite field per predicted time slice, the elementwise min of
 *     the environment field and the field of the humans (vertical
 *     cylinders) at their predicted positions;
 *   - the fields sampled, distance and gradient, at collision spheres for
 *     GPMP2's hinge-loss obstacle factors, with every time index past the
 *     last slice mapped to the last slice.
 *
 * Conventions shared by every call:
 *   - Grids are x fastest: idx = (k*ny + j)*nx + i, no padding; voxel
 *     (i,j,k) has its centre at origin + h*(i+1/2, j+1/2, k+1/2).
 *   - Fields come in two forms.  SSQ (int32) is the signed squared distance
 *     in voxel units: E_O(v) = min_{u in O} |v-u|^2 for a free voxel,
 *     -E_{G\O}(v) for an occupied one, +INT32_MAX / -INT32_MAX when the
 *     other set is empty.  SDF (fp32, metres) is
 *     F(x) = sign(x) * ((float)h * sqrtf(|x|)), +-inf for +-INT32_MAX.
 *   - Per-slice outputs are slice-major: [n_slices][nz][ny][nx].
 *   - Every device buffer is owned by the caller; the library never frees
 *     it.  The library owns only its handle's workspace.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream; no call waits for the device except
 *     where stated.  A handle is not reentrant: use one per host thread.
 *     Calls on one handle share its workspace, so calls enqueued on
 *     different streams must be ordered by the caller (events, or one
 *     handle per stream).
 *   - Every call returns PCSDF_OK (0) or an error code.  On error nothing
 *     has been enqueued unless the code is PCSDF_ERR_HIP, and output
 *     buffers are unspecified.  pcsdf_last_error() describes the failure.
 *     No C++ exception crosses this interface.
 */
#ifndef PCSDF_H_
#define PCSDF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pcsdf_status_code {
  PCSDF_OK = 0,
  PCSDF_ERR_INVALID_ARG = 1, /* null pointer, bad count or parameter */
  PCSDF_ERR_DIMS = 2,        /* grid dimension out of [1, 1024] etc. */
  PCSDF_ERR_ALIGN = 3,       /* device pointer not 4-byte aligned */
  PCSDF_ERR_OOM = 4,         /* workspace allocation failed */
  PCSDF_ERR_HIP = 5,         /* a HIP runtime call failed */
  PCSDF_ERR_NUMERIC = 6      /* NaN/Inf or out-of-range real input */
};

/* Status bits of a sphere query (pcsdf_query_spheres). */
#define PCSDF_Q_OOR_X 1u         /* centre outside the span of voxel centres in x; clamped */
#define PCSDF_Q_OOR_Y 2u
#define PCSDF_Q_OOR_Z 4u
#define PCSDF_Q_SLICE_CLAMPED 8u /* slice >= n_slices, slice n_slices-1 used */
#define PCSDF_Q_INF_CORNER 16u   /* a corner is +-inf: dist = +-inf, grad = 0 */
#define PCSDF_Q_SLICE_NEG 32u    /* slice < 0: dist, grad, cost are NaN */

/* Timed regions of pcsdf_profile_read. */
#define PCSDF_KERNEL_COMPOSITE 0 /* streaming composite epilogue kernel */
#define PCSDF_KERNEL_PLANES 1    /* humans' planar EDT (chords, coverage or
                                    row pass, then the planes) */
#define PCSDF_KERNEL_QUERY 2     /* sphere query kernel */
#define PCSDF_KERNEL_STATIC 3    /* the three passes of the static build */
#define PCSDF_KERNEL_BATCH 4     /* a batch: both of its launches */
#define PCSDF_KERNEL_MLP 5       /* surrogate forward (+ input gradient) */
#define PCSDF_KERNEL_MLP_TRAIN 6 /* one surrogate training step */
#define PCSDF_KERNEL_SURROGATE_DECIDE 7 /* surrogate accept / fallback split */
#define PCSDF_KERNEL_RECOMPUTE 8 /* full recompute: every slice's union EDT */
#define PCSDF_KERNEL_TEMPLATE 9  /* shifted-template composite epilogue */
#define PCSDF_KERNEL_FACTORS 10  /* obstacle factors of all support states */
#define PCSDF_KERNEL_COUNT 11

typedef struct pcsdf_handle pcsdf_handle;

/* Regular grid.  nx, ny, nz in [1, 1024]; voxel_m > 0 and finite; origin
 * finite (the world position of the grid's minimum corner). */
typedef struct pcsdf_grid {
  int32_t nx, ny, nz;
  int32_t reserved; /* must be 0 */
  double voxel_m;
  double origin_m[3];
} pcsdf_grid;

/* Creates a handle.  Touches no device; the workspace is allocated on the
 * device current at the first call that needs it, and that device is used
 * by the handle from then on.  Returns PCSDF_ERR_INVALID_ARG if out is
 * NULL, PCSDF_ERR_OOM if the host allocation fails. */
int pcsdf_create(pcsdf_handle **out);

/* Waits for the handle's pending uploads, frees its workspace, its second
 * stream and the handle.  NULL is ignored.  Device buffers passed to
 * earlier calls are not touched. */
void pcsdf_destroy(pcsdf_handle *h);

/* Message of the last failed call on this handle ("" if none).  The
 * pointer stays valid until the next call on the handle. */
const char *pcsdf_last_error(const pcsdf_handle *h);

/* Name of a status code. */
const char *pcsdf_status_string(int status);

/* Environment distance field (mapping section: the environment field is
 * computed once, or maintained; here one exact signed EDT of the caller's
 * voxel map).
 *   occ_dev  [V] uint8, nonzero = occupied.             (device, read)
 *   ssq_dev  [V] int32 SSQ of the occupied set.         (device, written)
 *   sdf_dev  [V] fp32 F(SSQ), may be NULL.              (device, written)
 * Uses a workspace of 4*V bytes.  Exact: the int32 result is unique.
 * Part of the work may run on a second stream the handle owns (created at
 * the first call that needs it, destroyed with the handle), ordered after
 * the work enqueued on `stream` before the call and joined back into
 * `stream` before the call returns (with events, so a capture of `stream`
 * into a HIP graph includes it). */
int pcsdf_build_static_sdf(pcsdf_handle *h, const pcsdf_grid *grid,
                           const uint8_t *occ_dev, int32_t *ssq_dev,
                           float *sdf_dev, void *stream);

/* The environment collapsed to the floor plane for the human-trajectory
 * predictor (RHAP-GPMP2 section: the 3-D voxel grid is collapsed to 2-D and
 * its EDT computed on the GPU): pixel (i, j) is occupied iff some voxel
 * (i, j, k) with z_lo <= k <= z_hi is, and the result is that planar map's
 * signed squared EDT and F, as pcsdf_build_static_sdf on an nx x ny x 1
 * grid.  ssq_dev [ny][nx] int32 (required), sdf_dev [ny][nx] fp32
 * (nullable).  Needs 0 <= z_lo <= z_hi < nz.  Uses 4*nx*ny + nx*ny bytes
 * of workspace. */
int pcsdf_build_floor_sdf(pcsdf_handle *h, const pcsdf_grid *grid,
                          const uint8_t *occ_dev, int32_t z_lo, int32_t z_hi,
                          int32_t *ssq_dev, float *sdf_dev, void *stream);

/* The sequence of predicted composite fields (mapping section: the
 * composite is a parallel min of the environment field and the fields of
 * the humans, modelled as cylinder primitives, at their predicted
 * positions; RHAP-GPMP2 section: one composite field per time slice).
 *   static_ssq_dev [V] int32 from pcsdf_build_static_sdf.   (device, read)
 *   n_slices >= 1, n_humans in [0, 256].
 *   human_xy_host  [n_slices][n_humans][2] fp64 metres, the predicted
 *                  (x, y) of each human in each slice.      (host, read
 *                  before the call returns)
 *   radius_m, height_m: the cylinder (base at z = origin_m[2]).
 *   out_ssq_dev    [n_slices][V] int32, may be NULL.        (device, written)
 *   out_sdf_dev    [n_slices][V] fp32, may be NULL.         (device, written)
 * At least one output must be non-NULL.  Per slice s the humans' voxels
 * are the closed integer voxelisation on a 2^-16 voxel lattice:
 *   X = rint(((x - o_x)/h)*2^16), Y likewise, R = rint((r/h)*2^16),
 *   Hq = rint((H/h)*2^16); voxel (i,j,k) is in a cylinder iff
 *   (2^15(2i+1) - X)^2 + (2^15(2j+1) - Y)^2 <= R^2 and 2^15(2k+1) <= Hq.
 * Voxels outside the grid do not exist (humans are clipped).  The result
 * is min(static SSQ, SSQ of the humans' voxels), both signed, and its F.
 * Errors: PCSDF_ERR_NUMERIC for non-finite inputs or when a fixed-point
 * value reaches 2^62 in magnitude or R reaches 2^31.
 * Uses a workspace of 8*n_slices*nx*ny + 24*n_slices*n_humans*ny bytes,
 * plus 2*V bytes for the 16-bit static copy (see pcsdf_tuning) when the
 * outputs are written in per-slice packs of 4, 2 or 1 voxels. */
int pcsdf_predicted_composite_sdf(pcsdf_handle *h, const pcsdf_grid *grid,
                                  const int32_t *static_ssq_dev,
                                  int32_t n_slices, int32_t n_humans,
                                  const double *human_xy_host,
                                  double radius_m, double height_m,
                                  int32_t *out_ssq_dev, float *out_sdf_dev,
                                  void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same call
 * and result as pcsdf_predicted_composite_sdf, with the planar fields, row
 * passes and chords in a library-owned device array of 64 MiB per device
 * (held until the process ends) instead of the handle's workspace.  It
 * calls no allocating routine; the caller passes every input and output.
 * Limits (PCSDF_ERR_INVALID_ARG beyond them):
 *   2*n_slices*n_humans + n_slices <= 240 (the fixed-point centres travel
 *   in the kernels' arguments), and
 *   align256(8*n_slices*nx*ny) + 8*n_slices*max(n_humans,1)*ny <= 64 MiB.
 * Every call on one device shares that array: calls that overlap on one
 * device (other streams, other handles, other threads) race and must be
 * ordered by the caller.  No profiling region is timed. */
int pcsdf_predicted_composite_sdf_noalloc(
    pcsdf_handle *h, const pcsdf_grid *grid, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream);

/* The same sequence with a radius per slice (discussion section: the
 * cylinders could grow over the prediction horizon to account for the
 * growing uncertainty of the predicted positions, e.g. r(t) = r0 + sigma*t).
 * radius_per_slice_m [n_slices] fp64 metres (host, read before the call
 * returns); every human of slice s has radius radius_per_slice_m[s].  All
 * other arguments, the voxelisation and the result as for
 * pcsdf_predicted_composite_sdf. */
int pcsdf_predicted_composite_sdf_growing(
    pcsdf_handle *h, const pcsdf_grid *grid, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    const double *radius_per_slice_m, double height_m, int32_t *out_ssq_dev,
    float *out_sdf_dev, void *stream);

/* Full recompute, the baseline of the mapping section's benchmark (Fig. 6:
 * composite fields against computing every slice's distance field from
 * scratch): for every slice, the exact signed squared EDT of the union of
 * the environment's occupied voxels and the humans' voxels, by the same
 * three passes as pcsdf_build_static_sdf.
 *   static_occ_dev [V] uint8 environment map (nonzero = occupied). (device)
 *   human arguments and voxelisation as pcsdf_predicted_composite_sdf.
 *   out_ssq_dev [n_slices][V] int32, required (the x pass writes it first).
 *   out_sdf_dev [n_slices][V] fp32, may be NULL.
 * Outside both sets the result equals the composite; inside it is the
 * depth in the union.  Uses the static build's workspace plus V bytes. */
int pcsdf_recompute_sdf(pcsdf_handle *h, const pcsdf_grid *grid,
                        const uint8_t *static_occ_dev, int32_t n_slices,
                        int32_t n_humans, const double *human_xy_host,
                        double radius_m, double height_m,
                        int32_t *out_ssq_dev, float *out_sdf_dev,
                        void *stream);

/* The mapping section's own placement of the humans: each human's cylinder
 * field is computed once (at its first-slice position, sub-voxel phase
 * included, in a window of (2(nx+m)+1) x (2(ny+m)+1) voxels around it,
 * m = floor(R/2^16) + 2, unclipped by the grid) and every slice composites
 * it shifted by the whole number of voxels nearest to the human's
 * displacement since the first slice, d = floor((X_s - X_0 + 2^15)/2^16):
 *   C_s = min(static SSQ, min over humans of the shifted templates),
 * a human contributing nothing where its window does not reach.
 * Arguments, layouts and outputs as pcsdf_predicted_composite_sdf.  Equal
 * to that call's result when every displacement is a whole number of
 * voxels, the humans do not overlap and their cylinders lie inside the
 * grid; otherwise an approximation of it (sub-voxel shift, the first
 * slice's voxelisation phase, unclipped windows at the grid's edge, the
 * min of separate signed fields where humans overlap).
 * Uses a workspace of 8*n_humans*(window pixels) bytes. */
int pcsdf_template_composite_sdf(pcsdf_handle *h, const pcsdf_grid *grid,
                                 const int32_t *static_ssq_dev,
                                 int32_t n_slices, int32_t n_humans,
                                 const double *human_xy_host,
                                 double radius_m, double height_m,
                                 int32_t *out_ssq_dev, float *out_sdf_dev,
                                 void *stream);

/* Sphere queries on a sequence of fp32 fields (GPMP2 obstacle factors
 * sample distance and gradient; RHAP-GPMP2 assigns the last field to every
 * time index past the horizon).
 *   sdf_dev    [n_slices][V] fp32 fields.                   (device, read)
 *   centre_dev [Q][3] fp32 metres, radius_dev [Q] fp32,
 *   slice_dev  [Q] int32.                                   (device, read)
 *   dist_dev   [Q] fp32: trilinear distance at the centre minus radius.
 *   grad_dev   [Q][3] fp32: gradient of the trilinear field (m/m).
 *   status_dev [Q] uint8 PCSDF_Q_* bits, may be NULL.
 *   cost_dev   [Q] fp32 hinge max(0, hinge_eps_m - dist), may be NULL.
 * Interpolation is in fp64: g_a = (c_a - o_a)/h - 1/2 clamped to
 * [0, n_a - 1], cell i_a = min(floor(g_a), n_a - 2).  Requires every
 * n_a >= 2 (else PCSDF_ERR_DIMS).  n_queries = 0 is a no-op. */
int pcsdf_query_spheres(pcsdf_handle *h, const pcsdf_grid *grid,
                        const float *sdf_dev, int32_t n_slices,
                        int32_t n_queries, const float *centre_dev,
                        const float *radius_dev, const int32_t *slice_dev,
                        double hinge_eps_m, float *dist_dev, float *grad_dev,
                        uint8_t *status_dev, float *cost_dev, void *stream);

/* The same sphere queries on the composite fields that
 * pcsdf_predicted_composite_sdf would build (its arguments), answered
 * without building them: the humans' voxels of a slice are D x {0..Kt}
 * (a disk union times the cylinders' layers), so the composite at voxel
 * (i, j, k) is min(static SSQ, the humans' value from the planar signed
 * field of D at pixel (i, j) and layer k).  Only the planar fields are
 * built (n_slices * nx * ny values); each query reads four planar and
 * eight static values.  Outputs, status bits and layouts as
 * pcsdf_query_spheres, and bit-identical to building the fields and
 * sampling them.  Uses the planes' workspace only. */
int pcsdf_query_spheres_direct(
    pcsdf_handle *h, const pcsdf_grid *grid, const int32_t *static_ssq_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, int32_t n_queries,
    const float *centre_dev, const float *radius_dev,
    const int32_t *slice_dev, double hinge_eps_m, float *dist_dev,
    float *grad_dev, uint8_t *status_dev, float *cost_dev, void *stream);

/* Obstacle factors of the planner (RHAP-GPMP2 section: the obstacle factor
 * of time index i reads composite field i, the last field past the
 * horizon; GPMP2's hinge loss on the distance field, as adopted in the
 * human-trajectory section).  For support state i and sphere j:
 *   e_ij = max(0, eps_m - (d_s(c_ij) - r_j)),  s = min(state_slice[i], n-1)
 *   J_ij = -grad d_s(c_ij) where e_ij > 0, else 0
 *   cost_i = sum_j 0.5 * (e_ij / sigma)^2   (fp64)
 * with d and grad sampled exactly as pcsdf_query_spheres does.
 *   sdf_dev          [n_slices][V] fp32 composite fields.     (device, read)
 *   centre_dev       [n_states][n_spheres][3] fp32 metres.    (device, read)
 *   radius_dev       [n_spheres] fp32 metres.                 (device, read)
 *   state_slice_dev  [n_states] int32; < 0 gives NaN.         (device, read)
 *   err_dev          [n_states][n_spheres] fp32.              (device, written)
 *   jac_dev          [n_states][n_spheres][3] fp32.           (device, written)
 *   cost_dev         [n_states] fp64 (8-byte aligned).        (device, written)
 * An infinite corner gives e = 0 (+inf) or +inf (-inf) and J = 0.
 * Errors: sigma must be > 0 and eps finite (PCSDF_ERR_NUMERIC). */
int pcsdf_obstacle_factors(pcsdf_handle *h, const pcsdf_grid *grid,
                           const float *sdf_dev, int32_t n_slices,
                           int32_t n_states, int32_t n_spheres,
                           const float *centre_dev, const float *radius_dev,
                           const int32_t *state_slice_dev, double eps_m,
                           double sigma, float *err_dev, float *jac_dev,
                           double *cost_dev, void *stream);

/* ---- Batches of scenes ------------------------------------------------
 * One scene: the arguments of pcsdf_predicted_composite_sdf.  Scenes of a
 * batch may differ in grid size, voxel size, slice count and humans. */
typedef struct pcsdf_scene {
  pcsdf_grid grid;
  const int32_t *static_ssq_dev; /* [V] device, read */
  int32_t n_slices, n_humans;
  const double *human_xy_host; /* [n_slices][n_humans][2] host, read */
  double radius_m, height_m;
  int32_t *out_ssq_dev; /* [n_slices][V] device, may be NULL */
  float *out_sdf_dev;   /* [n_slices][V] device, may be NULL */
} pcsdf_scene;

/* Launch shapes (0 = library default).  Chosen by the autotuner
 * (pcsdf_autotune_*) or set directly. */
typedef struct pcsdf_tuning {
  int32_t composite_slices_per_block; /* composite: slices per block row */
  int32_t batch_slices_per_item;      /* batch: slices per composite item */
  int32_t batch_chunk_quads;          /* batch: voxel quads per composite
                                         item, a multiple of 256 */
  int32_t batch_blocks_per_cu;        /* batch: persistent workgroups per CU
                                         of both launches, at most 32; 0:
                                         8 per CU for the planar items and
                                         one workgroup per composite item */
  int32_t static_segments;            /* static EDT column passes: segments
                                         (one wave each) per column, 1, 2,
                                         4 or 8; 0: one per 32 voxels of
                                         the column, at most 8 */
  int32_t composite_order;            /* composite: 0 (default) blocks in
                                         flight write the same few slices
                                         over consecutive voxel chunks; 1
                                         the slice groups of a chunk run in
                                         succession on one XCD and re-read
                                         its static values from L2 */
  int32_t composite_static16;         /* composite: 1 the slice groups read
                                         the static field; 2 a 16-bit copy
                                         of it made first (half the bytes;
                                         values beyond +-32767 are read
                                         from the field), in the handle's
                                         workspace (2 B per voxel); 0 the
                                         copy for grids of at least 2^25
                                         voxels with at least 4 slice
                                         groups */
} pcsdf_tuning;

int pcsdf_set_tuning(pcsdf_handle *h, const pcsdf_tuning *t);
int pcsdf_get_tuning(const pcsdf_handle *h, pcsdf_tuning *t);

/* All scenes' composite fields in two launches: the same outputs, byte
 * for byte, as one pcsdf_predicted_composite_sdf call per scene.  A
 * persistent grid strides over the (scene, slice, pixel tile) planar-field
 * items of all scenes; then the (scene, slice group, voxel chunk)
 * composite items run one per workgroup or under a persistent grid (see
 * pcsdf_tuning); no workgroup waits on another.  Host arrays are read
 * before the call returns.  Workspace: per scene
 * 8*n_slices*nx*ny + 8*n_slices*max(n_humans,1)*ny bytes, plus the work
 * list.  Errors as pcsdf_predicted_composite_sdf, prefixed with the scene
 * index; PCSDF_ERR_DIMS when the batch has 2^31 or more composite items. */
int pcsdf_predicted_composite_sdf_batch(pcsdf_handle *h, int32_t n_scenes,
                                        const pcsdf_scene *scenes,
                                        void *stream);

/* The same batch captured once in a hipGraph (parameter upload from pinned
 * memory owned by the graph, then the batch's two launches) and
 * replayed with one hipGraphLaunch.  The graph owns its workspace; the
 * scenes' device buffers must outlive it.  set_positions replaces one
 * scene's predicted positions for later launches (waiting for a launch
 * still reading them).  Errors of graph calls are reported through the
 * creating handle. */
typedef struct pcsdf_batch_graph pcsdf_batch_graph;
int pcsdf_batch_graph_create(pcsdf_handle *h, int32_t n_scenes,
                             const pcsdf_scene *scenes, void *stream,
                             pcsdf_batch_graph **out);
int pcsdf_batch_graph_set_positions(pcsdf_batch_graph *g, int32_t scene,
                                    const double *human_xy_host);
int pcsdf_batch_graph_launch(pcsdf_batch_graph *g, void *stream);
void pcsdf_batch_graph_destroy(pcsdf_batch_graph *g);

/* Autotuners: time candidate launch shapes on the caller's real inputs by
 * the GPU time of the kernels they shape (HIP events on `stream`, `reps`
 * runs each after a warm-up run; host work between calls does not count),
 * store the fastest in the handle's tuning and return it with its time in
 * milliseconds per run.  The composite tuner makes three interleaved
 * rounds over its slice groups in both block orders and keeps each
 * candidate's fastest round.
 * Outputs are written as by the tuned call.  They synchronise with the
 * device and leave the handle's profiling state and totals unchanged. */
int pcsdf_autotune_batch(pcsdf_handle *h, int32_t n_scenes,
                         const pcsdf_scene *scenes, void *stream,
                         int32_t reps, pcsdf_tuning *best, double *best_ms);
int pcsdf_autotune_composite(pcsdf_handle *h, const pcsdf_scene *scene,
                             void *stream, int32_t reps, pcsdf_tuning *best,
                             double *best_ms);

/* ---- Learned surrogate for sphere queries (not in the paper) ----------
 * A multilayer perceptron mapping n_in <= 32 input features to one value:
 * u = (x - offset) * scale;  4 hidden layers of 128 SiLU units;
 * y = out_scale * (W4 a4 + b4).  Weights are fp32 masters used as BF16 on
 * the matrix cores with FP32 accumulation; inputs, activations, SiLU
 * derivatives and backward pre-activation gradients are rounded to BF16
 * before each product.  Parameter vector (fp32, pcsdf_mlp_param_count):
 * W0[128][n_in] b0[128] W1[128][128] b1 W2[128][128] b2 W3[128][128] b3
 * W4[1][128] b4[1].  The network object owns its weights, optimiser state
 * and workspace on the handle's device; calls on one network must not
 * overlap.  Training batches are padded internally to a multiple of 1024
 * rows. */
#define PCSDF_MLP_MAX_IN 32
#define PCSDF_SURROGATE_IN 16 /* features per (query, human) row */
typedef struct pcsdf_mlp pcsdf_mlp;
/* Parameters of a network with n_in inputs (-1 outside [1, 32]). */
int pcsdf_mlp_param_count(int32_t n_in);
int pcsdf_mlp_create(pcsdf_handle *h, int32_t n_in, pcsdf_mlp **out);
void pcsdf_mlp_destroy(pcsdf_mlp *m);
/* Uploads parameters and the input/output normalisation (n_in values
 * each), and resets the optimiser (waits for the device).
 * PCSDF_ERR_NUMERIC on non-finite values. */
int pcsdf_mlp_set_params(pcsdf_mlp *m, const float *params_host,
                         const float *in_offset_host,
                         const float *in_scale_host, float out_scale);
int pcsdf_mlp_get_params(pcsdf_mlp *m, float *params_host);
/* y[n] = network(x[n][n_in]) and, if grad_x_dev is given, dy/dx
 * [n][n_in]. */
int pcsdf_mlp_forward(pcsdf_mlp *m, int32_t n, const float *x_dev,
                      float *y_dev, float *grad_x_dev, void *stream);
/* Gradient of sum_m dy[m] * y[m] w.r.t. every parameter (grad_params_dev,
 * fp32 [param count]) and, if given, w.r.t. the inputs. */
int pcsdf_mlp_gradients(pcsdf_mlp *m, int32_t n, const float *x_dev,
                        const float *dy_dev, float *grad_params_dev,
                        float *grad_x_dev, void *stream);
/* One Adam step (bias-corrected) on the mean squared error between y(x)
 * and target [n]; loss_dev [1] receives the loss before the step, if
 * given.  The same as pcsdf_mlp_loss_gradients followed by
 * pcsdf_mlp_adam_step with that gradient. */
int pcsdf_mlp_train_step(pcsdf_mlp *m, int32_t n, const float *x_dev,
                         const float *target_dev, float lr, float beta1,
                         float beta2, float eps, float *loss_dev,
                         void *stream);
/* Gradient of the mean squared error (1/n) sum_m (y(x_m) - target_m)^2
 * w.r.t. every parameter, grad_params_dev fp32 [param count] (device,
 * written), as the training step forms it; loss_dev [1] (nullable) gets
 * the loss.  No parameter changes. */
int pcsdf_mlp_loss_gradients(pcsdf_mlp *m, int32_t n, const float *x_dev,
                             const float *target_dev, float *grad_params_dev,
                             float *loss_dev, void *stream);
/* One Adam step (Kingma and Ba, with bias correction) from the gradient
 * grad_params_dev fp32 [param count] (device, read): with t the step
 * count after it is advanced by one,
 *   m1 = beta1 m1 + (1 - beta1) g,  m2 = beta2 m2 + (1 - beta2) g^2,
 *   p -= lr (m1 / c1) / (sqrt(m2 / c2) + eps),
 *   c1 = fp32(1 - beta1^t), c2 = fp32(1 - beta2^t) (powers in fp64),
 * in fp32 per parameter, then the BF16 weight copies are refreshed.
 * PCSDF_ERR_NUMERIC for lr < 0, betas outside [0, 1) or eps <= 0. */
int pcsdf_mlp_adam_step(pcsdf_mlp *m, const float *grad_params_dev, float lr,
                        float beta1, float beta2, float eps, void *stream);
/* The optimiser's whole state for checkpoints: the fp32 masters, Adam's
 * first and second moments (each fp32 [param count], host) and the step
 * count.  get waits for the device.  set uploads all of it with the
 * normalisation (as pcsdf_mlp_set_params, which it calls first, but keeps
 * the given moments and step instead of resetting them); a network
 * restored this way continues training exactly as the saved one would.
 * PCSDF_ERR_NUMERIC on non-finite values or a negative second moment. */
int pcsdf_mlp_get_state(pcsdf_mlp *m, float *params_host, float *m1_host,
                        float *m2_host, int64_t *step);
int pcsdf_mlp_set_state(pcsdf_mlp *m, const float *params_host,
                        const float *m1_host, const float *m2_host,
                        int64_t step, const float *in_offset_host,
                        const float *in_scale_host, float out_scale);

/* The surrogate's input row for one (query, human) pair: the
 * PCSDF_SURROGATE_IN features the network of pcsdf_query_spheres_surrogate
 * reads, in voxel units of the grid.  With the humans' fixed-point centres
 * X, Y and radius R of the query's slice s' = clamp(slice, 0, n_slices-1)
 * (as pcsdf_predicted_composite_sdf converts them), the top layer Kt of
 * the cylinders, g = (c - origin)/h - 1/2 (fp64), the human's axis
 * (cx, cy) = (X, Y)/2^16 - 1/2, Rv = R/2^16, (ux, uy) = g_xy - (cx, cy),
 * rho = |(ux, uy)|, a = rho - Rv, w = g_z - Kt, d = |(max(a,0), max(w,0))|
 * (the distance to the continuous cylinder), phi = ((X, Y) - 2^15) mod
 * 2^16 / 2^16 and f = g - floor(g):
 *   x = [ux/rho, uy/rho, a, w, d, 1/(1+d), sin 2pi phi_x, cos 2pi phi_x,
 *        sin 2pi phi_y, cos 2pi phi_y, sin 2pi f_x, cos 2pi f_x,
 *        sin 2pi f_y, cos 2pi f_y, sin 2pi f_z, cos 2pi f_z]
 * (computed in fp64, rounded to fp32; ux/rho = uy/rho = 0 when rho = 0).
 *   centre_dev [Q][3] fp32, slice_dev [Q] int32,
 *   human_dev  [Q] int32 human index of each row (NULL: 0),
 *   label_dev  [Q] fp32 metres, nullable (the exact distance at the centre),
 *   x_dev      [Q][16] fp32 (written),
 *   base_dev   [Q] fp32 d in voxels, nullable,
 *   target_dev [Q] fp32 label/h - d in voxels, nullable (needs labels).
 * Human arguments as pcsdf_predicted_composite_sdf (n_humans >= 1). */
int pcsdf_surrogate_human_features(
    pcsdf_handle *h, const pcsdf_grid *grid, int32_t n_slices,
    int32_t n_humans, const double *human_xy_host, double radius_m,
    double height_m, int32_t n_queries, const float *centre_dev,
    const int32_t *slice_dev, const int32_t *human_dev, const float *label_dev,
    float *x_dev, float *base_dev, float *target_dev, void *stream);

/* Sphere queries answered by the surrogate, with the exact path as
 * fallback, for the composite fields that pcsdf_predicted_composite_sdf
 * would build from the same static field and humans (arguments as there;
 * for humans moving at constant velocity the positions of slice j are
 * p + v j dt).  The network m (PCSDF_SURROGATE_IN inputs, created on
 * handle h) predicts one human's exact field: per (query, human) row
 * y_k = fp32(h (d + clamp(network(x), -1/2, 3/2))) metres, x and d as in
 * pcsdf_surrogate_human_features; its gradient is the closed-form
 * gradient of d plus, when the network's value is not clamped, the
 * network's feature gradient through the features' closed-form
 * derivatives.  The environment's value e is the static fp32 field
 * static_sdf_dev [V] sampled at the centre exactly as pcsdf_query_spheres
 * samples it (zero radius).  A human is absent when no voxel centre of the
 * grid lies within Rv of its axis along x or y (cx + Rv < 0, cx - Rv >
 * nx - 1, likewise y) and clipped when present and its disk may reach
 * beyond the grid (cx - Rv <= -1, cx + Rv >= nx, likewise y).  With
 * y = min(e, y_k of the present humans) (the environment wins ties, then
 * the lower index) and m2 the second smallest candidate, a query falls
 * back to the exact path when
 *   - its centre lies outside the span of voxel centres,
 *   - y - r is below fallback_margin_m, or y - r or the gradient is not
 *     finite,
 *   - m2 - y < band_m (the candidates' order may change inside the
 *     query's cell; 2 sqrt(3) h covers every such cell), or
 *   - a clipped human's y_k <= y + band_m,
 * and otherwise gets dist = y - r, grad = the winner's gradient, status =
 * SLICE_CLAMPED or 0, cost = max(0, hinge_eps_m - dist).  Queries with
 * slice < 0 get NaN and SLICE_NEG.  Humans whose lower bound
 * h (d - 1/2) exceeds the least upper bound h (d + 3/2) (or e) by more
 * than band_m cannot change the answer and are not evaluated; rows beyond
 * the workspace's cap of max(4 Q, 2^20) rows make their queries fall back.
 * rows_dev [1] int32 (nullable, device) receives the number of (query,
 * human) rows the network evaluated.
 * used_fallback_dev [Q] (nullable) is 1 for exact answers, which are
 * computed as pcsdf_query_spheres_direct computes them: no 3-D field is
 * built, only the planar fields of the slices that some fallback query
 * reads.  Outputs and layouts as pcsdf_query_spheres.  No host
 * synchronisation. */
int pcsdf_query_spheres_surrogate(
    pcsdf_handle *h, pcsdf_mlp *m, const pcsdf_grid *grid,
    const int32_t *static_ssq_dev, const float *static_sdf_dev,
    int32_t n_slices, int32_t n_humans, const double *human_xy_host,
    double radius_m, double height_m, double fallback_margin_m,
    double band_m, int32_t n_queries, const float *centre_dev,
    const float *radius_dev, const int32_t *slice_dev, double hinge_eps_m,
    float *dist_dev, float *grad_dev, uint8_t *status_dev, float *cost_dev,
    uint8_t *used_fallback_dev, int32_t *rows_dev, void *stream);

/* Kernel timing for measurement.  When on, the kernels of the planar
 * fields, the composite and the sphere queries (PCSDF_KERNEL_PLANES,
 * _COMPOSITE, _QUERY) are each timed by their own dispatch
 * (hipExtLaunchKernel's start and stop events), which adds no packets
 * between kernels, and a region's time is the sum of its kernels'
 * durations; these are not timed while the stream is being captured.
 * The other regions are bracketed by two hipEventRecord calls on the
 * launch stream.  pcsdf_profile_read waits for the events and returns
 * the accumulated milliseconds and region count (calls) of one id.
 * pcsdf_profile_enable(h, 0) stops recording; pcsdf_profile_reset clears
 * the totals (waiting for pending events first). */
int pcsdf_profile_enable(pcsdf_handle *h, int on);
/* Times only the regions whose bit (1 << PCSDF_KERNEL_<id>) is set in
 * region_mask; pcsdf_profile_enable(h, 1) sets every bit, (h, 0) none.
 * A timed kernel costs the stream a few microseconds of idle time before
 * it, so a measurement of whole steps selects only what it reads.
 * PCSDF_ERR_INVALID_ARG for bits at or beyond PCSDF_KERNEL_COUNT. */
int pcsdf_profile_select(pcsdf_handle *h, uint32_t region_mask);
int pcsdf_profile_read(pcsdf_handle *h, int kernel_id, double *total_ms,
                       int64_t *count);
int pcsdf_profile_reset(pcsdf_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* PCSDF_H_ */
