// Runs the library's device code on the CPU: the planar-field helpers and
// the batch planner with its two persistent workers (OS threads play
// workgroups of one lane).  Input and output files are written and read by
// tests/test_cpu_device_code.py.  Test infrastructure only.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../paper_2201_05058_amd/csrc/batch_plan.h"

thread_local Dim3 threadIdx, blockIdx, blockDim, gridDim;

namespace pcsdf {
// The library's validation helpers live in api.hip (HIP runtime code);
// the planner only needs their error-reporting behaviour here.
int fail(Handle *h, int code, const std::string &m) {
  if (h) h->err = m;
  return code;
}
int check_grid(Handle *h, const pcsdf_grid *g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > 1024 ||
      g->ny > 1024 || g->nz > 1024)
    return fail(h, PCSDF_ERR_DIMS, "grid dimensions");
  return PCSDF_OK;
}
}  // namespace pcsdf
using namespace pcsdf;

template <class T>
static bool rd(FILE *f, T *p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

// mode "planes": nx ny n K R xy -> planes [n][ny][nx]
static int planes(FILE *f, FILE *o) {
  int hdr[4];
  int64_t R;
  if (!rd(f, hdr, 4) || !rd(f, &R, 1)) return 2;
  const int nx = hdr[0], ny = hdr[1], n = hdr[2], K = hdr[3];
  std::vector<int64_t> xy((size_t)n * K * 2);
  if (!rd(f, xy.data(), xy.size())) return 2;
  std::vector<int32_t> P((size_t)nx * ny), F1((size_t)nx * ny);
  for (int s = 0; s < n; ++s) {
    std::vector<int2> ch((size_t)K * ny);
    std::vector<int4> box(K);
    for (int k = 0; k < K; ++k) {
      const int64_t X = xy[2 * ((size_t)s * K + k)];
      const int64_t Y = xy[2 * ((size_t)s * K + k) + 1];
      box[k] = disk_box(X, Y, R, nx, ny);
      for (int j = 0; j < ny; ++j) ch[(size_t)k * ny + j] = disk_chord(X, Y, R, nx, j);
    }
    const GlobalTab tab{ch.data()};
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        F1[(size_t)j * nx + i] = row_free_dist(tab, K, ny, nx, j, i);
    const int4 *bp = box.data();
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        P[(size_t)j * nx + i] = plane_value(tab, bp, F1.data() + i, K, nx, ny, i, j);
    fwrite(P.data(), 4, P.size(), o);
  }
  return 0;
}

// mode "batch": scenes -> composite int32 and fp32 outputs of every scene
static int batch(FILE *f, FILE *o) {
  int ns, nthreads, tune[4];
  if (!rd(f, &ns, 1) || !rd(f, &nthreads, 1) || !rd(f, tune, 4)) return 2;
  std::vector<pcsdf_scene> sc(ns);
  std::vector<std::vector<int32_t>> stat(ns), oc(ns);
  std::vector<std::vector<float>> of(ns);
  std::vector<std::vector<double>> xy(ns);
  for (int q = 0; q < ns; ++q) {
    int d[5];
    double g[6];
    if (!rd(f, d, 5) || !rd(f, g, 6)) return 2;
    pcsdf_grid gr{};
    gr.nx = d[0]; gr.ny = d[1]; gr.nz = d[2]; gr.voxel_m = g[0];
    gr.origin_m[0] = g[1]; gr.origin_m[1] = g[2]; gr.origin_m[2] = g[3];
    const size_t V = (size_t)d[0] * d[1] * d[2];
    xy[q].resize((size_t)d[3] * d[4] * 2);
    stat[q].resize(V);
    if (!rd(f, xy[q].data(), xy[q].size()) || !rd(f, stat[q].data(), V)) return 2;
    oc[q].assign(V * d[3], 12345);
    of[q].assign(V * d[3], -1.f);
    sc[q].grid = gr;
    sc[q].static_ssq_dev = stat[q].data();
    sc[q].n_slices = d[3];
    sc[q].n_humans = d[4];
    sc[q].human_xy_host = d[4] ? xy[q].data() : nullptr;
    sc[q].radius_m = g[4];
    sc[q].height_m = g[5];
    sc[q].out_ssq_dev = oc[q].data();
    sc[q].out_sdf_dev = of[q].data();
  }
  Handle h;
  const pcsdf_tuning tu{tune[0], tune[1], tune[2], tune[3]};
  BatchPlan bp;
  int rc = plan_batch(&h, ns, sc.data(), tu, 1, &bp);
  if (rc) {
    fprintf(stderr, "plan failed: %s\n", h.err.c_str());
    return 1;
  }
  std::vector<char> params(param_layout(bp).total + 256);
  std::vector<char> scratch(plan_scratch(bp) + 256), host;
  char *pbase = (char *)(((uintptr_t)params.data() + 255) & ~(uintptr_t)255);
  char *sbase = (char *)(((uintptr_t)scratch.data() + 255) & ~(uintptr_t)255);
  bind_plan(&bp, sc.data(), pbase, sbase, &host);
  memcpy(pbase, host.data(), host.size());
  const SceneDev *scenes = (const SceneDev *)pbase;
  const int4 *items = (const int4 *)(pbase + param_layout(bp).items);
  const int32_t *scene_of = (const int32_t *)(pbase + param_layout(bp).groups);
  const int np = (int)bp.items.size();
  for (int phase = 0; phase < 2; ++phase) {
    std::vector<std::thread> th;
    for (int b = 0; b < nthreads; ++b)
      th.emplace_back([&, b] {
        threadIdx.x = 0; blockDim.x = 1; blockIdx.x = b; gridDim.x = nthreads;
        std::vector<int4> lds(bp.lds_cap / 16 + 1);
        if (phase == 0)
          batch_planes(scenes, items, np, bp.lds_cap, lds.data());
        else
          batch_composites(scenes, scene_of, bp.composite_items, bp.G,
                           bp.chunk_voxels);
      });
    for (auto &t : th) t.join();
  }
  for (int q = 0; q < ns; ++q) {
    fwrite(oc[q].data(), 4, oc[q].size(), o);
    fwrite(of[q].data(), 4, of[q].size(), o);
  }
  printf("planar items %d composite items %u\n", np, bp.composite_items);
  return 0;
}

int main(int argc, char **argv) {
  if (argc != 4) return 2;
  FILE *f = fopen(argv[2], "rb");
  FILE *o = fopen(argv[3], "wb");
  if (!f || !o) return 2;
  const std::string mode = argv[1];
  const int rc = mode == "planes" ? planes(f, o) : batch(f, o);
  fclose(f);
  fclose(o);
  return rc;
}
