// C-ABI of the surrogate MLP: parameters, forward with input gradient,
// full gradients and the Adam training step.  Kernels in mlp_kernels.h.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mlp_fused.h"
#include "mlp_kernels.h"

namespace pcsdf {

constexpr int kChunk = 1024;  // rows per weight-gradient chunk
// 32-row blocks per wave in fused inference: 2 fits two workgroups per CU
// (70 KB of LDS each), 4 halves the weight reads per row.
constexpr int kInferRowBlocks = 2;
constexpr int kWofs[5] = {0, 4096, 20480, 36864, 53248};
constexpr int kWbfTotal = 53376;

struct Mlp {
  Handle *h = nullptr;
  int n_in = 0;    // inputs per row, 1..kInPad
  int nparam = 0;  // mlp_nparam(n_in)
  DevBuf params, grad, m1, m2, wbf, wtbf, norm, wofs;
  float out_scale = 1.f;
  int64_t step = 0;  // Adam steps taken
  // workspace, grown with the batch
  int cap = 0;
  DevBuf a0, act, dact, dz, seed, y, wpart, bpart, lpart;
};

static int ws(Mlp *m, int npad, hipStream_t s) {
  Handle *h = m->h;
  if (npad <= m->cap) return PCSDF_OK;
  const size_t r = (size_t)npad;
  int rc;
  if ((rc = ensure_buffer(h, m->a0, r * kInPad * 2, s)) ||
      (rc = ensure_buffer(h, m->act, 4 * r * kHid * 2, s)) ||
      (rc = ensure_buffer(h, m->dact, 4 * r * kHid * 2, s)) ||
      (rc = ensure_buffer(h, m->dz, 4 * r * kHid * 2, s)) ||
      (rc = ensure_buffer(h, m->seed, r * 4, s)) ||
      (rc = ensure_buffer(h, m->y, r * 4, s)) ||
      (rc = ensure_buffer(h, m->wpart, (r / kChunk) * kHid * kHid * 4, s)) ||
      (rc = ensure_buffer(h, m->bpart, (r / kChunk) * (kHid + 1) * 4, s)) ||
      (rc = ensure_buffer(h, m->lpart, (r / 256 + 1) * 4, s)))
    return rc;
  m->cap = npad;
  return PCSDF_OK;
}

static uint16_t *actp(Mlp *m, int l) {  // A_l, l = 1..4, [cap][128]
  return reinterpret_cast<uint16_t *>(m->act.ptr) + (size_t)(l - 1) * m->cap * kHid;
}
static uint16_t *dp(Mlp *m, int l) {  // D_l, l = 0..3
  return reinterpret_cast<uint16_t *>(m->dact.ptr) + (size_t)l * m->cap * kHid;
}
static uint16_t *dzp(Mlp *m, int l) {  // dZ_l, l = 0..3
  return reinterpret_cast<uint16_t *>(m->dz.ptr) + (size_t)l * m->cap * kHid;
}
static const uint16_t *wb(Mlp *m, int l) {
  return reinterpret_cast<const uint16_t *>(m->wbf.ptr) + kWofs[l];
}
static const uint16_t *wtb(Mlp *m, int l) {
  return reinterpret_cast<const uint16_t *>(m->wtbf.ptr) + kWofs[l];
}
static int np(const Mlp *m) { return m->nparam; }
static const float *pf(Mlp *m) {
  return reinterpret_cast<const float *>(m->params.ptr);
}

static unsigned blocks(int64_t n, int per) {
  return (unsigned)((n + per - 1) / per);
}

// Sums the chunk partials of one layer's weight gradient into the flat
// gradient vector: W [out][in] from part [chunks][out][in_pad].
__global__ __launch_bounds__(256) void k_sum_w(const float *__restrict__ part,
                                               int chunks, int out, int in,
                                               int in_pad,
                                               float *__restrict__ g) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= out * in) return;
  const int o = t / in, i = t - o * in;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c)
    s += part[((int64_t)c * out + o) * in_pad + i];
  g[t] = s;
}

__global__ void k_fill(float *p, float v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_copy_pad(const float *__restrict__ src, int n, int npad,
                           float *__restrict__ dst) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < npad) dst[t] = t < n ? src[t] : 0.f;
}

__global__ void k_loss_final(const float *__restrict__ part, int nparts,
                             float inv_n, float *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += part[i];
    out[0] = s * inv_n;
  }
}

// Forward pass over rows [0, npad): activations and SiLU derivatives of
// every hidden layer in the workspace; y [n] if given.
static int forward(Mlp *m, int n, int npad, const float *x, float *y,
                   hipStream_t s) {
  const float *norm = reinterpret_cast<const float *>(m->norm.ptr);
  uint16_t *a0 = reinterpret_cast<uint16_t *>(m->a0.ptr);
  hipLaunchKernelGGL(k_mlp_input, dim3(blocks((int64_t)npad * kInPad, 256)),
                     dim3(256), 0, s, x, n, npad, m->n_in, norm,
                     norm + kInPad, a0);
  const float *p = pf(m);
  const unsigned g = (unsigned)(npad / 128);
  const int ni = m->n_in;
  hipLaunchKernelGGL(k_mlp_fwd<kInPad>, dim3(g), dim3(256), 0, s, a0,
                     wb(m, 0), p + layer_desc(0, ni).b_off, actp(m, 1),
                     dp(m, 0));
  for (int l = 1; l < kLayers; ++l)
    hipLaunchKernelGGL(k_mlp_fwd<kHid>, dim3(g), dim3(256), 0, s, actp(m, l),
                       wb(m, l), p + layer_desc(l, ni).b_off, actp(m, l + 1),
                       dp(m, l));
  if (y)
    hipLaunchKernelGGL(k_mlp_out, dim3(blocks(n, 256)), dim3(256), 0, s,
                       actp(m, 4), wb(m, 4), p + layer_desc(4, ni).b_off,
                       m->out_scale, n, y);
  return check_launch(m->h, "mlp forward");
}

// Backward pass from seed [npad] (dLoss/dy, zero on padded rows).  With
// gp, writes the parameter gradient; with grad_x, the input gradient.
static int backward(Mlp *m, int n, int npad, float *gp, float *grad_x,
                    hipStream_t s) {
  const float *norm = reinterpret_cast<const float *>(m->norm.ptr);
  const float *seed = reinterpret_cast<const float *>(m->seed.ptr);
  float *wpart = reinterpret_cast<float *>(m->wpart.ptr);
  float *bpart = reinterpret_cast<float *>(m->bpart.ptr);
  const int chunks = npad / kChunk;
  const unsigned g = (unsigned)(npad / 128);
  const int ni = m->n_in;
  if (gp) {
    hipLaunchKernelGGL(k_mlp_wgrad_out, dim3(chunks), dim3(256), 0, s, seed,
                       m->out_scale, actp(m, 4), n, bpart);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, bpart, chunks,
                       kHid + 1, gp + layer_desc(4, ni).w_off);
  }
  hipLaunchKernelGGL(k_mlp_bwd_out, dim3(blocks((int64_t)npad * kHid, 256)),
                     dim3(256), 0, s, seed, m->out_scale, wb(m, 4), dp(m, 3),
                     npad, dzp(m, 3));
  for (int l = kLayers - 1; l >= 0; --l) {
    const LayerDesc d = layer_desc(l, ni);
    if (gp) {
      const uint16_t *A = l == 0 ? reinterpret_cast<const uint16_t *>(m->a0.ptr)
                                 : actp(m, l);
      if (l == 0)
        hipLaunchKernelGGL(k_mlp_wgrad<kInPad>, dim3(chunks), dim3(256), 0, s,
                           dzp(m, 0), A, wpart, bpart);
      else
        hipLaunchKernelGGL(k_mlp_wgrad<kHid>, dim3(chunks), dim3(256), 0, s,
                           dzp(m, l), A, wpart, bpart);
      hipLaunchKernelGGL(k_sum_w, dim3(blocks(kHid * d.in, 256)), dim3(256), 0,
                         s, wpart, chunks, kHid, d.in, d.in_pad,
                         gp + d.w_off);
      hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, bpart, chunks,
                         kHid, gp + d.b_off);
    }
    if (l > 0)
      hipLaunchKernelGGL(k_mlp_bwd<kHid>, dim3(g), dim3(256), 0, s, dzp(m, l),
                         wtb(m, l), dp(m, l - 1), dzp(m, l - 1),
                         norm + kInPad, n, ni, nullptr);
    else if (grad_x)
      hipLaunchKernelGGL(k_mlp_bwd<kInPad>, dim3(g), dim3(256), 0, s,
                         dzp(m, 0), wtb(m, 0), nullptr, nullptr,
                         norm + kInPad, n, ni, grad_x);
  }
  return check_launch(m->h, "mlp backward");
}

static int check_rows(Mlp *m, int n, const void *x) {
  if (n < 0 || n > (1 << 28))
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "n must be in [0, 2^28]");
  if (n > 0 && !x) return fail(m->h, PCSDF_ERR_INVALID_ARG, "x is NULL");
  return PCSDF_OK;
}

static int pad_rows(int n) { return ((n + kChunk - 1) / kChunk) * kChunk; }

// Fused inference (value and input gradient) of rows [0, n) (with n_dev,
// [0, min(n, *n_dev)) read on the device): one workgroup per tile of
// 32 * kInferRowBlocks rows, at most 2048 workgroups striding over tiles.
static int mlp_infer(Mlp *m, int n, const int *n_dev, const float *x,
                     float *y, float *gx, hipStream_t s) {
  NetWeights w;
  for (int l = 0; l <= kLayers; ++l) w.W[l] = wb(m, l);
  for (int l = 0; l < kLayers; ++l) w.Wt[l] = wtb(m, l);
  constexpr int RB = kInferRowBlocks;
  const int tiles = (n + 32 * RB - 1) / (32 * RB);
  const int grid = tiles < 2048 ? tiles : 2048;
  if (grid == 0) return PCSDF_OK;
  hipLaunchKernelGGL(k_mlp_infer<RB>, dim3(grid), dim3(256), 0, s, x, n,
                     n_dev, m->n_in,
                     reinterpret_cast<const float *>(m->norm.ptr), w, pf(m),
                     m->out_scale, y, gx);
  return check_launch(m->h, "mlp inference");
}

}  // namespace pcsdf

using namespace pcsdf;

struct pcsdf_mlp : Mlp {};

Handle *pcsdf::mlp_handle(pcsdf_mlp *m) { return m ? m->h : nullptr; }
int pcsdf::mlp_inputs(const pcsdf_mlp *m) { return m ? m->n_in : 0; }
int pcsdf::mlp_rows(pcsdf_mlp *m, int n, const int32_t *n_dev,
                    const float *x, float *y, float *gx, hipStream_t s) {
  return mlp_infer(m, n, n_dev, x, y, gx, s);
}

extern "C" int pcsdf_mlp_param_count(int32_t n_in) {
  return n_in >= 1 && n_in <= kInPad ? mlp_nparam(n_in) : -1;
}

extern "C" int pcsdf_mlp_create(pcsdf_handle *hp, int32_t n_in,
                                pcsdf_mlp **out) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  if (!out) return fail(h, PCSDF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || n_in > kInPad)
    return fail(h, PCSDF_ERR_INVALID_ARG, "n_in must be in [1, 32]");
  int rc;
  if ((rc = bind_device(h))) return rc;
  pcsdf_mlp *m = new (std::nothrow) pcsdf_mlp();
  if (!m) return fail(h, PCSDF_ERR_OOM, "mlp allocation failed");
  m->h = h;
  m->n_in = n_in;
  m->nparam = mlp_nparam(n_in);
  const size_t P = (size_t)m->nparam * 4;
  if ((rc = ensure_buffer(h, m->params, P, nullptr)) ||
      (rc = ensure_buffer(h, m->grad, P, nullptr)) ||
      (rc = ensure_buffer(h, m->m1, P, nullptr)) ||
      (rc = ensure_buffer(h, m->m2, P, nullptr)) ||
      (rc = ensure_buffer(h, m->wbf, kWbfTotal * 2, nullptr)) ||
      (rc = ensure_buffer(h, m->wtbf, kWbfTotal * 2, nullptr)) ||
      (rc = ensure_buffer(h, m->norm, 2 * kInPad * 4, nullptr)) ||
      (rc = ensure_buffer(h, m->wofs, 5 * 4, nullptr))) {
    pcsdf_mlp_destroy(m);
    return rc;
  }
  if (hipMemset(m->wbf.ptr, 0, m->wbf.bytes) != hipSuccess ||
      hipMemset(m->wtbf.ptr, 0, m->wtbf.bytes) != hipSuccess ||
      hipMemcpy(m->wofs.ptr, kWofs, sizeof(kWofs), hipMemcpyHostToDevice) !=
          hipSuccess) {
    pcsdf_mlp_destroy(m);
    return fail(h, PCSDF_ERR_HIP, "mlp initialisation failed");
  }
  *out = m;
  return PCSDF_OK;
}

extern "C" void pcsdf_mlp_destroy(pcsdf_mlp *m) {
  if (!m) return;
  DevBuf *bufs[] = {&m->params, &m->grad, &m->m1,   &m->m2,    &m->wbf,
                    &m->wtbf,   &m->norm, &m->wofs, &m->a0,    &m->act,
                    &m->dact,   &m->dz,   &m->seed, &m->y,     &m->wpart,
                    &m->bpart,  &m->lpart};
  bool any = false;
  for (DevBuf *b : bufs) any = any || b->ptr;
  if (any) (void)hipDeviceSynchronize();
  for (DevBuf *b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  delete m;
}

extern "C" int pcsdf_mlp_set_params(pcsdf_mlp *m, const float *params_host,
                                    const float *in_offset_host,
                                    const float *in_scale_host,
                                    float out_scale) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  Handle *h = m->h;
  if (!params_host || !in_offset_host || !in_scale_host)
    return fail(h, PCSDF_ERR_INVALID_ARG, "params, offset and scale required");
  const int P = np(m), ni = m->n_in;
  for (int i = 0; i < P; ++i)
    if (!std::isfinite(params_host[i]))
      return fail(h, PCSDF_ERR_NUMERIC,
                  "non-finite parameter at index " + std::to_string(i));
  for (int i = 0; i < ni; ++i)
    if (!std::isfinite(in_offset_host[i]) || !std::isfinite(in_scale_host[i]))
      return fail(h, PCSDF_ERR_NUMERIC, "non-finite normalisation");
  if (!std::isfinite(out_scale))
    return fail(h, PCSDF_ERR_NUMERIC, "non-finite output scale");
  // [offset 32][scale 32]; padding columns read offset 0, scale 1
  std::vector<float> norm(2 * kInPad, 0.f);
  std::fill(norm.begin() + kInPad, norm.end(), 1.f);
  std::memcpy(norm.data(), in_offset_host, (size_t)ni * 4);
  std::memcpy(norm.data() + kInPad, in_scale_host, (size_t)ni * 4);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(m->params.ptr, params_host, (size_t)P * 4,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->norm.ptr, norm.data(), norm.size() * 4,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m1.ptr, 0, (size_t)P * 4) != hipSuccess ||
      hipMemset(m->m2.ptr, 0, (size_t)P * 4) != hipSuccess)
    return fail(h, PCSDF_ERR_HIP, "uploading the parameters failed");
  m->out_scale = out_scale;
  m->step = 0;
  hipLaunchKernelGGL(k_cast_weights, dim3(blocks(P, 256)), dim3(256), 0,
                     nullptr, reinterpret_cast<const float *>(m->params.ptr),
                     reinterpret_cast<uint16_t *>(m->wbf.ptr),
                     reinterpret_cast<uint16_t *>(m->wtbf.ptr),
                     reinterpret_cast<const int *>(m->wofs.ptr), ni);
  if (hipDeviceSynchronize() != hipSuccess)
    return fail(h, PCSDF_ERR_HIP, "casting the weights failed");
  return PCSDF_OK;
}

extern "C" int pcsdf_mlp_get_params(pcsdf_mlp *m, float *params_host) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  if (!params_host) return fail(m->h, PCSDF_ERR_INVALID_ARG, "params NULL");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(params_host, m->params.ptr, (size_t)np(m) * 4,
                hipMemcpyDeviceToHost) != hipSuccess)
    return fail(m->h, PCSDF_ERR_HIP, "reading the parameters failed");
  return PCSDF_OK;
}

// Inference (value and input gradient) runs fused, one workgroup per tile
// of 64 rows (mlp_fused.h); training keeps the layer-by-layer kernels,
// whose stored activations the weight gradients need.
extern "C" int pcsdf_mlp_forward(pcsdf_mlp *m, int32_t n, const float *x_dev,
                                 float *y_dev, float *grad_x_dev,
                                 void *stream) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  int rc = check_rows(m, n, x_dev);
  if (rc || n == 0) return rc;
  if (!y_dev) return fail(m->h, PCSDF_ERR_INVALID_ARG, "y_dev is NULL");
  if (((uintptr_t)x_dev | (uintptr_t)y_dev | (uintptr_t)grad_x_dev) & 3)
    return fail(m->h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(m->h, PCSDF_KERNEL_MLP, s);
  return mlp_infer(m, n, nullptr, x_dev, y_dev, grad_x_dev, s);
}

extern "C" int pcsdf_mlp_gradients(pcsdf_mlp *m, int32_t n,
                                   const float *x_dev, const float *dy_dev,
                                   float *grad_params_dev, float *grad_x_dev,
                                   void *stream) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  int rc = check_rows(m, n, x_dev);
  if (rc) return rc;
  if (n == 0 || !dy_dev || !grad_params_dev)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "need n > 0, dy and grad");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int npad = pad_rows(n);
  if ((rc = ws(m, npad, s))) return rc;
  if ((rc = forward(m, n, npad, x_dev, nullptr, s))) return rc;
  hipLaunchKernelGGL(k_copy_pad, dim3(blocks(npad, 256)), dim3(256), 0, s,
                     dy_dev, n, npad, reinterpret_cast<float *>(m->seed.ptr));
  return backward(m, n, npad, grad_params_dev, grad_x_dev, s);
}

// dLoss/dparams of the mean squared error into gp [nparam] (and the loss
// into loss_dev): the forward pass, k_mse's seed and the backward pass.
static int loss_gradients(Mlp *m, int n, const float *x_dev,
                          const float *target_dev, float *gp,
                          float *loss_dev, hipStream_t s) {
  const int npad = pad_rows(n);
  int rc;
  if ((rc = ws(m, npad, s))) return rc;
  float *y = reinterpret_cast<float *>(m->y.ptr);
  if ((rc = forward(m, n, npad, x_dev, y, s))) return rc;
  float *lpart = reinterpret_cast<float *>(m->lpart.ptr);
  hipLaunchKernelGGL(k_mse, dim3(blocks(npad, 256)), dim3(256), 0, s, y,
                     target_dev, n, npad,
                     reinterpret_cast<float *>(m->seed.ptr), lpart);
  if (loss_dev)
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, lpart,
                       (int)blocks(npad, 256), 1.f / (float)n, loss_dev);
  return backward(m, n, npad, gp, nullptr, s);
}

// One bias-corrected Adam step from the gradient g (device, fp32
// [nparam]); the step counter advances first, so the first step uses
// c1 = 1 - beta1, c2 = 1 - beta2.
static int adam(Mlp *m, const float *g, float lr, float beta1, float beta2,
                float eps, hipStream_t s) {
  m->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)m->step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks(np(m), 256)), dim3(256), 0, s,
                     reinterpret_cast<float *>(m->params.ptr), g,
                     reinterpret_cast<float *>(m->m1.ptr),
                     reinterpret_cast<float *>(m->m2.ptr), lr, beta1, beta2,
                     eps, c1, c2, reinterpret_cast<uint16_t *>(m->wbf.ptr),
                     reinterpret_cast<uint16_t *>(m->wtbf.ptr),
                     reinterpret_cast<const int *>(m->wofs.ptr), m->n_in);
  return check_launch(m->h, "mlp adam step");
}

static int check_adam(Mlp *m, float lr, float beta1, float beta2, float eps) {
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
      !(eps > 0) || !std::isfinite(lr) || !std::isfinite(eps))
    return fail(m->h, PCSDF_ERR_NUMERIC, "bad optimiser hyper-parameters");
  return PCSDF_OK;
}

extern "C" int pcsdf_mlp_loss_gradients(pcsdf_mlp *m, int32_t n,
                                        const float *x_dev,
                                        const float *target_dev,
                                        float *grad_params_dev,
                                        float *loss_dev, void *stream) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  int rc = check_rows(m, n, x_dev);
  if (rc) return rc;
  if (n == 0 || !target_dev || !grad_params_dev)
    return fail(m->h, PCSDF_ERR_INVALID_ARG,
                "need n > 0, targets and a gradient buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (((uintptr_t)x_dev | (uintptr_t)target_dev | (uintptr_t)grad_params_dev |
       (uintptr_t)loss_dev) & 3)
    return fail(m->h, PCSDF_ERR_ALIGN, "device buffers must be 4-byte aligned");
  return loss_gradients(m, n, x_dev, target_dev, grad_params_dev, loss_dev,
                        s);
}

extern "C" int pcsdf_mlp_adam_step(pcsdf_mlp *m, const float *grad_params_dev,
                                   float lr, float beta1, float beta2,
                                   float eps, void *stream) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  if (!grad_params_dev)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "gradient is NULL");
  if ((uintptr_t)grad_params_dev & 3)
    return fail(m->h, PCSDF_ERR_ALIGN, "gradient must be 4-byte aligned");
  int rc;
  if ((rc = check_adam(m, lr, beta1, beta2, eps))) return rc;
  return adam(m, grad_params_dev, lr, beta1, beta2, eps,
              reinterpret_cast<hipStream_t>(stream));
}

extern "C" int pcsdf_mlp_train_step(pcsdf_mlp *m, int32_t n,
                                    const float *x_dev,
                                    const float *target_dev, float lr,
                                    float beta1, float beta2, float eps,
                                    float *loss_dev, void *stream) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  int rc = check_rows(m, n, x_dev);
  if (rc) return rc;
  if (n == 0 || !target_dev)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "need n > 0 and targets");
  if ((rc = check_adam(m, lr, beta1, beta2, eps))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(m->h, PCSDF_KERNEL_MLP_TRAIN, s);
  float *gp = reinterpret_cast<float *>(m->grad.ptr);
  if ((rc = loss_gradients(m, n, x_dev, target_dev, gp, loss_dev, s)))
    return rc;
  return adam(m, gp, lr, beta1, beta2, eps, s);
}

extern "C" int pcsdf_mlp_get_state(pcsdf_mlp *m, float *params_host,
                                   float *m1_host, float *m2_host,
                                   int64_t *step) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  if (!params_host || !m1_host || !m2_host || !step)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "every output is required");
  const size_t P = (size_t)np(m) * 4;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(params_host, m->params.ptr, P, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(m1_host, m->m1.ptr, P, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m2_host, m->m2.ptr, P, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(m->h, PCSDF_ERR_HIP, "reading the optimiser state failed");
  *step = m->step;
  return PCSDF_OK;
}

extern "C" int pcsdf_mlp_set_state(pcsdf_mlp *m, const float *params_host,
                                   const float *m1_host, const float *m2_host,
                                   int64_t step, const float *in_offset_host,
                                   const float *in_scale_host,
                                   float out_scale) {
  if (!m) return PCSDF_ERR_INVALID_ARG;
  if (!m1_host || !m2_host)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "moments are required");
  if (step < 0 || step > (int64_t)1 << 40)
    return fail(m->h, PCSDF_ERR_INVALID_ARG, "step out of range");
  for (int i = 0; i < np(m); ++i)
    if (!std::isfinite(m1_host[i]) || !std::isfinite(m2_host[i]) ||
        m2_host[i] < 0.f)
      return fail(m->h, PCSDF_ERR_NUMERIC,
                  "bad moment at index " + std::to_string(i));
  int rc = pcsdf_mlp_set_params(m, params_host, in_offset_host,
                                in_scale_host, out_scale);
  if (rc) return rc;
  const size_t P = (size_t)np(m) * 4;
  if (hipMemcpy(m->m1.ptr, m1_host, P, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->m2.ptr, m2_host, P, hipMemcpyHostToDevice) != hipSuccess)
    return fail(m->h, PCSDF_ERR_HIP, "uploading the moments failed");
  m->step = step;
  return PCSDF_OK;
}
