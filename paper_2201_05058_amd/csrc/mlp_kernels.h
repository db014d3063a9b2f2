// Kernels of the surrogate MLP (included by mlp.hip).
#pragma once

// Learned surrogate for sphere queries: an n_in -> 4 x 128 SiLU -> 1 MLP
// (n_in <= 32 inputs, padded to 32 columns) with BF16 operands and FP32
// accumulation on the matrix cores, its input gradient by reverse mode,
// and its training (weight gradients + Adam).
//
// Every product of the network is a dense contraction with one dimension
// of 128, so each layer is one MFMA GEMM over a batch of rows:
//   forward    Z_l  = A_l W_l^T + b_l,   A_{l+1} = bf16(SiLU(Z_l)),
//                                       D_l     = bf16(SiLU'(Z_l));
//   backward   dA_l = dZ_l W_l,          dZ_{l-1} = bf16(dA_l * D_{l-1});
//   weights    dW_l = dZ_l^T A_l (a reduction over the batch).
// The BF16 rounding points are exactly those of the CPU oracle.
//
// Matrix-core tile: v_mfma_f32_32x32x16_bf16.  For a 32-row by 32-column
// output block and a 16-deep slice of the contraction, lane l supplies
// A[row l%32][k 8*(l/32) .. +7] and B[k 8*(l/32) .. +7][col l%32] as eight
// BF16 values each, and receives output element
// (row 8*(r/4) + 4*(l/32) + r%4, col l%32) in accumulator register r.
// Each workgroup of four waves computes 128 rows: wave w owns rows
// 32w..32w+31 of the block and all 128 output columns (four 32-column
// blocks).  The layer's weights are staged in LDS once per workgroup with
// rows padded by 16 bytes so that the 32 lanes reading 32 different rows
// hit different banks.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace pcsdf {

constexpr int kInPad = 32, kHid = 128, kLayers = 4;
// Parameters of a network with n_in inputs: W0 [128][n_in] and the rest.
__host__ __device__ constexpr int mlp_nparam(int n_in) {
  return kHid * n_in + kHid + 3 * (kHid * kHid + kHid) + kHid + 1;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ float silu(float z) { return z / (1.f + expf(-z)); }
__device__ __forceinline__ float silu_prime(float z) {
  const float s = 1.f / (1.f + expf(-z));
  return s * (1.f + z * (1.f - s));
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

// Row index (within the 32-row block) of accumulator register r.
__device__ __forceinline__ int acc_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// ----------------------------------------------------------- forward

// A0 = bf16((x - offset) * scale), x [n][n_in], padded with zeros to 32
// columns and to npad rows.
__global__ __launch_bounds__(256) void k_mlp_input(
    const float *__restrict__ x, int n, int npad, int n_in,
    const float *__restrict__ off, const float *__restrict__ scale,
    uint16_t *__restrict__ a0) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)npad * kInPad) return;
  const int64_t m = t / kInPad;
  const int c = (int)(t - m * kInPad);
  a0[t] = (c < n_in && m < n)
              ? to_bf16((x[m * n_in + c] - off[c]) * scale[c])
              : (uint16_t)0;
}

// Stages a [128][K] bf16 matrix into LDS with row stride K + 8.
template <int K>
__device__ __forceinline__ void stage_rows(const uint16_t *__restrict__ src,
                                           uint16_t *lds) {
  constexpr int S = K + 8;
  for (int t = threadIdx.x; t < kHid * (K / 8); t += blockDim.x) {
    const int r = t / (K / 8), c = (t - r * (K / 8)) * 8;
    *reinterpret_cast<uint4 *>(lds + r * S + c) =
        *reinterpret_cast<const uint4 *>(src + r * K + c);
  }
}

// Hidden layer forward: rows [128*blockIdx.x, +128) of A [M][K] times
// W [128][K]^T plus b; writes A_out [M][128] and D [M][128] (bf16).
// M is a multiple of 128 (the caller pads the batch).
template <int K>
__global__ __launch_bounds__(256) void k_mlp_fwd(
    const uint16_t *__restrict__ A, const uint16_t *__restrict__ W,
    const float *__restrict__ b, uint16_t *__restrict__ Aout,
    uint16_t *__restrict__ D) {
  constexpr int S = K + 8;
  __shared__ uint16_t w[kHid * S];
  stage_rows<K>(W, w);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const uint16_t *arow = A + (row0 + (lane & 31)) * K + 8 * (lane >> 5);
  f32x16 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8 a = load8(arow + k0);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 bv =
          load8(w + (nb * 32 + (lane & 31)) * S + k0 + 8 * (lane >> 5));
      acc[nb] = mfma(a, bv, acc[nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int col = nb * 32 + (lane & 31);
    const float bias = b[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + acc_row(r, lane);
      const float z = acc[nb][r] + bias;
      Aout[row * kHid + col] = to_bf16(silu(z));
      D[row * kHid + col] = to_bf16(silu_prime(z));
    }
  }
}

// Output layer: y = (A4 . W4 + b4) * out_scale, one lane per row.
__global__ __launch_bounds__(256) void k_mlp_out(
    const uint16_t *__restrict__ A4, const uint16_t *__restrict__ W4,
    const float *__restrict__ b4, float out_scale, int n,
    float *__restrict__ y) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= n) return;
  const uint16_t *a = A4 + (int64_t)m * kHid;
  float s = 0.f;
  for (int c = 0; c < kHid; c += 8) {
    const uint4 av = *reinterpret_cast<const uint4 *>(a + c);
    const uint4 wv = *reinterpret_cast<const uint4 *>(W4 + c);
    const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
    const uint32_t ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s += from_bf16((uint16_t)(aw[q] & 0xFFFF)) *
           from_bf16((uint16_t)(ww[q] & 0xFFFF));
      s += from_bf16((uint16_t)(aw[q] >> 16)) *
           from_bf16((uint16_t)(ww[q] >> 16));
    }
  }
  y[m] = (s + b4[0]) * out_scale;
}

// ----------------------------------------------------------- backward

// dZ3 = bf16(seed[m] * out_scale * W4 (.) D3): the gradient entering the
// last hidden layer, seed = dLoss/dy (or 1 for the input gradient).
__global__ __launch_bounds__(256) void k_mlp_bwd_out(
    const float *__restrict__ seed, float out_scale,
    const uint16_t *__restrict__ W4, const uint16_t *__restrict__ D3, int n,
    uint16_t *__restrict__ dZ3) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * kHid) return;
  const int64_t m = t / kHid;
  const int c = (int)(t - m * kHid);
  const float da = seed[m] * out_scale * from_bf16(W4[c]);
  dZ3[t] = to_bf16(da * from_bf16(D3[t]));
}

// Hidden layer backward: dA [rows][KO] = dZ [rows][128] * W [128][KO],
// with Wt = W^T [KO][128] staged in LDS.  If Dp is given the result is
// dZ_prev = bf16(dA (.) Dp) [M][KO]; otherwise dA is the gradient of the
// normalised input and grad_x[m][c] = dA[m][c] * scale[c] for c < n_in.
template <int KO>
__global__ __launch_bounds__(256) void k_mlp_bwd(
    const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ Wt,
    const uint16_t *__restrict__ Dp, uint16_t *__restrict__ dZp,
    const float *__restrict__ scale, int n, int n_in,
    float *__restrict__ grad_x) {
  constexpr int S = kHid + 8;
  __shared__ uint16_t w[KO * S];
  for (int t = threadIdx.x; t < KO * (kHid / 8); t += blockDim.x) {
    const int r = t / (kHid / 8), c = (t - r * (kHid / 8)) * 8;
    *reinterpret_cast<uint4 *>(w + r * S + c) =
        *reinterpret_cast<const uint4 *>(Wt + r * kHid + c);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 128 + wave * 32;
  const uint16_t *zrow = dZ + (row0 + (lane & 31)) * kHid + 8 * (lane >> 5);
  constexpr int NB = KO / 32;
  f32x16 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
#pragma unroll
  for (int k0 = 0; k0 < kHid; k0 += 16) {
    const bf16x8 a = load8(zrow + k0);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 bv =
          load8(w + (nb * 32 + (lane & 31)) * S + k0 + 8 * (lane >> 5));
      acc[nb] = mfma(a, bv, acc[nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = nb * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + acc_row(r, lane);
      if (Dp) {
        dZp[row * KO + col] =
            to_bf16(acc[nb][r] * from_bf16(Dp[row * KO + col]));
      } else if (col < n_in && row < n) {
        grad_x[row * n_in + col] = acc[nb][r] * scale[col];
      }
    }
  }
}

// Weight gradient of one layer over a chunk of 1024 rows:
// part[chunk][o][i] = sum_m dZ[m][o] A[m][i] (fp32), part_b[chunk][o] =
// sum_m dZ[m][o].  Rows of the chunk beyond n are zero in dZ (the caller
// pads with zero gradients), so they contribute nothing.  16-row slices
// of dZ and A are staged transposed in LDS so that the lane fragments
// (eight consecutive rows of one column) are contiguous.
template <int K>
__global__ __launch_bounds__(256) void k_mlp_wgrad(
    const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ A,
    float *__restrict__ part, float *__restrict__ part_b) {
  constexpr int TS = 16 + 8;  // transposed tile row stride (16 rows + pad)
  __shared__ uint16_t zt[kHid * TS];
  __shared__ uint16_t at[K * TS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 1024;
  constexpr int NB = K / 32;
  f32x16 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
  float bs = 0.f;  // thread t < 128 sums column t of dZ
  for (int s = 0; s < 1024; s += 16) {
    __syncthreads();
    for (int t = threadIdx.x; t < 16 * kHid; t += blockDim.x) {
      const int m = t / kHid, o = t - m * kHid;
      const uint16_t v = dZ[(r0 + s + m) * kHid + o];
      zt[o * TS + m] = v;
    }
    for (int t = threadIdx.x; t < 16 * K; t += blockDim.x) {
      const int m = t / K, i = t - m * K;
      at[i * TS + m] = A[(r0 + s + m) * K + i];
    }
    __syncthreads();
    if (threadIdx.x < kHid)
      for (int m = 0; m < 16; ++m) bs += from_bf16(zt[threadIdx.x * TS + m]);
    const bf16x8 a =
        load8(zt + (wave * 32 + (lane & 31)) * TS + 8 * (lane >> 5));
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 bv =
          load8(at + (nb * 32 + (lane & 31)) * TS + 8 * (lane >> 5));
      acc[nb] = mfma(a, bv, acc[nb]);
    }
  }
  float *p = part + (int64_t)blockIdx.x * kHid * K;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = nb * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = wave * 32 + acc_row(r, lane);
      p[o * K + col] = acc[nb][r];
    }
  }
  if (threadIdx.x < kHid) part_b[(int64_t)blockIdx.x * kHid + threadIdx.x] = bs;
}

// Output layer gradients over chunks of 1024 rows: part[chunk][c] =
// sum_m s[m] A4[m][c] for c < 128 and part[chunk][128] = sum_m s[m], with
// s = seed * out_scale.
__global__ __launch_bounds__(256) void k_mlp_wgrad_out(
    const float *__restrict__ seed, float out_scale,
    const uint16_t *__restrict__ A4, int n, float *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * 1024;
  const int c = threadIdx.x;
  if (c > kHid) return;
  float acc = 0.f;
  for (int m = 0; m < 1024; ++m) {
    const int64_t row = r0 + m;
    if (row >= n) break;
    const float s = seed[row] * out_scale;
    acc += c < kHid ? s * from_bf16(A4[row * kHid + c]) : s;
  }
  part[(int64_t)blockIdx.x * (kHid + 1) + c] = acc;
}

// Sums `chunks` partial vectors of length len (fixed order, deterministic).
__global__ __launch_bounds__(256) void k_sum_parts(
    const float *__restrict__ part, int chunks, int len,
    float *__restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * len + i];
  out[i] = s;
}

// ----------------------------------------------------------- training

// Mean squared error: seed[m] = 2 (y[m] - t[m]) / n (zero for padded
// rows) and per-block partial sums of the squared residual.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y,
                                             const float *__restrict__ tgt,
                                             int n, int npad,
                                             float *__restrict__ seed,
                                             float *__restrict__ part) {
  __shared__ float red[256];
  const int m = blockIdx.x * 256 + threadIdx.x;
  float r2 = 0.f;
  if (m < npad) {
    float g = 0.f;
    if (m < n) {
      const float r = y[m] - tgt[m];
      g = 2.f * r / (float)n;
      r2 = r * r;
    }
    seed[m] = g;
  }
  red[threadIdx.x] = r2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Per-layer geometry of the flat parameter vector.
struct LayerDesc {
  int w_off, b_off, out, in, in_pad;
};
__host__ __device__ inline LayerDesc layer_desc(int l, int n_in) {
  // W0[128][n_in] b0 W1 b1 W2 b2 W3 b3 W4[1][128] b4
  const int sizes_in[5] = {n_in, kHid, kHid, kHid, kHid};
  const int sizes_out[5] = {kHid, kHid, kHid, kHid, 1};
  int off = 0;
  for (int q = 0; q < l; ++q) off += sizes_out[q] * sizes_in[q] + sizes_out[q];
  LayerDesc d;
  d.w_off = off;
  d.b_off = off + sizes_out[l] * sizes_in[l];
  d.out = sizes_out[l];
  d.in = sizes_in[l];
  d.in_pad = l == 0 ? kInPad : sizes_in[l];
  return d;
}

// Adam on the fp32 masters, then refresh the BF16 weights W_l [out][in_pad]
// and their transposes Wt_l [in_pad][out] (padding columns stay zero).
__global__ __launch_bounds__(256) void k_adam(
    float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
    float *__restrict__ m2, float lr, float b1, float b2, float eps,
    float c1, float c2, uint16_t *__restrict__ wbf, uint16_t *__restrict__ wtbf,
    const int *__restrict__ wofs, int n_in) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= mlp_nparam(n_in)) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  const float th = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
  p[i] = th;
  for (int l = 0; l <= kLayers; ++l) {
    const LayerDesc d = layer_desc(l, n_in);
    if (i >= d.w_off && i < d.b_off) {
      const int o = (i - d.w_off) / d.in, c = (i - d.w_off) - o * d.in;
      const uint16_t hb = to_bf16(th);
      wbf[wofs[l] + o * d.in_pad + c] = hb;
      if (l < kLayers) wtbf[wofs[l] + c * d.out + o] = hb;
    }
  }
}

// BF16 copies of every weight matrix from the fp32 masters.
__global__ __launch_bounds__(256) void k_cast_weights(
    const float *__restrict__ p, uint16_t *__restrict__ wbf,
    uint16_t *__restrict__ wtbf, const int *__restrict__ wofs, int n_in) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= mlp_nparam(n_in)) return;
  for (int l = 0; l <= kLayers; ++l) {
    const LayerDesc d = layer_desc(l, n_in);
    if (i >= d.w_off && i < d.b_off) {
      const int o = (i - d.w_off) / d.in, c = (i - d.w_off) - o * d.in;
      const uint16_t hb = to_bf16(p[i]);
      wbf[wofs[l] + o * d.in_pad + c] = hb;
      if (l < kLayers) wtbf[wofs[l] + c * d.out + o] = hb;
    }
  }
}

}  // namespace pcsdf
