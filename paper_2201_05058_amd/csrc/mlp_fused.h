// Fused inference of the surrogate MLP (included by mlp.hip): forward pass
// and input gradient of a tile of 32 RB rows in one workgroup, with no
// intermediate in HBM.
//
// Layout.  Four waves; wave w owns hidden units 32w..32w+31 of every layer
// for all rows of the tile (RB 32-row blocks): in the forward pass as
// its output columns, in the backward pass as the input units whose
// gradient it forms.  The forward output block of layer l and the backward
// output block of layer l+1 therefore cover the same rows and units in the
// same accumulator layout, so each wave keeps its SiLU derivatives D_l
// private from the forward to the backward pass: D_2 and D_3 in registers,
// D_0 and D_1 in LDS (registers would spill).  Activations and
// pre-activation gradients of the whole tile are exchanged through two LDS
// tiles [128][136] (ping-pong).  The weight operand of a wave (its 32 rows
// of W_l, or of W_l^T going backward) is read from the BF16 weight copies
// in global memory: 8 KB per wave and layer, common to all workgroups and
// served by the caches.
//
// The rounding points are those of the layered kernels and of the oracle:
// A_{l+1} = bf16(SiLU(Z_l)), D_l = bf16(SiLU'(Z_l)), dZ_3 = bf16(out_scale
// W4 (.) D_3), dZ_{l-1} = bf16((dZ_l W_l) (.) D_{l-1}); y and the input
// gradient are FP32.  SiLU and SiLU' share one logistic value computed with
// the approximate exponential and reciprocal: the epilogue of a layer is
// VALU work of the same order as the layer's matrix products.
#pragma once

#include "mlp_kernels.h"

namespace pcsdf {

constexpr int kTS = kHid + 8;  // LDS row stride of a tile (bf16 elements)

struct NetWeights {
  const uint16_t *W[kLayers + 1];  // W_l [128][in_pad] (W4: [128])
  const uint16_t *Wt[kLayers];     // W_l^T [in_pad][128]
};

// SiLU and its derivative from one logistic value, with the hardware's
// approximate exponential and reciprocal (a few ulp of fp32; the results
// are rounded to BF16 next, whose unit is 2^16 fp32 ulps).
__device__ __forceinline__ void silu_pair(float z, float *a, float *d) {
  const float e = __expf(-z);
  const float sg = __builtin_amdgcn_rcpf(1.f + e);
  *a = z * sg;
  *d = sg * (1.f + z * (1.f - sg));
}

// Two fp32 values to BF16 by round-to-nearest-even in one hardware
// conversion (the same rounding as to_bf16 for finite values): a in the
// low half, b in the high half.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt2(float a, float b) {
  const f32x2_t v = {a, b};
  const bf16x2_t r = __builtin_convertvector(v, bf16x2_t);
  return __builtin_bit_cast(uint32_t, r);
}

__device__ __forceinline__ uint16_t lo16(uint32_t v) { return (uint16_t)v; }
__device__ __forceinline__ uint16_t hi16(uint32_t v) {
  return (uint16_t)(v >> 16);
}

// acc[rb] = A_tile[rb rows] x B^T for this wave's 32 units: A from LDS
// ([32 RB][kTS], K columns used), B [128][K] in global memory, row `unit`.
template <int K, int RB>
__device__ __forceinline__ void tile_gemm(const uint16_t *a_lds,
                                          const uint16_t *__restrict__ B,
                                          int unit, int lane, f32x16 acc[RB]) {
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[rb][r] = 0.f;
  const uint16_t *brow = B + (size_t)unit * K + 8 * (lane >> 5);
  bf16x8 bv[K / 16];
#pragma unroll
  for (int ks = 0; ks < K / 16; ++ks) bv[ks] = load8(brow + ks * 16);
  const uint16_t *arow = a_lds + (lane & 31) * kTS + 8 * (lane >> 5);
#pragma unroll
  for (int ks = 0; ks < K / 16; ++ks)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
      acc[rb] = mfma(load8(arow + rb * 32 * kTS + ks * 16), bv[ks], acc[rb]);
}

// y [n] and, when gx is given, dy/dx [n][n_in] for rows [0, n), x
// [n][n_in], in tiles of 32 RB rows (RB row blocks per wave).  With n_dev
// the row count is min(n, *n_dev), read on the device (a grid sized for n
// then leaves its surplus workgroups idle).
template <int RB>
__global__ __launch_bounds__(256, RB == 4 ? 1 : 2) void k_mlp_infer(
    const float *__restrict__ x, int n, const int *__restrict__ n_dev,
    int n_in, const float *__restrict__ norm, NetWeights w,
    const float *__restrict__ p, float out_scale, float *__restrict__ y,
    float *__restrict__ gx) {
  constexpr int kTileRows = 32 * RB;
  __shared__ uint16_t tl[2][kTileRows * kTS];
  __shared__ uint16_t dl[2][kTileRows * kTS];  // D_0, D_1
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int unit = wave * 32 + (lane & 31);
  const float *off = norm, *scale = norm + kInPad;
  if (n_dev) n = min(n, *n_dev);
  const int tiles = (n + kTileRows - 1) / kTileRows;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row0 = (int64_t)tile * kTileRows;
    // A0 = bf16((x - offset) * scale), zero beyond n_in columns and n rows
    for (int t = threadIdx.x; t < kTileRows * kInPad; t += 256) {
      const int r = t / kInPad, c = t - r * kInPad;
      const int64_t m = row0 + r;
      tl[0][r * kTS + c] =
          (c < n_in && m < n)
              ? to_bf16((x[m * n_in + c] - off[c]) * scale[c])
              : (uint16_t)0;
    }
    __syncthreads();
    uint32_t D[2][RB][8];  // bf16 SiLU' of layers 2, 3 for this wave, 2 a word
    f32x16 acc[RB];
    // forward: layer l reads tile l&1 and writes tile (l+1)&1
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      if (l == 0)
        tile_gemm<kInPad, RB>(tl[0], w.W[0], unit, lane, acc);
      else
        tile_gemm<kHid, RB>(tl[l & 1], w.W[l], unit, lane, acc);
      uint16_t *aout = tl[(l + 1) & 1];
      const float bias = p[layer_desc(l, n_in).b_off + unit];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int row = rb * 32 + acc_row(r, lane);  // r+1: row+1
          float a0, a1, s0, s1;
          silu_pair(acc[rb][r] + bias, &a0, &s0);
          silu_pair(acc[rb][r + 1] + bias, &a1, &s1);
          const uint32_t av = cvt2(a0, a1), dv = cvt2(s0, s1);
          aout[row * kTS + unit] = lo16(av);
          aout[(row + 1) * kTS + unit] = hi16(av);
          if (l < 2) {
            dl[l][row * kTS + unit] = lo16(dv);
            dl[l][(row + 1) * kTS + unit] = hi16(dv);
          } else {
            D[l - 2][rb][r >> 1] = dv;
          }
        }
      __syncthreads();
    }
    // y from A4 (tile 0): two threads per row, 64 units each
    if (threadIdx.x < 2 * kTileRows) {
      const int row = threadIdx.x >> 1, half = threadIdx.x & 1;
      const uint16_t *a = tl[0] + row * kTS + half * 64;
      const uint16_t *w4 = w.W[kLayers] + half * 64;
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < 64; c += 8) {
        const uint4 av = *reinterpret_cast<const uint4 *>(a + c);
        const uint4 wv = *reinterpret_cast<const uint4 *>(w4 + c);
        const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
        const uint32_t ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s += from_bf16(lo16(aw[q])) * from_bf16(lo16(ww[q]));
          s += from_bf16(hi16(aw[q])) * from_bf16(hi16(ww[q]));
        }
      }
      s += __shfl_xor(s, 1);
      const int64_t m = row0 + row;
      if (half == 0 && m < n)
        y[m] = (s + p[layer_desc(kLayers, n_in).b_off]) * out_scale;
    }
    if (gx) {
      // dZ3 = bf16(out_scale W4 (.) D3) into tile 1 (A3 is consumed)
      const float da3 = out_scale * from_bf16(w.W[kLayers][unit]);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int row = rb * 32 + acc_row(r, lane);
          const uint32_t d = D[1][rb][r >> 1];
          const uint32_t zv = cvt2(da3 * from_bf16(lo16(d)),
                                   da3 * from_bf16(hi16(d)));
          tl[1][row * kTS + unit] = lo16(zv);
          tl[1][(row + 1) * kTS + unit] = hi16(zv);
        }
      __syncthreads();
      // dZ_{l-1} = bf16((dZ_l W_l) (.) D_{l-1}): layer l reads tile l&1,
      // writes tile (l+1)&1
#pragma unroll
      for (int l = kLayers - 1; l >= 1; --l) {
        tile_gemm<kHid, RB>(tl[l & 1], w.Wt[l], unit, lane, acc);
        uint16_t *zout = tl[(l + 1) & 1];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int r = 0; r < 16; r += 2) {
            const int row = rb * 32 + acc_row(r, lane);
            uint16_t d0, d1;  // D_{l-1} at (row, unit), (row + 1, unit)
            if (l - 1 >= 2) {
              const uint32_t d = D[l - 3][rb][r >> 1];
              d0 = lo16(d);
              d1 = hi16(d);
            } else {
              d0 = dl[l - 1][row * kTS + unit];
              d1 = dl[l - 1][(row + 1) * kTS + unit];
            }
            const uint32_t zv = cvt2(acc[rb][r] * from_bf16(d0),
                                     acc[rb][r + 1] * from_bf16(d1));
            zout[row * kTS + unit] = lo16(zv);
            zout[(row + 1) * kTS + unit] = hi16(zv);
          }
        __syncthreads();
      }
      // dy/dx = (dZ0 W0) * scale: wave w < RB forms row block w, columns
      // 0..31
      if (wave < RB) {
      f32x16 g;
#pragma unroll
      for (int r = 0; r < 16; ++r) g[r] = 0.f;
      const uint16_t *zrow =
          tl[0] + (wave * 32 + (lane & 31)) * kTS + 8 * (lane >> 5);
      const uint16_t *brow = w.Wt[0] + (size_t)(lane & 31) * kHid +
                             8 * (lane >> 5);
#pragma unroll
      for (int ks = 0; ks < kHid / 16; ++ks)
        g = mfma(load8(zrow + ks * 16), load8(brow + ks * 16), g);
      const int col = lane & 31;
      if (col < n_in) {
        const float sc = scale[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t m = row0 + wave * 32 + acc_row(r, lane);
          if (m < n) gx[m * n_in + col] = g[r] * sc;
        }
      }
      }
    }
    __syncthreads();  // the tiles are reused by the next tile of rows
  }
}

}  // namespace pcsdf
