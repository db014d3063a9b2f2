// Exact separable squared Euclidean distance transform on gfx950.
//
// The environment field of the mapping section (computed once for the
// static map) and the humans' planar fields are both exact signed squared
// EDTs.  Squared distance is a sum of per-axis terms, so the transform is
// three 1-D passes; the x pass finds the nearest voxel of the other type
// along each row, and every later pass takes the lower envelope of
// parabolas g(q) = min_p f(p) + (q - p)^2 along its axis.
//
// Both channels travel in one signed int32 array.  Between passes a free
// voxel holds +f_O (partial squared distance to the occupied set, >= 1)
// and an occupied voxel holds -f_F (partial squared distance to the free
// set, <= -1); +-kInf mean "no such voxel yet".  For the occupied-set
// channel an occupied voxel is a site of value 0, and for the free-set
// channel a free voxel is; so each channel's sites are recoverable from
// the one array and the sign of every voxel never changes.
//
// Layout and mapping (CDNA4, wave64):
//   - x pass: one wave per row; occupancy of 64 voxels at a time is a
//     wave ballot, and nearest-left / nearest-right indices come from
//     count-leading / trailing-zeros of the masked ballot with a carry
//     across chunks.  No LDS.
//   - y and z passes: lanes run along x, so every step of a column sweep is
//     one coalesced load of adjacent columns, and no transpose is needed
//     because x is the contiguous axis.  On the static build the occupied
//     set's channel (every free voxel's value) is a lower envelope per
//     column, split into segments with one wave each (k_pass_col_seg), and
//     the free set's channel, needed only at the occupied voxels, is a
//     bounded search over groups of rows (k_pass_col_inside).  Envelope
//     stacks live in LDS laid out [depth][lane] so a wave's accesses spread
//     over all banks, and intersections are compared by cross-multiplication,
//     so the envelope has no division.  Columns too long for the segmented
//     kernel's LDS run both channels in one wave per 32 columns
//     (k_pass_col), and passes with few columns one lane per voxel
//     (k_pass_col_search).
#include "device_common.h"
#include "internal.h"

#include <type_traits>

namespace pcsdf {

// ------------------------------------------------------------------ x pass

struct OccU8 {
  const uint8_t *p;
  int nx;
  __device__ __forceinline__ void row_begin(int64_t) const {}
  __device__ __forceinline__ bool at(int64_t row, int i) const {
    return p[row * nx + i] != 0;
  }
};

template <int MAXCH, class Occ>
__global__ __launch_bounds__(256) void k_pass_x(Occ occ, int32_t *out,
                                                int nx, int64_t rows) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;  // uniform across the wave
  int32_t *dst = out + row * nx;
  const int nch = (nx + 63) >> 6;
  constexpr int kNone = 0x40000000;
  const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t ge = ~0ull << lane;

  int left[MAXCH];
  bool isocc[MAXCH];
  int lastO = -kNone, lastF = -kNone;
#pragma unroll
  for (int c = 0; c < MAXCH; ++c) {
    if (c < nch) {
      const int i = c * 64 + lane;
      const bool valid = i < nx;
      const bool o = valid && occ.at(row, i);
      const uint64_t mO = __ballot(o);
      const uint64_t mF = __ballot(valid && !o);
      const uint64_t tO = mO & le, tF = mF & le;
      const int lo = tO ? c * 64 + 63 - __builtin_clzll(tO) : lastO;
      const int lf = tF ? c * 64 + 63 - __builtin_clzll(tF) : lastF;
      left[c] = o ? lf : lo;
      isocc[c] = o;
      if (mO) lastO = c * 64 + 63 - __builtin_clzll(mO);
      if (mF) lastF = c * 64 + 63 - __builtin_clzll(mF);
    }
  }
  int nextO = kNone, nextF = kNone;
#pragma unroll
  for (int c = MAXCH - 1; c >= 0; --c) {
    if (c < nch) {
      const int i = c * 64 + lane;
      const bool valid = i < nx;
      const bool o = isocc[c];
      const uint64_t mO = __ballot(o);
      const uint64_t mF = __ballot(valid && !o);
      const uint64_t tO = mO & ge, tF = mF & ge;
      const int ro = tO ? c * 64 + __builtin_ctzll(tO) : nextO;
      const int rf = tF ? c * 64 + __builtin_ctzll(tF) : nextF;
      const int r = o ? rf : ro;
      const int l = left[c];
      if (mO) nextO = c * 64 + __builtin_ctzll(mO);
      if (mF) nextF = c * 64 + __builtin_ctzll(mF);
      if (valid) {
        const bool none_l = l < 0, none_r = r >= nx;
        int32_t v;
        if (none_l && none_r) {
          v = kInf;
        } else {
          const int dl = none_l ? kNone : i - l;
          const int dr = none_r ? kNone : r - i;
          const int d = dl < dr ? dl : dr;
          v = d * d;
        }
        dst[i] = o ? -v : v;
      }
    }
  }
}

// The same pass with VPL adjacent voxels per lane (nx a multiple of VPL,
// at most 64 VPL): the row's occupancy is one load of VPL bytes per lane
// and its values VPL / 4 stores of 16 bytes.  Each lane finds the last and
// first voxel of either type among its own; the nearest lane to the left
// (right) holding a voxel of a type is a masked ballot's highest (lowest)
// bit, and that lane's last (first) voxel is read across lanes; a sweep
// over the lane's voxels then gives each voxel its nearest voxel of the
// other type on either side.
template <int VPL>
struct BytePack;
template <>
struct BytePack<4> {
  typedef uint32_t T;
};
template <>
struct BytePack<8> {
  typedef uint2 T;
};
template <>
struct BytePack<16> {
  typedef uint4 T;
};

template <int VPL>
__global__ __launch_bounds__(256) void k_pass_x_vec(const uint8_t *occ,
                                                    int32_t *out, int nx,
                                                    int64_t rows) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;  // uniform across the wave
  constexpr int kNone = 0x40000000;
  const int i0 = lane * VPL;
  const bool valid = i0 < nx;  // the whole pack: nx is a multiple of VPL
  typename BytePack<VPL>::T raw{};
  if (valid)
    raw = *reinterpret_cast<const typename BytePack<VPL>::T *>(
        occ + row * nx + i0);
  const uint8_t *bytes = reinterpret_cast<const uint8_t *>(&raw);
  uint32_t mo = 0;  // bit j: voxel i0 + j is occupied
#pragma unroll
  for (int j = 0; j < VPL; ++j) mo |= (bytes[j] != 0 ? 1u : 0u) << j;
  const uint32_t mf = valid ? ~mo & ((1u << VPL) - 1u) : 0u;
  // last / first voxel of each type in this lane
  const int lastO = mo ? i0 + 31 - __builtin_clz(mo) : -kNone;
  const int lastF = mf ? i0 + 31 - __builtin_clz(mf) : -kNone;
  const int firstO = mo ? i0 + __builtin_ctz(mo) : kNone;
  const int firstF = mf ? i0 + __builtin_ctz(mf) : kNone;
  const uint64_t anyO = __ballot(mo != 0), anyF = __ballot(mf != 0);
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t above = lane == 63 ? 0ull : ~0ull << (lane + 1);
  const uint64_t bO = anyO & below, bF = anyF & below;
  const uint64_t aO = anyO & above, aF = anyF & above;
  // source lanes (this lane where there is none; its value is not used)
  const int sbO = bO ? 63 - __builtin_clzll(bO) : lane;
  const int sbF = bF ? 63 - __builtin_clzll(bF) : lane;
  const int saO = aO ? __builtin_ctzll(aO) : lane;
  const int saF = aF ? __builtin_ctzll(aF) : lane;
  const int pO = __shfl(lastO, sbO), pF = __shfl(lastF, sbF);
  const int nO = __shfl(firstO, saO), nF = __shfl(firstF, saF);
  int lO = bO ? pO : -kNone, lF = bF ? pF : -kNone;  // nearest at or left
  int rO = aO ? nO : kNone, rF = aF ? nF : kNone;    // nearest at or right
  int left[VPL];  // nearest voxel of the other type to the left
#pragma unroll
  for (int j = 0; j < VPL; ++j) {
    const bool o = (mo >> j) & 1u;
    left[j] = o ? lF : lO;
    if (o)
      lO = i0 + j;
    else
      lF = i0 + j;
  }
  int32_t v[VPL];
#pragma unroll
  for (int j = VPL - 1; j >= 0; --j) {
    const bool o = (mo >> j) & 1u;
    const int i = i0 + j;
    const int r = o ? rF : rO;
    if (o)
      rO = i;
    else
      rF = i;
    const int l = left[j];
    const bool none_l = l < 0, none_r = r >= nx;
    int32_t d2;
    if (none_l && none_r) {
      d2 = kInf;
    } else {
      const int dl = none_l ? kNone : i - l;
      const int dr = none_r ? kNone : r - i;
      const int d = dl < dr ? dl : dr;
      d2 = d * d;
    }
    v[j] = o ? -d2 : d2;
  }
  if (valid) {
    int4 *dst = reinterpret_cast<int4 *>(out + row * nx + i0);
#pragma unroll
    for (int c = 0; c < VPL / 4; ++c)
      dst[c] = make_int4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  }
}

template <class Occ>
static int launch_x(Handle *h, const Occ &occ, int32_t *out, int nx,
                    int64_t rows, hipStream_t s, const char *what) {
  if (rows <= 0) return PCSDF_OK;
  const int nch = (nx + 63) / 64;
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (nch <= 1)
    launch_timed(h, k_pass_x<1, Occ>, grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 2)
    launch_timed(h, k_pass_x<2, Occ>, grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 4)
    launch_timed(h, k_pass_x<4, Occ>, grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 8)
    launch_timed(h, k_pass_x<8, Occ>, grid, block, 0, s, occ, out, nx,
                       rows);
  else
    launch_timed(h, k_pass_x<16, Occ>, grid, block, 0, s, occ, out, nx,
                       rows);
  return check_launch(h, what);
}

int launch_pass_x_u8(Handle *h, const uint8_t *occ, int32_t *out, int nx,
                     int64_t rows, hipStream_t s) {
  // VPL voxels per lane where the row fits one wave and every pack is
  // aligned (occupancy to VPL bytes, values to 16)
  int vpl = 0;
  for (int c : {4, 8, 16})
    if (nx <= 64 * c && nx % c == 0 && !((uintptr_t)occ % c) &&
        !((uintptr_t)out % 16)) {
      vpl = c;
      break;
    }
  if (vpl == 0 || rows <= 0)
    return launch_x(h, OccU8{occ, nx}, out, nx, rows, s, "pass_x_u8");
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (vpl == 4)
    launch_timed(h, k_pass_x_vec<4>, grid, block, 0, s, occ, out, nx,
                       rows);
  else if (vpl == 8)
    launch_timed(h, k_pass_x_vec<8>, grid, block, 0, s, occ, out, nx,
                       rows);
  else
    launch_timed(h, k_pass_x_vec<16>, grid, block, 0, s, occ, out, nx,
                       rows);
  return check_launch(h, "pass_x_vec");
}

// ------------------------------------------------------- y / z column pass

__device__ __forceinline__ int site_of(uint32_t e) { return (int)(e >> 22); }
__device__ __forceinline__ int val_of(uint32_t e) {
  return (int)(e & 0x3FFFFFu);
}

template <bool kGlobalStack, bool kWriteSdf>
__global__ __launch_bounds__(64) void k_pass_col(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride, int64_t nblocks, int tiles, uint32_t *gstack) {
  extern __shared__ uint32_t lds_stack[];
  const int lane = threadIdx.x;
  const int col = lane & 31;
  const bool inside_ch = lane >= 32;  // channel of the free set
  uint32_t *stk = kGlobalStack
                      ? gstack + (int64_t)blockIdx.x * (int64_t)m * 64
                      : lds_stack;

  for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int64_t o = b / tiles;
    const int tile = (int)(b - o * tiles);
    const int i = tile * 32 + col;
    const bool active = i < nfast;
    const int32_t *src = in + o * outer_stride + (active ? i : 0);
    int32_t *dst = out + o * outer_stride + (active ? i : 0);
    float *dsdf = kWriteSdf ? sdf + o * outer_stride + (active ? i : 0)
                            : nullptr;

    // Forward sweep: build the lower envelope of this lane's channel.
    int top = -1;
    uint32_t etop = 0;  // stk[top] cached in a register
    for (int q0 = 0; q0 < m; q0 += 8) {
      int32_t xb[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int q = q0 + t;
        xb[t] = (active && q < m) ? src[(int64_t)q * stride] : 0;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int q = q0 + t;
        const int32_t x = xb[t];
        bool site;
        int f;
        if (!inside_ch) {  // sites: occupied voxels (0), free with f_O
          site = x != kInf;
          f = x > 0 ? x : 0;
        } else {           // sites: free voxels (0), occupied with f_F
          site = x != -kInf;
          f = x < 0 ? -x : 0;
        }
        site = site && active && q < m;
        if (site) {
          const int fq = f + q * q;
          while (top >= 1) {
            const uint32_t eb = stk[(top - 1) * 64 + lane];
            const int sa = site_of(etop), fa = val_of(etop);
            const int sb = site_of(eb), fb = val_of(eb);
            const int64_t lhs = (int64_t)(fq - fa - sa * sa) * (sa - sb);
            const int64_t rhs =
                (int64_t)(fa + sa * sa - fb - sb * sb) * (q - sa);
            if (lhs <= rhs) {
              --top;
              etop = eb;
            } else {
              break;
            }
          }
          ++top;
          etop = ((uint32_t)q << 22) | (uint32_t)f;
          stk[top * 64 + lane] = etop;
        }
      }
    }

    // Fill sweep: walk the envelope and write this channel's voxels.
    int k = 0;
    uint32_t ek = top >= 0 ? stk[lane] : 0;
    uint32_t ek1 = top >= 1 ? stk[64 + lane] : 0;
    for (int q0 = 0; q0 < m; q0 += 8) {
      int32_t xb[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int q = q0 + t;
        xb[t] = (active && q < m) ? src[(int64_t)q * stride] : 0;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int q = q0 + t;
        const int32_t x = xb[t];
        const bool mine = inside_ch ? (x < 0) : (x > 0);
        int32_t val = kInf;
        if (top >= 0) {
          while (k < top) {
            const int dk = q - site_of(ek), dk1 = q - site_of(ek1);
            const int vk = dk * dk + val_of(ek);
            const int vk1 = dk1 * dk1 + val_of(ek1);
            if (vk1 <= vk) {
              ++k;
              ek = ek1;
              ek1 = k < top ? stk[(k + 1) * 64 + lane] : 0;
            } else {
              break;
            }
          }
          const int d = q - site_of(ek);
          val = d * d + val_of(ek);
        }
        if (mine && active && q < m) {
          const int32_t v = inside_ch ? -val : val;
          dst[(int64_t)q * stride] = v;
          if (kWriteSdf) dsdf[(int64_t)q * stride] = ssq_to_metres(v, hf);
        }
      }
    }
  }
}

// The same pass with each column split into S segments, one wave per
// segment (workgroup = S waves), for the occupied set's channel only:
// every lane runs one column (64 adjacent columns per wave), and the free
// set's channel, which only the occupied voxels need, is left to
// k_pass_col_search.  Wave w builds the lower envelope of the sites in its
// segment; after a barrier it fills its segment's voxels with the minimum
// over the S envelopes, walking each one as the fill sweep above walks its
// single envelope (the minimizing parabola of an envelope moves right as q
// grows).  The envelope of the whole column is the lower envelope of the
// segments' envelopes, so the result is exact.  Its own segment is
// evaluated first, then the other segments of each side nearest first; a
// side ends at the first segment that no lane of the wave can use (its
// nearest voxel is no closer than the square root of the value so far,
// and farther segments are farther still).
//
// Arithmetic.  A parabola of site p and value f is held as (p, h) with
// h = f + p^2, so its value at q is q^2 - 2 q p + h.  Every operand fits in
// 24 bits (p, q < 1024 and h < 2^22 for grids of at most 1024 voxels per
// axis: f < 2 * 1023^2 before the last pass), so every product runs on the
// full-rate 24-bit multiplier, including the 48-bit cross-products of the
// stack test.
constexpr int kSegBatch = 16;

// The low 24 bits, sign-extended: marks a value as fitting the 24-bit
// multiplier, which reads only those bits (the extension costs nothing).
// mul24 is the product of two such values on that multiplier, mul48 its
// full 48-bit product.
__device__ __forceinline__ int32_t i24(int32_t v) { return (v << 8) >> 8; }
__device__ __forceinline__ int32_t mul24(int32_t a, int32_t b) {
  return __mul24(a, b);
}
__device__ __forceinline__ int64_t mul48(int32_t a, int32_t b) {
  return (int64_t)i24(a) * (int64_t)i24(b);
}

// LDS home of the segments' envelopes, [S][L][64] entries.  An entry is
// p << 22 | h in 32 bits.  With kRoot the pass's inputs are squares of
// integers below 1024 (the x pass's squared distances), and an entry is
// stored in 16 bits: p's offset within its segment (L <= 64: 6 bits) and
// the square root of f (10 bits), which halves the LDS of a column.
template <bool kRoot>
struct EnvLds {
  void *base;
  int L;
  typedef typename std::conditional<kRoot, uint16_t, uint32_t>::type Raw;
  __device__ __forceinline__ uint32_t raw(int s, int idx, int lane) const {
    return static_cast<const Raw *>(base)[(uint32_t)(s * L + idx) * 64u +
                                          (uint32_t)lane];
  }
  __device__ __forceinline__ void decode(int s, uint32_t e, int *p,
                                         int *h) const {
    if (kRoot) {
      const int pp = s * L + (int)(e >> 10), r = (int)(e & 1023u);
      *p = pp;
      *h = mul24(r, r) + mul24(pp, pp);
    } else {
      *p = (int)(e >> 22);
      *h = (int)(e & 0x3FFFFFu);
    }
  }
  __device__ __forceinline__ void get(int s, int idx, int lane, int *p,
                                      int *h) const {
    decode(s, raw(s, idx, lane), p, h);
  }
  // r: the square root of the site's value (kRoot only)
  __device__ __forceinline__ void put(int s, int idx, int lane, int p, int h,
                                      int r) const {
    const uint32_t at = (uint32_t)(s * L + idx) * 64u + (uint32_t)lane;
    if (kRoot)
      static_cast<uint16_t *>(base)[at] =
          (uint16_t)(((uint32_t)(p - s * L) << 10) | (uint32_t)r);
    else
      static_cast<uint32_t *>(base)[at] = ((uint32_t)p << 22) | (uint32_t)h;
  }
  static constexpr int bytes() { return kRoot ? 2 : 4; }
};

// Square root of a perfect square below 2^20: the hardware's approximate
// root is within an ulp (2^-13 here) of the integer, so rounding to
// nearest recovers it exactly.
__device__ __forceinline__ int root_of_square(int f) {
  return (int)(__builtin_amdgcn_sqrtf((float)f) + 0.5f);
}

template <int S, bool kWriteSdf, bool kRoot>
__global__ __launch_bounds__(64 * S) void k_pass_col_seg(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride, int64_t nblocks, int tiles) {
  extern __shared__ uint32_t lds_seg[];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int L = (m + S - 1) / S;
  const EnvLds<kRoot> env{lds_seg, L};  // [S][L][64]
  int *const tops = reinterpret_cast<int *>(
      reinterpret_cast<char *>(lds_seg) +
      (size_t)S * L * 64 * EnvLds<kRoot>::bytes());
  const int q0 = w * L;
  const int q1 = min(m, q0 + L);

  for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int64_t o = b / tiles;
    const int tile = (int)(b - o * tiles);
    const int i = tile * 64 + lane;
    const bool active = i < nfast;
    const int64_t at0 = o * outer_stride + (active ? i : 0) + q0 * stride;
    const int32_t *src = in + at0;  // row q0 of this lane's column
    int32_t *dst = out + at0;
    float *dsdf = kWriteSdf ? sdf + at0 : nullptr;

    // Envelope of this segment's sites; its top three entries in registers,
    // so that a pop reads the LDS only for the entry that a second pop
    // would need.
    int top = -1;
    int pa = 0, ha = 0;  // entry top
    int pb = 0, hb = 0;  // entry top - 1
    int pc = 0, hc = 0;  // entry top - 2
    for (int qb = q0; qb < q1; qb += kSegBatch) {
      int32_t xb[kSegBatch];
#pragma unroll
      for (int t = 0; t < kSegBatch; ++t)
        xb[t] = (active && qb + t < q1)
                    ? src[(int64_t)(qb - q0 + t) * stride]
                    : kInf;
#pragma unroll
      for (int t = 0; t < kSegBatch; ++t) {
        const int q = qb + t;
        const int32_t x = xb[t];
        if (x == kInf) continue;  // no site in this row (or past the end)
        const int f = x > 0 ? x : 0;
        const int hq = f + mul24(q, q);
        while (top >= 1) {
          // The top stays if the new parabola overtakes it to the right
          // of where it overtakes the entry below (cross-multiplied).
          if (mul48(hq - ha, pa - pb) > mul48(ha - hb, q - pa)) break;
          --top;
          pa = pb;
          ha = hb;
          pb = pc;
          hb = hc;
          if (top >= 2) env.get(w, top - 2, lane, &pc, &hc);
        }
        pc = pb;
        hc = hb;
        pb = pa;
        hb = ha;
        pa = q;
        ha = hq;
        ++top;
        env.put(w, top, lane, q, hq, kRoot ? root_of_square(f) : 0);
      }
    }
    tops[w * 64 + lane] = top;
    __syncthreads();

    // Fill this segment from the S envelopes.  Envelope j is that of
    // segment (w + j) mod S: j = 0 is this wave's own, j = 1 .. S-1-w the
    // segments above, the rest those below.  Per envelope: its walk
    // position k, entries k and k + 1 decoded and entry k + 2 as read
    // ahead.  An empty envelope holds one entry of value kFar at every q
    // (above every real value), so no lane tests for emptiness.
    constexpr int kFar = 1 << 30;
    int tp[S], k[S], p0[S], h0[S], p1[S], h1[S];
    uint32_t e2[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int s = w + j < S ? w + j : w + j - S;
      tp[j] = tops[s * 64 + lane];
      k[j] = 0;
      p1[j] = h1[j] = 0;
      e2[j] = 0;
      if (tp[j] >= 0) {
        env.get(s, 0, lane, &p0[j], &h0[j]);
      } else {
        p0[j] = 0;
        h0[j] = kFar;
        tp[j] = 0;
      }
      if (tp[j] >= 1) env.get(s, 1, lane, &p1[j], &h1[j]);
      if (tp[j] >= 2) e2[j] = env.raw(s, 2, lane);
    }
    int32_t *dq = dst;
    float *fq = dsdf;
    for (int q = q0; q < q1; ++q) {
      const int q2 = 2 * q, qq = mul24(q, q);
      // value of envelope j at q (its walk position moves right only; an
      // envelope skipped for some q catches up when next evaluated)
      auto eval = [&](int j) -> int32_t {
        const int s = w + j < S ? w + j : w + j - S;
        while (k[j] < tp[j]) {
          // entry k + 1 is no higher at q: h1 - h0 <= 2 q (p1 - p0)
          if (h1[j] - h0[j] > mul24(q2, p1[j] - p0[j])) break;
          ++k[j];
          p0[j] = p1[j];
          h0[j] = h1[j];
          if (k[j] < tp[j]) {
            env.decode(s, e2[j], &p1[j], &h1[j]);
            e2[j] = env.raw(s, min(k[j] + 2, tp[j]), lane);
          }
        }
        return qq + h0[j] - mul24(q2, p0[j]);
      };
      int32_t val = eval(0);
      // segments above, nearest first
#pragma unroll
      for (int j = 1; j < S; ++j) {
        if (j >= S - w) break;
        const int gap = (w + j) * L - q;
        const bool reach = mul24(gap, gap) < val;
        if (__ballot(reach) == 0) break;
        if (reach) val = min(val, eval(j));
      }
      // segments below, nearest first
#pragma unroll
      for (int j = S - 1; j >= 1; --j) {
        if (j < S - w) break;
        const int gap = q - ((w + j - S + 1) * L - 1);
        const bool reach = mul24(gap, gap) < val;
        if (__ballot(reach) == 0) break;
        if (reach) val = min(val, eval(j));
      }
      // The free voxels get their value; an occupied voxel is a site of
      // value 0 (left to the free set's channel).
      if (val > 0 && active) {
        const int32_t v = val >= kFar ? kInf : val;
        *dq = v;
        if (kWriteSdf) *fq = ssq_to_metres(v, hf);
      }
      dq += stride;
      if (kWriteSdf) fq += stride;
    }
    __syncthreads();  // the stacks are reused by the next column tile
  }
}

// The same pass with one lane per voxel, for passes with few columns (a
// one-layer grid, e.g. the map collapsed to the floor, has only nx/32 column
// tiles): voxel q of its channel takes g(q) = min_p f(p) + (q - p)^2 by
// searching p = q -+ d for d = 1, 2, ... until d^2 >= the best value so
// far (no farther p can be smaller, f >= 0).  Exact, like the envelope;
// its work grows with the distance found, so it is kept to small passes.
// Grid: (voxels of one outer index / 256, outer indices).
constexpr int kSearchBatch = 4;

template <bool kWriteSdf>
__global__ __launch_bounds__(256) void k_pass_col_search(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (uint32_t)nfast * (uint32_t)m) return;
  const int q = (int)(t / (uint32_t)nfast);
  const int i = (int)(t - (uint32_t)q * (uint32_t)nfast);
  // The outer index's slab is uniform across the block, so each access is
  // a uniform base plus a 32-bit lane byte offset (a slab holds at most
  // 2^30 elements).
  const int64_t o = blockIdx.y;
  const char *base = reinterpret_cast<const char *>(in + o * outer_stride);
  char *obase = reinterpret_cast<char *>(out + o * outer_stride);
  char *fbase = kWriteSdf ? reinterpret_cast<char *>(sdf + o * outer_stride)
                          : nullptr;
  const uint32_t st = (uint32_t)stride * 4u;  // bytes
  auto ld = [&](uint32_t off) -> int32_t {
    return *reinterpret_cast<const int32_t *>(base + off);
  };
  const uint32_t at = (uint32_t)i * 4u + (uint32_t)q * st;
  const int32_t x = ld(at);
  const bool inside = x < 0;  // occupied: the free set's channel
  // value of row p in this voxel's channel (kInf: no site in that row)
  auto f_of = [&](int32_t v) -> int32_t {
    if (!inside) return v == kInf ? kInf : (v > 0 ? v : 0);
    return v == -kInf ? kInf : (v < 0 ? -v : 0);
  };
  int32_t best = f_of(x);
  const int dmax = max(q, m - 1 - q);
  // kSearchBatch distances per step: their loads are issued together, so a
  // step costs one memory latency (rows past the stopping distance are read
  // and cannot lower the value: d^2 >= best there).
  for (int d0 = 1; d0 <= dmax; d0 += kSearchBatch) {
    if (d0 * d0 >= best) break;
    int32_t lo[kSearchBatch], hi[kSearchBatch];
#pragma unroll
    for (int u = 0; u < kSearchBatch; ++u) {
      const int d = d0 + u;
      lo[u] = q - d >= 0 ? ld(at - (uint32_t)d * st) : kInf;
      hi[u] = q + d < m ? ld(at + (uint32_t)d * st) : kInf;
    }
#pragma unroll
    for (int u = 0; u < kSearchBatch; ++u) {
      const int d = d0 + u;
      const int32_t d2 = d * d;
      const int32_t fl = q - d >= 0 ? f_of(lo[u]) : kInf;
      const int32_t fh = q + d < m ? f_of(hi[u]) : kInf;
      if (fl != kInf) best = min(best, d2 + fl);
      if (fh != kInf) best = min(best, d2 + fh);
    }
  }
  const int32_t v = inside ? (best == kInf ? -kInf : -best) : best;
  *reinterpret_cast<int32_t *>(obase + at) = v;
  if (kWriteSdf)
    *reinterpret_cast<float *>(fbase + at) = ssq_to_metres(v, hf);
}

// The free set's channel of the occupied voxels, beside k_pass_col_seg's
// occupied-set channel (the distances found there are bounded by the
// obstacles' half-widths).  Lane t takes column i = t mod nfast and the G
// consecutive rows qa = G (t / nfast) .. qa + G - 1 of it.  It loads those
// rows and, if any of them is occupied, searches outward from the group:
// kSearchBatch rows below and above per step (their loads issued
// together), each row read once and offered to every row of the group.  A
// side ends when no occupied row of the group can still be lowered from
// it (the next row's distance squared is at least that row's value so far;
// farther rows are farther still).  Neighbouring rows share their
// neighbours, so a group costs about one search instead of G.  Exact, like
// the envelope.  Grid: (lanes of one outer index / 256, outer indices).
template <bool kWriteSdf, int G>
__global__ __launch_bounds__(256) void k_pass_col_inside(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride) {
  const uint32_t mg = (uint32_t)(m + G - 1) / G;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (uint32_t)nfast * mg) return;
  const int qg = (int)(t / (uint32_t)nfast);
  const int i = (int)(t - (uint32_t)qg * (uint32_t)nfast);
  // The outer index's slab is uniform across the block, so each access is
  // a uniform base plus a 32-bit lane byte offset (a slab holds at most
  // 2^30 elements).
  const int64_t o = blockIdx.y;
  const char *base = reinterpret_cast<const char *>(in + o * outer_stride);
  char *obase = reinterpret_cast<char *>(out + o * outer_stride);
  char *fbase = kWriteSdf ? reinterpret_cast<char *>(sdf + o * outer_stride)
                          : nullptr;
  const uint32_t st = (uint32_t)stride * 4u;  // bytes
  auto ld = [&](uint32_t off) -> int32_t {
    return *reinterpret_cast<const int32_t *>(base + off);
  };
  // value of a row in the free set's channel: 0 on a free voxel, f_F on an
  // occupied one, kInf where the row has no free voxel (rows outside the
  // column are passed as -kInf)
  auto f_free = [](int32_t v) -> int32_t {
    return v == -kInf ? kInf : (v < 0 ? -v : 0);
  };
  const int qa = qg * G;
  const int n = min(G, m - qa);  // rows of the group inside the column
  const uint32_t at0 = (uint32_t)i * 4u + (uint32_t)qa * st;
  int32_t x[G];
#pragma unroll
  for (int r = 0; r < G; ++r) x[r] = r < n ? ld(at0 + (uint32_t)r * st) : -kInf;
  bool need[G];  // occupied rows: the ones this channel writes
  bool any = false;
#pragma unroll
  for (int r = 0; r < G; ++r) {
    need[r] = r < n && x[r] < 0;
    any = any || need[r];
  }
  if (!any) return;
  int32_t best[G];
#pragma unroll
  for (int r = 0; r < G; ++r) best[r] = kInf;
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const int32_t fp = f_free(x[p]);
    if (fp == kInf) continue;
#pragma unroll
    for (int r = 0; r < G; ++r) best[r] = min(best[r], fp + (r - p) * (r - p));
  }
  for (int d0 = 1;; d0 += kSearchBatch) {
    bool lo = false, hi = false;
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if (!need[r]) continue;
      const int dl = r + d0, dh = n - 1 - r + d0;
      lo = lo || mul24(dl, dl) < best[r];
      hi = hi || mul24(dh, dh) < best[r];
    }
    lo = lo && qa - d0 >= 0;
    hi = hi && qa + n - 1 + d0 < m;
    if (!lo && !hi) break;
    int32_t vl[kSearchBatch], vh[kSearchBatch];
#pragma unroll
    for (int u = 0; u < kSearchBatch; ++u) {
      const int d = d0 + u;
      vl[u] = lo && qa - d >= 0 ? ld(at0 - (uint32_t)d * st) : -kInf;
      vh[u] = hi && qa + n - 1 + d < m
                  ? ld(at0 + (uint32_t)(n - 1 + d) * st)
                  : -kInf;
    }
#pragma unroll
    for (int u = 0; u < kSearchBatch; ++u) {
      const int d = d0 + u;
      const int32_t fl = f_free(vl[u]), fh = f_free(vh[u]);
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int dl = r + d, dh = n - 1 - r + d;
        if (fl != kInf) best[r] = min(best[r], fl + mul24(dl, dl));
        if (fh != kInf) best[r] = min(best[r], fh + mul24(dh, dh));
      }
    }
  }
#pragma unroll
  for (int r = 0; r < G; ++r) {
    if (!need[r]) continue;
    const int32_t v = best[r] == kInf ? -kInf : -best[r];
    const uint32_t at = at0 + (uint32_t)r * st;
    *reinterpret_cast<int32_t *>(obase + at) = v;
    if (kWriteSdf)
      *reinterpret_cast<float *>(fbase + at) = ssq_to_metres(v, hf);
  }
}

// Rows per lane of the free set's channel.
constexpr int kInsideRows = 4;

// Column tiles below which a pass runs one lane per voxel.
constexpr int64_t kSearchTiles = 64;

// Workgroups using more than 64 KB of LDS need the kernel's limit raised
// on the current device; the call is cheap and made before each such
// launch (a cached flag would be process-wide, not per device, and shared
// between threads).
static hipError_t allow_lds(const void *kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int S, bool kRoot>
static hipError_t launch_seg(Handle *h, const int32_t *in, int32_t *out,
                             float *sdf_out,
                             float h_f, int nfast, int m, int64_t stride,
                             int64_t outer_stride, int64_t nblocks, int tiles,
                             size_t lds, hipStream_t s) {
  const unsigned grid =
      (unsigned)(nblocks < (1LL << 30) ? nblocks : (1LL << 30));
  if (sdf_out) {
    const hipError_t e = allow_lds(
        reinterpret_cast<const void *>(&k_pass_col_seg<S, true, kRoot>),
        lds);
    if (e != hipSuccess) return e;
    launch_timed(h, k_pass_col_seg<S, true, kRoot>, dim3(grid),
                       dim3(64 * S), lds, s, in, out, sdf_out, h_f, nfast, m,
                       stride, outer_stride, nblocks, tiles);
  } else {
    const hipError_t e = allow_lds(
        reinterpret_cast<const void *>(&k_pass_col_seg<S, false, kRoot>),
        lds);
    if (e != hipSuccess) return e;
    launch_timed(h, k_pass_col_seg<S, false, kRoot>, dim3(grid),
                       dim3(64 * S), lds, s, in, out, sdf_out, h_f, nfast, m,
                       stride, outer_stride, nblocks, tiles);
  }
  return hipSuccess;
}

template <bool kRoot>
static hipError_t launch_seg_any(Handle *h, int S, const int32_t *in,
                                 int32_t *out,
                                 float *sdf_out, float h_f, int nfast, int m,
                                 int64_t stride, int64_t outer_stride,
                                 int64_t nblocks, int tiles, size_t lds,
                                 hipStream_t s) {
  switch (S) {
    case 2:
      return launch_seg<2, kRoot>(h, in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
    case 4:
      return launch_seg<4, kRoot>(h, in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
    default:
      return launch_seg<8, kRoot>(h, in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
  }
}

// The handle's side stream and its fork and join events, created on first
// use.
static int ensure_side_stream(Handle *h) {
  hipError_t e = hipSuccess;
  if (!h->side) e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  if (e == hipSuccess && !h->fork_ev)
    e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess && !h->join_ev)
    e = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming);
  if (e != hipSuccess)
    return fail(h, PCSDF_ERR_HIP,
                std::string("creating the side stream: ") +
                    hipGetErrorString(e));
  return PCSDF_OK;
}

// Segments per column: the tuning's, else one per 32 voxels of the column
// (at most 8: 16 waves of this kernel exceed the registers of a CU's
// share and were measured slower).
static int column_segments(const Handle *h, int m) {
  if (h->tuning.static_segments > 0) return h->tuning.static_segments;
  return m >= 256 ? 8 : m >= 128 ? 4 : m >= 64 ? 2 : 1;
}

int launch_pass_col(Handle *h, const int32_t *in, int32_t *out,
                    float *sdf_out, float h_f, int nfast, int nouter, int m,
                    int64_t stride, int64_t outer_stride, bool square_input,
                    bool use_side, hipStream_t s) {
  if (nfast <= 0 || nouter <= 0 || m <= 0) return PCSDF_OK;
  const int tiles = (nfast + 31) / 32;
  const int64_t nblocks = (int64_t)tiles * nouter;
  // the search kernel's grid: (lanes of one outer index / 256, nouter)
  auto sgrid = [&](int rows) {
    const int64_t mg = (m + rows - 1) / rows;
    return dim3((unsigned)(((int64_t)nfast * mg + 255) / 256),
                (unsigned)nouter);
  };
  if (nblocks < kSearchTiles && h->tuning.static_segments == 0) {
    if (sdf_out)
      launch_timed(h, k_pass_col_search<true>, sgrid(1),
                         dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                         stride, outer_stride);
    else
      launch_timed(h, k_pass_col_search<false>, sgrid(1),
                         dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                         stride, outer_stride);
    return check_launch(h, "pass_col_search");
  }
  int S = column_segments(h, m);
  while (S > 1 && S > m) S >>= 1;  // a power of two, at most m
  if (S > 1) {
    const int L = (m + S - 1) / S;
    // 16-bit envelope entries when the inputs are squares and a segment's
    // site offsets fit in 6 bits
    const bool root = square_input && L <= 64;
    const size_t lds_seg =
        (size_t)S * L * 64 * (root ? 2 : 4) + (size_t)S * 64 * 4;
    if ((int64_t)lds_seg <= h->max_lds) {
      // The free set's channel of the occupied voxels by search, on the
      // side stream (use_side), beside the occupied set's channel by
      // envelopes (64 columns per wave) on the caller's: they read the same
      // input and write disjoint voxels, and the search's memory waits
      // fill the envelope kernel's issue gaps.  Without use_side both run
      // on the caller's stream, one after the other.
      hipStream_t ss = s;
      int rc = PCSDF_OK;
      hipError_t e = hipSuccess;
      if (use_side) {
        if ((rc = ensure_side_stream(h))) return rc;
        e = hipEventRecord(h->fork_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->side, h->fork_ev, 0);
        if (e != hipSuccess)
          return fail(h, PCSDF_ERR_HIP,
                      std::string("forking the side stream: ") +
                          hipGetErrorString(e));
        ss = h->side;
      }
      if (sdf_out)
        launch_timed(h, k_pass_col_inside<true, kInsideRows>,
                     sgrid(kInsideRows), dim3(256), 0, ss, in, out, sdf_out,
                     h_f, nfast, m, stride, outer_stride);
      else
        launch_timed(h, k_pass_col_inside<false, kInsideRows>,
                     sgrid(kInsideRows), dim3(256), 0, ss, in, out, sdf_out,
                     h_f, nfast, m, stride, outer_stride);
      rc = check_launch(h, "pass_col_inside");
      if (!rc) {
        const int tiles64 = (nfast + 63) / 64;
        const int64_t nblocks64 = (int64_t)tiles64 * nouter;
        e = root ? launch_seg_any<true>(h, S, in, out, sdf_out, h_f, nfast, m,
                                        stride, outer_stride, nblocks64,
                                        tiles64, lds_seg, s)
                 : launch_seg_any<false>(h, S, in, out, sdf_out, h_f, nfast, m,
                                         stride, outer_stride, nblocks64,
                                         tiles64, lds_seg, s);
        if (e != hipSuccess)
          rc = fail(h, PCSDF_ERR_HIP,
                    std::string("raising the LDS limit of pass_col_seg: ") +
                        hipGetErrorString(e));
        else
          rc = check_launch(h, "pass_col_seg");
      }
      if (!use_side) return rc;
      // join in every case, so that no work of this call outlives it on
      // the side stream
      e = hipEventRecord(h->join_ev, h->side);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, h->join_ev, 0);
      if (rc) return rc;
      if (e != hipSuccess)
        return fail(h, PCSDF_ERR_HIP,
                    std::string("joining the side stream: ") +
                        hipGetErrorString(e));
      return PCSDF_OK;
    }
  }
  const size_t lds = (size_t)m * 64 * sizeof(uint32_t);
  const dim3 block(64);
  if ((int64_t)lds <= h->max_lds) {
    const unsigned grid = (unsigned)(nblocks < (1LL << 30) ? nblocks
                                                           : (1LL << 30));
    const void *kfn =
        sdf_out ? reinterpret_cast<const void *>(&k_pass_col<false, true>)
                : reinterpret_cast<const void *>(&k_pass_col<false, false>);
    const hipError_t e = allow_lds(kfn, lds);
    if (e != hipSuccess)
      return fail(h, PCSDF_ERR_HIP,
                  std::string("raising the LDS limit of pass_col: ") +
                      hipGetErrorString(e));
    if (sdf_out)
      launch_timed(h, k_pass_col<false, true>, dim3(grid), block, lds,
                         s, in, out, sdf_out, h_f, nfast, m, stride,
                         outer_stride, nblocks, tiles, nullptr);
    else
      launch_timed(h, k_pass_col<false, false>, dim3(grid), block, lds,
                         s, in, out, sdf_out, h_f, nfast, m, stride,
                         outer_stride, nblocks, tiles, nullptr);
    return check_launch(h, "pass_col");
  }
  // Columns too long for LDS: stacks in a workspace slab, a bounded
  // number of resident blocks striding over all columns.
  const int64_t gblocks = nblocks < 4096 ? nblocks : 4096;
  int rc = ensure_buffer(h, h->stack_buf, (size_t)gblocks * lds, s);
  if (rc) return rc;
  uint32_t *gstack = reinterpret_cast<uint32_t *>(h->stack_buf.ptr);
  if (sdf_out)
    launch_timed(h, k_pass_col<true, true>, dim3((unsigned)gblocks),
                       block, 0, s, in, out, sdf_out, h_f, nfast, m, stride,
                       outer_stride, nblocks, tiles, gstack);
  else
    launch_timed(h, k_pass_col<true, false>, dim3((unsigned)gblocks),
                       block, 0, s, in, out, sdf_out, h_f, nfast, m, stride,
                       outer_stride, nblocks, tiles, gstack);
  return check_launch(h, "pass_col_global_stack");
}

// --------------------------------------------------------- static build

}  // namespace pcsdf

using namespace pcsdf;

extern "C" int pcsdf_build_static_sdf(pcsdf_handle *hp, const pcsdf_grid *g,
                                      const uint8_t *occ_dev,
                                      int32_t *ssq_dev, float *sdf_dev,
                                      void *stream) {
  Handle *h = reinterpret_cast<Handle *>(hp);
  if (!h) return PCSDF_ERR_INVALID_ARG;
  int rc = check_grid(h, g);
  if (rc) return rc;
  if (!occ_dev || !ssq_dev)
    return fail(h, PCSDF_ERR_INVALID_ARG, "occ_dev and ssq_dev are required");
  if (((uintptr_t)ssq_dev & 3) || ((uintptr_t)sdf_dev & 3))
    return fail(h, PCSDF_ERR_ALIGN, "ssq_dev/sdf_dev must be 4-byte aligned");
  if ((rc = bind_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t V = (int64_t)nx * ny * nz;
  if ((rc = ensure_buffer(h, h->tmp_buf, (size_t)V * 4, s))) return rc;
  int32_t *tmp = reinterpret_cast<int32_t *>(h->tmp_buf.ptr);
  const float hf = (float)g->voxel_m;
  // x: occ -> ssq (as scratch); y: ssq -> tmp; z: tmp -> ssq (+ sdf)
  ProfScope ps(h, PCSDF_KERNEL_STATIC, s);
  if ((rc = launch_pass_x_u8(h, occ_dev, ssq_dev, nx, (int64_t)ny * nz, s)))
    return rc;
  // the y pass reads the x pass's squared distances (perfect squares)
  if ((rc = launch_pass_col(h, ssq_dev, tmp, nullptr, hf, nx, nz, ny, nx,
                            (int64_t)nx * ny, true, true, s)))
    return rc;
  return launch_pass_col(h, tmp, ssq_dev, sdf_dev, hf, nx, ny, nz,
                         (int64_t)nx * ny, nx, false, true, s);
}
