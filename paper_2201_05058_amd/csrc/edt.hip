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
//     one coalesced 128-byte load shared by both halves of the wave:
//     lanes 0..31 run the occupied-set channel of 32 adjacent columns and
//     lanes 32..63 the free-set channel of the same columns.  No transpose
//     is needed because x is the contiguous axis.  Each lane keeps its
//     envelope stack in LDS, one packed 32-bit entry per site (site index
//     in 10 bits, value in 22 bits: values stay below 2*1023^2 < 2^22
//     before the last pass), laid out [depth][lane] so a wave's accesses
//     spread over all banks.  Intersections are compared by
//     cross-multiplication in int64, so the envelope has no division.
#include "device_common.h"
#include "internal.h"

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

template <class Occ>
static int launch_x(Handle *h, const Occ &occ, int32_t *out, int nx,
                    int64_t rows, hipStream_t s, const char *what) {
  if (rows <= 0) return PCSDF_OK;
  const int nch = (nx + 63) / 64;
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (nch <= 1)
    hipLaunchKernelGGL((k_pass_x<1, Occ>), grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 2)
    hipLaunchKernelGGL((k_pass_x<2, Occ>), grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 4)
    hipLaunchKernelGGL((k_pass_x<4, Occ>), grid, block, 0, s, occ, out, nx,
                       rows);
  else if (nch <= 8)
    hipLaunchKernelGGL((k_pass_x<8, Occ>), grid, block, 0, s, occ, out, nx,
                       rows);
  else
    hipLaunchKernelGGL((k_pass_x<16, Occ>), grid, block, 0, s, occ, out, nx,
                       rows);
  return check_launch(h, what);
}

int launch_pass_x_u8(Handle *h, const uint8_t *occ, int32_t *out, int nx,
                     int64_t rows, hipStream_t s) {
  return launch_x(h, OccU8{occ, nx}, out, nx, rows, s, "pass_x_u8");
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
// segment (workgroup = S waves, 32 columns x 2 channels per wave as
// above).  Wave w builds the lower envelope of the sites in its segment;
// after a barrier it fills its segment's voxels with the minimum over the
// S envelopes, walking each one as the fill sweep above walks its single
// envelope (the minimizing parabola of an envelope moves right as q
// grows).  The envelope of the whole column is the lower envelope of the
// segments' envelopes, so the result is exact.  Its own segment is
// evaluated first and another segment only while it could still lower
// the value (its nearest voxel is closer than the square root of the
// value so far), so a fill usually reads one or two envelopes.  The
// workgroup's LDS is the same as one wave's above (S segments of m/S
// entries), so S times as many waves share a CU.
// Column values read per batch of loads in the segmented pass.
constexpr int kSegBatch = 16;

// LDS home of the segments' envelopes, [S][L][64] entries.  Registers hold
// an entry as above (site << 22 | value).  With kRoot the pass's inputs
// are squares of integers below 1024 (the x pass's squared distances), and
// an entry is stored in 16 bits: the site's offset within its segment (L
// <= 64: 6 bits) and the square root of its value (10 bits), which halves
// the LDS of a column.
template <bool kRoot>
struct EnvLds {
  void *base;
  int L;
  __device__ __forceinline__ uint32_t get(int s, int idx, int lane) const {
    const size_t at = ((size_t)s * L + idx) * 64 + lane;
    if (kRoot) {
      const uint32_t e = static_cast<const uint16_t *>(base)[at];
      const uint32_t site = (uint32_t)(s * L) + (e >> 10), r = e & 1023u;
      return (site << 22) | (r * r);
    }
    return static_cast<const uint32_t *>(base)[at];
  }
  __device__ __forceinline__ void put(int s, int idx, int lane,
                                      uint32_t e) const {
    const size_t at = ((size_t)s * L + idx) * 64 + lane;
    if (kRoot) {
      const uint32_t f = e & 0x3FFFFFu;
      uint32_t r = (uint32_t)__builtin_sqrtf((float)f);  // exact: f < 2^20
      r -= r * r > f ? 1u : 0u;
      r += (r + 1) * (r + 1) <= f ? 1u : 0u;
      static_cast<uint16_t *>(base)[at] =
          (uint16_t)((((e >> 22) - (uint32_t)(s * L)) << 10) | r);
    } else {
      static_cast<uint32_t *>(base)[at] = e;
    }
  }
  static constexpr int bytes() { return kRoot ? 2 : 4; }
};

//
// With kOutside, every lane runs the occupied set's channel (64 adjacent
// columns per wave) and the free set's channel, which only the occupied
// voxels need, is left to k_pass_col_search: a column's LDS then serves
// twice the columns.
template <int S, bool kWriteSdf, bool kOutside, bool kRoot>
__global__ __launch_bounds__(64 * S) void k_pass_col_seg(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride, int64_t nblocks, int tiles) {
  extern __shared__ uint32_t lds_seg[];
  constexpr int kCols = kOutside ? 64 : 32;  // columns per wave
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = kOutside ? lane : lane & 31;
  const bool inside_ch = !kOutside && lane >= 32;  // the free set's channel
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
    const int i = tile * kCols + col;
    const bool active = i < nfast;
    const int32_t *src = in + o * outer_stride + (active ? i : 0);
    int32_t *dst = out + o * outer_stride + (active ? i : 0);
    float *dsdf = kWriteSdf ? sdf + o * outer_stride + (active ? i : 0)
                            : nullptr;

    // Envelope of this segment's sites.
    int top = -1;
    uint32_t etop = 0;  // stk[top] cached in a register
    for (int qb = q0; qb < q1; qb += kSegBatch) {
      int32_t xb[kSegBatch];
#pragma unroll
      for (int t = 0; t < kSegBatch; ++t) {
        const int q = qb + t;
        xb[t] = (active && q < q1) ? src[(int64_t)q * stride] : 0;
      }
#pragma unroll
      for (int t = 0; t < kSegBatch; ++t) {
        const int q = qb + t;
        const int32_t x = xb[t];
        bool site;
        int f;
        if (!inside_ch) {
          site = x != kInf;
          f = x > 0 ? x : 0;
        } else {
          site = x != -kInf;
          f = x < 0 ? -x : 0;
        }
        site = site && active && q < q1;
        if (site) {
          const int fq = f + q * q;
          while (top >= 1) {
            const uint32_t eb = env.get(w, top - 1, lane);
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
          env.put(w, top, lane, etop);
        }
      }
    }
    tops[w * 64 + lane] = top;
    __syncthreads();

    // Fill this segment from all S envelopes.
    int tp[S], k[S];
    uint32_t ek[S], ek1[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      tp[s] = tops[s * 64 + lane];
      k[s] = 0;
      ek[s] = tp[s] >= 0 ? env.get(s, 0, lane) : 0;
      ek1[s] = tp[s] >= 1 ? env.get(s, 1, lane) : 0;
    }
    for (int q = q0; q < q1; ++q) {
      {
        // Value of envelope s at q (its walk pointer moves right only; an
        // envelope skipped for some q catches up when next evaluated).
        auto eval = [&](int s) -> int32_t {
          while (k[s] < tp[s]) {
            const int dk = q - site_of(ek[s]), dk1 = q - site_of(ek1[s]);
            const int vk = dk * dk + val_of(ek[s]);
            const int vk1 = dk1 * dk1 + val_of(ek1[s]);
            if (vk1 <= vk) {
              ++k[s];
              ek[s] = ek1[s];
              ek1[s] = k[s] < tp[s] ? env.get(s, k[s] + 1, lane) : 0;
            } else {
              break;
            }
          }
          const int d = q - site_of(ek[s]);
          return d * d + val_of(ek[s]);
        };
        // Own segment first; another segment s is gap voxels away at
        // least, so it cannot lower a value already <= gap^2.
        int32_t val = kInf;
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (s == w && tp[s] >= 0) val = eval(s);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (s == w || tp[s] < 0) continue;
          const int gap = s < w ? q - ((s + 1) * L - 1) : s * L - q;
          if (gap * gap >= val) continue;
          val = min(val, eval(s));
        }
        // A voxel of this channel's own set (free for the outside
        // channel, occupied for the inside one) is a site of the other
        // channel at distance 0, so each channel's value is positive
        // exactly on the voxels it owns: no second read of the input.
        if (val > 0 && active) {
          const int32_t v = inside_ch ? -val : val;
          dst[(int64_t)q * stride] = v;
          if (kWriteSdf) dsdf[(int64_t)q * stride] = ssq_to_metres(v, hf);
        }
      }
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
//
// With kInsideOnly only the occupied voxels are computed (the free set's
// channel, beside k_pass_col_seg's occupied-set channel); the distances
// found there are bounded by the obstacles' half-widths.  Grid: (voxels
// of one outer index / 256, outer indices).
constexpr int kSearchBatch = 4;

template <bool kWriteSdf, bool kInsideOnly, int kSearchRows>
__global__ __launch_bounds__(256) void k_pass_col_search(
    const int32_t *__restrict__ in, int32_t *__restrict__ out,
    float *__restrict__ sdf, float hf, int nfast, int m, int64_t stride,
    int64_t outer_stride) {
  // Lane t takes column i = t mod nfast and rows q = kSearchRows (t /
  // nfast) + 0 .. kSearchRows-1: their values are loaded together, and
  // only the voxels that need a value are searched (with kInsideOnly most
  // are free and cost one load; several rows per lane save launching a
  // wave per load on large passes, one row per lane keeps the searches of
  // small passes parallel).
  const uint32_t mg = (uint32_t)(m + kSearchRows - 1) / kSearchRows;
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
  int32_t xs[kSearchRows];
#pragma unroll
  for (int r = 0; r < kSearchRows; ++r) {
    const int q = qg * kSearchRows + r;
    xs[r] = q < m ? ld((uint32_t)i * 4u + (uint32_t)q * st) : 0;
  }
#pragma unroll 1
  for (int r = 0; r < kSearchRows; ++r) {
    const int q = qg * kSearchRows + r;
    const int32_t x = xs[r];
    const bool inside = x < 0;  // occupied: the free set's channel
    if (q >= m || (kInsideOnly && !inside)) continue;
    const uint32_t at = (uint32_t)i * 4u + (uint32_t)q * st;
    // value of row p in this voxel's channel (kInf: no site in that row)
    auto f_of = [&](int32_t v) -> int32_t {
      if (!inside) return v == kInf ? kInf : (v > 0 ? v : 0);
      return v == -kInf ? kInf : (v < 0 ? -v : 0);
    };
    int32_t best = f_of(x);
    const int dmax = max(q, m - 1 - q);
    // kSearchBatch distances per step: their loads are issued together,
    // so a step costs one memory latency (rows past the stopping distance
    // are read and cannot lower the value: d^2 >= best there).
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
}

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
static hipError_t launch_seg(const int32_t *in, int32_t *out, float *sdf_out,
                             float h_f, int nfast, int m, int64_t stride,
                             int64_t outer_stride, int64_t nblocks, int tiles,
                             size_t lds, hipStream_t s) {
  const unsigned grid =
      (unsigned)(nblocks < (1LL << 30) ? nblocks : (1LL << 30));
  if (sdf_out) {
    const hipError_t e = allow_lds(
        reinterpret_cast<const void *>(&k_pass_col_seg<S, true, true, kRoot>),
        lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pass_col_seg<S, true, true, kRoot>), dim3(grid),
                       dim3(64 * S), lds, s, in, out, sdf_out, h_f, nfast, m,
                       stride, outer_stride, nblocks, tiles);
  } else {
    const hipError_t e = allow_lds(
        reinterpret_cast<const void *>(&k_pass_col_seg<S, false, true, kRoot>),
        lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pass_col_seg<S, false, true, kRoot>), dim3(grid),
                       dim3(64 * S), lds, s, in, out, sdf_out, h_f, nfast, m,
                       stride, outer_stride, nblocks, tiles);
  }
  return hipSuccess;
}

template <bool kRoot>
static hipError_t launch_seg_any(int S, const int32_t *in, int32_t *out,
                                 float *sdf_out, float h_f, int nfast, int m,
                                 int64_t stride, int64_t outer_stride,
                                 int64_t nblocks, int tiles, size_t lds,
                                 hipStream_t s) {
  switch (S) {
    case 2:
      return launch_seg<2, kRoot>(in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
    case 4:
      return launch_seg<4, kRoot>(in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
    default:
      return launch_seg<8, kRoot>(in, out, sdf_out, h_f, nfast, m, stride,
                                  outer_stride, nblocks, tiles, lds, s);
  }
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
                    hipStream_t s) {
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
      hipLaunchKernelGGL((k_pass_col_search<true, false, 1>), sgrid(1),
                         dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                         stride, outer_stride);
    else
      hipLaunchKernelGGL((k_pass_col_search<false, false, 1>), sgrid(1),
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
      // the occupied set's channel by envelopes, 64 columns per wave; then
      // the free set's channel of the occupied voxels by search
      const int tiles64 = (nfast + 63) / 64;
      const int64_t nblocks64 = (int64_t)tiles64 * nouter;
      const hipError_t e =
          root ? launch_seg_any<true>(S, in, out, sdf_out, h_f, nfast, m,
                                      stride, outer_stride, nblocks64,
                                      tiles64, lds_seg, s)
               : launch_seg_any<false>(S, in, out, sdf_out, h_f, nfast, m,
                                       stride, outer_stride, nblocks64,
                                       tiles64, lds_seg, s);
      if (e != hipSuccess)
        return fail(h, PCSDF_ERR_HIP,
                    std::string("raising the LDS limit of pass_col_seg: ") +
                        hipGetErrorString(e));
      int rc = check_launch(h, "pass_col_seg");
      if (rc) return rc;
      // four rows per lane from 2^25 voxels on (512^2 x 128: 3 % faster
      // than one; 256^2 x 128: 7 % slower)
      const bool big = (int64_t)nfast * m * nouter >= (1LL << 25);
      if (sdf_out && big)
        hipLaunchKernelGGL((k_pass_col_search<true, true, 4>), sgrid(4),
                           dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                           stride, outer_stride);
      else if (sdf_out)
        hipLaunchKernelGGL((k_pass_col_search<true, true, 1>), sgrid(1),
                           dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                           stride, outer_stride);
      else if (big)
        hipLaunchKernelGGL((k_pass_col_search<false, true, 4>), sgrid(4),
                           dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                           stride, outer_stride);
      else
        hipLaunchKernelGGL((k_pass_col_search<false, true, 1>), sgrid(1),
                           dim3(256), 0, s, in, out, sdf_out, h_f, nfast, m,
                           stride, outer_stride);
      return check_launch(h, "pass_col_inside");
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
      hipLaunchKernelGGL((k_pass_col<false, true>), dim3(grid), block, lds,
                         s, in, out, sdf_out, h_f, nfast, m, stride,
                         outer_stride, nblocks, tiles, nullptr);
    else
      hipLaunchKernelGGL((k_pass_col<false, false>), dim3(grid), block, lds,
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
    hipLaunchKernelGGL((k_pass_col<true, true>), dim3((unsigned)gblocks),
                       block, 0, s, in, out, sdf_out, h_f, nfast, m, stride,
                       outer_stride, nblocks, tiles, gstack);
  else
    hipLaunchKernelGGL((k_pass_col<true, false>), dim3((unsigned)gblocks),
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
                            (int64_t)nx * ny, true, s)))
    return rc;
  return launch_pass_col(h, tmp, ssq_dev, sdf_dev, hf, nx, ny, nz,
                         (int64_t)nx * ny, nx, false, s);
}
