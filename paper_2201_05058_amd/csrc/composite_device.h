// The composite epilogue shared by the single-scene kernel (composite.hip)
// and the batched workers (batch_device.h): for VEC consecutive voxels of
// the flattened [nz][ny][nx] grid, read the static field once and write
// min(static, humans' value) for a range of slices.
//
// The static field and the outputs are flat streams: VEC consecutive
// voxels starting at a multiple of VEC are one aligned VEC-wide access
// whenever VEC divides V = nx ny nz (so that every slice's outputs, at
// offset sl V, stay aligned) and the buffers are aligned.  The planar
// index of voxel v is v mod (nx ny), so the same voxels read VEC
// consecutive planar values of one layer when VEC also divides nx ny;
// otherwise those VEC values are read one by one (from the cached plane).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.h"

namespace pcsdf {

// Packs of VEC int32 or fp32 values, and their loads as global memory
// instructions.  Pointers read from memory (the batch's scene
// table) would otherwise be accessed with flat instructions, which the
// compiler cannot count in order: every wait for one of them then waits
// for all outstanding loads and stores.  The casts are written per
// concrete type because a global address space on a template-dependent
// type is not kept.
#if defined(__clang__)
#define PCSDF_GLOBAL_AS __attribute__((address_space(1)))
typedef int32_t pk_i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t pk_i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t pk_i32x1 __attribute__((ext_vector_type(1)));
typedef float pk_f32x4 __attribute__((ext_vector_type(4)));
typedef float pk_f32x2 __attribute__((ext_vector_type(2)));
typedef float pk_f32x1 __attribute__((ext_vector_type(1)));
#else  // a host compiler building the device code for CPU tests
#define PCSDF_GLOBAL_AS
template <class T, int N>
struct HostPack {
  T v[N];
  T &operator[](int i) { return v[i]; }
  const T &operator[](int i) const { return v[i]; }
};
typedef HostPack<int32_t, 4> pk_i32x4;
typedef HostPack<int32_t, 2> pk_i32x2;
typedef HostPack<int32_t, 1> pk_i32x1;
typedef HostPack<float, 4> pk_f32x4;
typedef HostPack<float, 2> pk_f32x2;
typedef HostPack<float, 1> pk_f32x1;
#endif

template <int VEC>
struct Pack;
template <>
struct Pack<4> {
  typedef pk_i32x4 I;
  typedef pk_f32x4 F;
};
template <>
struct Pack<2> {
  typedef pk_i32x2 I;
  typedef pk_f32x2 F;
};
template <>
struct Pack<1> {
  typedef pk_i32x1 I;
  typedef pk_f32x1 F;
};

#define PCSDF_GLOBAL_IO(T)                                           \
  __device__ __forceinline__ T ld_global(const T *p) {              \
    return *(PCSDF_GLOBAL_AS const T *)p;                            \
  }
PCSDF_GLOBAL_IO(pk_i32x4)
PCSDF_GLOBAL_IO(pk_i32x2)
PCSDF_GLOBAL_IO(pk_i32x1)
PCSDF_GLOBAL_IO(pk_f32x4)
PCSDF_GLOBAL_IO(pk_f32x2)
PCSDF_GLOBAL_IO(pk_f32x1)
#undef PCSDF_GLOBAL_IO

template <int VEC>
__device__ __forceinline__ typename Pack<VEC>::I load_i32(const int32_t *p) {
  return ld_global(reinterpret_cast<const typename Pack<VEC>::I *>(p));
}
// The outputs are written once and not read back by the kernel: stores
// with the nontemporal hint (no write-allocation in the caches; measured
// as fast at 256 x 256 x 128 and up to a quarter faster on smaller grids).
template <int VEC>
__device__ __forceinline__ void store_i32(int32_t *p,
                                          typename Pack<VEC>::I v) {
  __builtin_nontemporal_store(v, reinterpret_cast<typename Pack<VEC>::I *>(p));
}
template <int VEC>
__device__ __forceinline__ void store_f32(float *p, typename Pack<VEC>::F v) {
  __builtin_nontemporal_store(v, reinterpret_cast<typename Pack<VEC>::F *>(p));
}

// Pack shape of the streaming epilogue: `vec` voxels per lane (4, 2 or 1),
// set by V and the alignment of the three streams; `gather` when the
// plane size is not a multiple of vec, so that the vec planar values are
// read one by one (a pack may then cross a layer boundary).
struct PackShape {
  int vec;
  bool gather;
};
__host__ __device__ inline PackShape composite_shape(int64_t plane, int64_t V,
                                                     const void *S,
                                                     const void *oc,
                                                     const void *of) {
  const uintptr_t a = (uintptr_t)S | (uintptr_t)oc | (uintptr_t)of;
  if (V % 4 == 0 && !(a & 15)) return PackShape{4, plane % 4 != 0};
  if (V % 2 == 0 && !(a & 7)) return PackShape{2, plane % 2 != 0};
  return PackShape{1, false};
}

// Planar index and layer of voxels v0 .. v0+VEC-1.  Without kGather they
// share one layer and are consecutive in the plane; with it, each voxel
// gets its own (a pack may cross layer boundaries, several when the
// plane holds fewer than VEC pixels).
template <int VEC, bool kGather>
struct PackCoords {
  uint32_t pix[kGather ? VEC : 1];
  int k[kGather ? VEC : 1];
};
template <int VEC, bool kGather>
__device__ __forceinline__ PackCoords<VEC, kGather> pack_coords(
    uint32_t v0, uint32_t plane) {
  PackCoords<VEC, kGather> c;
  const uint32_t k0 = v0 / plane;
  uint32_t pix = v0 - k0 * plane;
  int kk = (int)k0;
#pragma unroll
  for (int e = 0; e < (kGather ? VEC : 1); ++e) {
    c.pix[e] = pix;
    c.k[e] = kk;
    if (++pix == plane) {  // pix < plane before the step
      pix = 0;
      ++kk;
    }
  }
  return c;
}

// Element `byte_off` bytes past a base pointer.  With a base that is the
// same for the whole wave and a 32-bit offset, the access is a global
// instruction with the base in scalar registers and only the offset in a
// vector register, so no 64-bit address arithmetic runs per lane.
template <class T>
__device__ __forceinline__ T *at_bytes(T *base, uint32_t byte_off) {
  return reinterpret_cast<T *>(
      reinterpret_cast<typename std::conditional<
          std::is_const<T>::value, const char, char>::type *>(base) +
      byte_off);
}

// The VEC planar values of a pack in slice plane Ps.
template <int VEC, bool kGather>
__device__ __forceinline__ typename Pack<VEC>::I load_planar(
    const int32_t *Ps, const PackCoords<VEC, kGather> &c) {
  if constexpr (kGather) {
    typename Pack<VEC>::I p;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      p[e] = ld_global(reinterpret_cast<const pk_i32x1 *>(
          at_bytes(Ps, c.pix[e] * 4u)))[0];
    return p;
  } else {
    return load_i32<VEC>(at_bytes(Ps, c.pix[0] * 4u));
  }
}

// Slices whose planar packs one lane loads before it stores any of them.
constexpr int kPackSlices = 8;

// The 16-bit copy of the static field (k_static16): values in
// [-32767, 32767] as they are, every other value as kS16Far, which sends
// the reader to the int32 field.
constexpr int32_t kS16Far = -32768;

// The VEC static values of a pack from the 16-bit copy, sign-extended
// (kS16Far where the int32 field must be read).
template <int VEC>
__device__ __forceinline__ typename Pack<VEC>::I load_s16(const int16_t *p) {
  typename Pack<VEC>::I s;
  if constexpr (VEC == 4) {
    const pk_i32x2 w = ld_global(reinterpret_cast<const pk_i32x2 *>(p));
    s[0] = (int32_t)(int16_t)(w[0] & 0xFFFF);
    s[1] = w[0] >> 16;
    s[2] = (int32_t)(int16_t)(w[1] & 0xFFFF);
    s[3] = w[1] >> 16;
  } else if constexpr (VEC == 2) {
    const pk_i32x1 w = ld_global(reinterpret_cast<const pk_i32x1 *>(p));
    s[0] = (int32_t)(int16_t)(w[0] & 0xFFFF);
    s[1] = w[0] >> 16;
  } else {
    s[0] = p[0];
  }
  return s;
}

// Voxels v0 .. v0+VEC-1 (v0 a multiple of VEC, all in [0, V)) for slices
// [s_begin, s_end); with kNeed, slices with need[sl] == 0 are skipped (a
// template parameter so that without it the stores are unconditional).
//
// One counter tracks a wave's outstanding vector loads and stores in issue
// order, so a load issued after a store can only be waited for together
// with that store.  The lane therefore issues the static load and the
// planar loads of up to kPackSlices slices first, and only then computes
// and stores them, so that no load waits behind the lane's own stores.
// (Longer slice groups still measure slower than groups of two or three:
// the blocks in flight then write more slices' outputs at once.)
//
// With S16 (the 16-bit copy of the static field, k_static16) the static
// values come from it and only the far ones from S: every slice group
// reads the static values again, and the copy is half their bytes.
template <int VEC, bool kGather, bool kSsq, bool kSdf, bool kNeed = false>
__device__ __forceinline__ void composite_pack(
    const int32_t *__restrict__ S, const int32_t *__restrict__ P,
    const int32_t *__restrict__ need, int32_t *__restrict__ oc,
    float *__restrict__ of, uint32_t plane, uint32_t V, uint32_t v0,
    int s_begin, int s_end, int Kt, int has_above, float hf,
    const int16_t *__restrict__ S16 = nullptr) {
  const PackCoords<VEC, kGather> pc = pack_coords<VEC, kGather>(v0, plane);
  constexpr int NL = kGather ? VEC : 1;
  HumanLayer hl[NL];
#pragma unroll
  for (int e = 0; e < NL; ++e) {
    hl[e] = human_layer(pc.k[e], Kt, has_above);
#if defined(__clang__)
    // Opaque to the optimiser, which would otherwise apply the addition
    // under a select of its own in the loop (one more instruction per
    // voxel and slice).
    asm("" : "+v"(hl[e].lo), "+v"(hl[e].add));
#endif
  }
  // V <= 2^30, so byte offsets within one slice fit in 32 bits.
  const uint32_t vb = v0 * 4u;
  typename Pack<VEC>::I s = S16 ? load_s16<VEC>(at_bytes(S16, v0 * 2u))
                                : load_i32<VEC>(at_bytes(S, vb));
  for (int sl0 = s_begin; sl0 < s_end; sl0 += kPackSlices) {
    const int cnt = min(kPackSlices, s_end - sl0);
    typename Pack<VEC>::I p[kPackSlices];
#pragma unroll
    for (int j = 0; j < kPackSlices; ++j)
      if (j < cnt && !(kNeed && need[sl0 + j] == 0))
        p[j] = load_planar<VEC, kGather>(P + (size_t)(sl0 + j) * plane, pc);
    if (S16 && sl0 == s_begin) {
      // the far values from the int32 field (after the planar loads are
      // issued, so that only the static load is waited for)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (s[e] == kS16Far)
          s[e] = ld_global(reinterpret_cast<const pk_i32x1 *>(
              at_bytes(S, vb + 4u * e)))[0];
    }
#pragma unroll
    for (int j = 0; j < kPackSlices; ++j) {
      if (j >= cnt) break;
      const int sl = sl0 + j;
      if (kNeed && need[sl] == 0) continue;
      typename Pack<VEC>::I c;
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        c[e] = min(s[e], human_value(p[j][e], hl[kGather ? e : 0]));
      if (kSsq) store_i32<VEC>(at_bytes(oc + (size_t)sl * V, vb), c);
      if (kSdf) {
        typename Pack<VEC>::F f;
#pragma unroll
        for (int e = 0; e < VEC; ++e) f[e] = ssq_to_metres(c[e], hf);
        store_f32<VEC>(at_bytes(of + (size_t)sl * V, vb), f);
      }
    }
  }
}

}  // namespace pcsdf
