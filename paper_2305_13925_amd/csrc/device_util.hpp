// Small device helpers shared by the kernels of libjacpcg.
#pragma once

#include "common.hpp"

namespace jacpcg {

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, and each
// XCD has its own L2. Re-number workgroups so that consecutive logical indices
// (the tiles of one instance, which read the same channel / system matrix) run
// on the same XCD. Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_remap(int g, int n) {
  if ((n & 7) != 0) return g;
  return (g & 7) * (n >> 3) + (g >> 3);
}

// Global-memory (address space 1) view of a generic pointer. Accesses through
// it compile to global_* instructions, which only the vector-memory counter
// tracks. Through a generic pointer (one selected from a pointer array or a
// base + offset) they become flat_* instructions, which the LDS counter tracks
// as well, so every LDS read would also wait for all loads still in flight.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

typedef float gfloat2 __attribute__((ext_vector_type(2)));
// Complex entry p[0] through a global pointer (one 8-byte load).
__device__ __forceinline__ float2 ld2(gptr<const float2> p) {
  const gfloat2 v = *reinterpret_cast<gptr<const gfloat2>>(p);
  return make_float2(v.x, v.y);
}
typedef double gdouble2 __attribute__((ext_vector_type(2)));
// Complex FP64 entry p[0] through a global pointer (one 16-byte load).
__device__ __forceinline__ double2 ld2d(gptr<const double2> p) {
  const gdouble2 v = *reinterpret_cast<gptr<const gdouble2>>(p);
  return make_double2(v.x, v.y);
}
typedef float gfloat4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(gptr<const float4> p) {
  const gfloat4 v = *reinterpret_cast<gptr<const gfloat4>>(p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(gptr<float4> p, float a, float b, float c, float d) {
  *reinterpret_cast<gptr<gfloat4>>(p) = gfloat4{a, b, c, d};
}
__device__ __forceinline__ void st2(gptr<float2> p, float re, float im) {
  *reinterpret_cast<gptr<gfloat2>>(p) = gfloat2{re, im};
}
// Streaming stores for outputs nothing reads back soon (the precoder W): they
// bypass cache allocation, so no dirty lines are left for later kernels'
// reads to write back.
__device__ __forceinline__ void st4_nt(gptr<float4> p, float a, float b, float c, float d) {
  __builtin_nontemporal_store(gfloat4{a, b, c, d}, reinterpret_cast<gptr<gfloat4>>(p));
}
__device__ __forceinline__ void st2_nt(gptr<float2> p, float re, float im) {
  __builtin_nontemporal_store(gfloat2{re, im}, reinterpret_cast<gptr<gfloat2>>(p));
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx16 zero16() {
  floatx16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

}  // namespace jacpcg

namespace jacpcg {

// ---------------------------------------------------------------------------
// Split-BF16 products. An FP32 value x is written as a sum of NS bfloat16
// parts, each the round-to-nearest bfloat16 of what the previous parts left:
// NS = 2 gives x ~ hi + lo (16 significant bits), NS = 3 gives x = hi + mid + lo
// exactly (8 + 8 + 8 bits, |mid| <= 2^-8 |x|, |lo| <= 2^-16 |x|). Products of
// parts are exact in the MFMA's FP32 accumulation. With NS = 3, keeping hi*hi,
// hi*mid, mid*hi, hi*lo, lo*hi and mid*mid drops mid*lo, lo*mid and lo*lo, at
// most 2^-23 of the product together: the size of one FP32 rounding. With
// NS = 2 (hi*hi + hi*lo + lo*hi) the dropped part is up to ~2^-16.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatv2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const floatv2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf16_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// Split 8 floats (4 packed pairs: x[0..1], x[2..3], ...) into NS bf16 parts of
// 4 packed pairs each.
template <int NS>
__device__ __forceinline__ void split8(const float (&x)[8], u32x4 (&parts)[NS]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float a = x[2 * q], b = x[2 * q + 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const uint32_t p = pack_bf16x2(a, b);
      parts[s][q] = p;
      if (s + 1 < NS) {
        a -= bf16_lo(p);
        b -= bf16_hi(p);
      }
    }
  }
}

// Negate every bf16 of a packed pair.
__device__ __forceinline__ uint32_t neg_bf16x2(uint32_t p) { return p ^ 0x80008000u; }
// (re, im) packed pair -> (im, -re)
__device__ __forceinline__ uint32_t rot_neg_hi(uint32_t p) { return ((p >> 16) | (p << 16)) ^ 0x80000000u; }
// (re, -im) packed pair -> (im, re)
__device__ __forceinline__ uint32_t rot_neg_lo(uint32_t p) { return ((p >> 16) | (p << 16)) ^ 0x00008000u; }

__device__ __forceinline__ floatx16 mfma_bf16(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// acc += the significant part products of a*b, smallest first. One MFMA adds 16
// products into the FP32 accumulator, so a split-BF16 product chain rounds less
// often than the FP32 MFMA chain it replaces (which adds 2 products per step).
template <int NS>
__device__ __forceinline__ void split_mma(const u32x4 (&a)[NS], const u32x4 (&b)[NS], floatx16& acc) {
  if constexpr (NS >= 3) {
    acc = mfma_bf16(a[1], b[1], acc);
    acc = mfma_bf16(a[0], b[2], acc);
    acc = mfma_bf16(a[2], b[0], acc);
  }
  acc = mfma_bf16(a[0], b[1], acc);
  acc = mfma_bf16(a[1], b[0], acc);
  acc = mfma_bf16(a[0], b[0], acc);
}

}  // namespace jacpcg
