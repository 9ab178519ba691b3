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
