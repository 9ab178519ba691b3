// Visibility-region sparsity of the Gram matrix (Sec. II, eq. 4; Sec. III:
// the regularised Gram P_i is sparse). D_k is binary, so user k's channel is
// zero outside its visibility region and A_ij = h_i^H h_j = 0 when the
// regions of users i and j do not overlap. This file forms, per instance and
// per 32-user block of A, the antenna span [x, y) that holds every nonzero
// channel entry of the block's users: the Gram tile (i, j) then needs only
// antennas in the overlap of blocks i and j, and a tile whose blocks' spans
// are disjoint is exactly zero (skipped by the solver).
//
// The per-user spans come from the caller (the regions are a property of the
// channel model) or are found here by scanning H for its first and last
// nonzero entry per user.
#include "device_util.hpp"

namespace jacpcg {
namespace {

// One workgroup per (instance, 32-user block); wave w handles users
// 8w .. 8w+7 of the block, lanes stride over the antennas.
__global__ __launch_bounds__(256) void span_kernel(SpanLaunch sl) {
  const int nt = (sl.K + 31) >> 5;
  const int b = blockIdx.x / nt, t = blockIdx.x - b * nt;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ int lo_s[32], hi_s[32];
  for (int q = 0; q < 8; ++q) {
    const int ul = w * 8 + q, u = t * 32 + ul;
    int lo = sl.M, hi = 0;  // empty span
    if (u < sl.K) {
      if (sl.user_span_in) {
        if (lane == 0) {
          lo = max(0, sl.user_span_in[((int64_t)b * sl.K + u) * 2]);
          hi = min(sl.M, sl.user_span_in[((int64_t)b * sl.K + u) * 2 + 1]);
        }
      } else {
        gptr<const float2> row = as_global(sl.H + (int64_t)b * sl.stride_h + (int64_t)u * sl.ldh);
        for (int m = lane; m < sl.M; m += 64) {
          const float2 v = ld2(row + m);
          if (v.x != 0.f || v.y != 0.f) {
            lo = min(lo, m);
            hi = max(hi, m + 1);
          }
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o));
      hi = max(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) {
      lo_s[ul] = lo;
      hi_s[ul] = hi;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int lo = sl.M, hi = 0;
    for (int q = 0; q < 32; ++q) {
      lo = min(lo, lo_s[q]);
      hi = max(hi, hi_s[q]);
    }
    if (hi <= lo) lo = hi = 0;  // no nonzero channel in the block
    sl.tile_span[(int64_t)b * nt + t] = make_int2(lo, hi);
  }
}

}  // namespace

hipError_t launch_spans(const SpanLaunch& sl, hipStream_t s) {
  if (sl.batch == 0) return hipSuccess;
  const int nt = (sl.K + 31) / 32;
  hipLaunchKernelGGL(span_kernel, dim3((unsigned)(sl.batch * nt)), dim3(256), 0, s, sl);
  return hipGetLastError();
}

}  // namespace jacpcg
