// Application-level evaluation of a precoder on its channel (Sec. II, eqs. 8-10):
// user k receives h_k^H g_k s_k, the leakage h_k^H g_j s_j of every other
// user's precoding vector, and noise of power sigma2, so
//   SINR_k = |h_k^H g_k|^2 / (sum_{j != k} |h_k^H g_j|^2 + sigma2),
//   SE     = sum_k log2(1 + SINR_k)            (bit/s/Hz per instance).
// With block-structured H and G (eqs. 2 and 6) the same expression gives the
// intra-group and inter-subarray terms of eq. 9.
//
// Two kernels: C = H^H W (K x K complex per instance) on the FP32 matrix cores,
// one workgroup per (instance, 32 x 32 tile of C) whose waves split the antenna
// range and sum their partial tiles in LDS in a fixed order; then one thread
// per user forms its SINR, summing the interference over j != k directly (no
// subtraction of the signal term, so no cancellation), and the instance's sum
// rate is added up in a fixed order.
#include "device_util.hpp"

namespace jacpcg {
namespace {

constexpr int kEvalWaves = 4;

// 8 consecutive complex entries row[m .. m+7], zero past `mend` or for a
// padding row. VEC: 16-byte aligned rows.
template <bool VEC>
__device__ __forceinline__ void ld8(gptr<const float2> row, int m, int mend, bool valid, float2 (&v)[8]) {
  if (VEC && valid && m + 8 <= mend) {
    gptr<const float4> p = reinterpret_cast<gptr<const float4>>(row + m);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = ld4(p + q);
      v[2 * q] = make_float2(t.x, t.y);
      v[2 * q + 1] = make_float2(t.z, t.w);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (valid && m + e < mend) ? ld2(row + m + e) : make_float2(0.f, 0.f);
  }
}

// Tile (ti, tj) of C = H^H W: rows are users i (A operand), columns precoding
// vectors j (B operand). For antenna m the two k slots carry (Re, Im):
//   Re C_ij = Re h_i Re w_j + Im h_i Im w_j,  Im C_ij = Re h_i Im w_j - Im h_i Re w_j.
template <bool VEC>
__global__ __launch_bounds__(64 * kEvalWaves) void cross_f32_kernel(EvalLaunch e) {
  const int nt = (e.K + 31) >> 5;
  const int ntiles = nt * nt;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / ntiles;
  const int t = L - b * ntiles;
  const int ti = t / nt, tj = t - ti * nt;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = lane >> 5, li = lane & 31;
  const int ui = ti * 32 + li, uj = tj * 32 + li;
  const bool vi = ui < e.K, vj = uj < e.K;
  gptr<const float2> hrow = as_global(e.H + (int64_t)b * e.stride_h) + (int64_t)(vi ? ui : 0) * e.ldh;
  gptr<const float2> wrow = as_global(e.W + (int64_t)b * e.stride_w) + (int64_t)(vj ? uj : 0) * e.ldw;

  const int chunk = ((e.M + kEvalWaves * 8 - 1) / (kEvalWaves * 8)) * 8;
  const int m0 = wave * chunk;
  const int m1 = min(e.M, m0 + chunk);
  floatx16 accR = zero16(), accI = zero16();
  for (int m = m0; m < m1; m += 8) {
    float2 a[8], c[8];
    ld8<VEC>(hrow, m, m1, vi, a);
    ld8<VEC>(wrow, m, m1, vj, c);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float av = half ? a[q].y : a[q].x;
      const float br = half ? c[q].y : c[q].x;
      const float bi = half ? -c[q].x : c[q].y;
      accR = mfma32(av, br, accR);
      accI = mfma32(av, bi, accI);
    }
  }

  __shared__ float red[kEvalWaves][2][16][64];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    red[wave][0][r][lane] = accR[r];
    red[wave][1][r][lane] = accI[r];
  }
  __syncthreads();
  // Tile element (i, j) sits in lane j + 32 * ((i >> 2) & 1), register 4 * (i >> 3) + (i & 3).
  gptr<float2> Cb = as_global(e.C + (int64_t)b * e.K * e.K);
  for (int idx = threadIdx.x; idx < 1024; idx += 64 * kEvalWaves) {
    const int i = idx >> 5, j = idx & 31;
    const int gi = ti * 32 + i, gj = tj * 32 + j;
    if (gi < e.K && gj < e.K) {
      const int l = j + 32 * ((i >> 2) & 1), r = 4 * (i >> 3) + (i & 3);
      float re = 0.f, im = 0.f;
      for (int w = 0; w < kEvalWaves; ++w) {
        re += red[w][0][r][l];
        im += red[w][1][r][l];
      }
      st2(Cb + (int64_t)gi * e.K + gj, re, im);
    }
  }
}

__global__ __launch_bounds__(256) void sinr_kernel(EvalLaunch e) {
  const int b = blockIdx.x;
  const int k = threadIdx.x;
  __shared__ float rate[256];
  float r = 0.f;
  if (k < e.K) {
    gptr<const float2> row = as_global(e.C + ((int64_t)b * e.K + k) * e.K);
    float interf = 0.f, sig = 0.f;
    for (int j = 0; j < e.K; ++j) {
      const float2 c = ld2(row + j);
      const float p = c.x * c.x + c.y * c.y;
      if (j == k)
        sig = p;
      else
        interf += p;
    }
    const float s = sig / (interf + e.sigma2);
    e.sinr[(int64_t)b * e.K + k] = s;
    r = log2f(1.f + s);
  }
  rate[k] = r;
  __syncthreads();
  if (k == 0 && e.se) {
    double sum = 0.0;
    for (int q = 0; q < e.K; ++q) sum += rate[q];
    e.se[b] = (float)sum;
  }
}

}  // namespace

hipError_t launch_eval(const EvalLaunch& e, hipStream_t s) {
  if (e.batch == 0) return hipSuccess;
  if (e.K > 256) return hipErrorInvalidValue;
  const int nt = (e.K + 31) / 32;
  const bool vec = ((uintptr_t)e.H % 16 == 0) && ((uintptr_t)e.W % 16 == 0) && e.ldh % 2 == 0 &&
                   e.ldw % 2 == 0 && e.stride_h % 2 == 0 && e.stride_w % 2 == 0;
  const dim3 grid((unsigned)(e.batch * nt * nt)), block(64 * kEvalWaves);
  if (vec)
    hipLaunchKernelGGL(cross_f32_kernel<true>, grid, block, 0, s, e);
  else
    hipLaunchKernelGGL(cross_f32_kernel<false>, grid, block, 0, s, e);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(sinr_kernel, dim3((unsigned)e.batch), dim3(256), 0, s, e);
  return hipGetLastError();
}

}  // namespace jacpcg
