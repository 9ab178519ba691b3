// Power-normalised RZF precoder W = beta_pow H X (eq. 7, the power factor
// beta = sqrt(P / tr(F^H F)) with F = H X, and eq. 15), streamed along the
// antenna dimension.
//
// beta_pow is known before any W entry is written: the PCG kernel leaves
// per-workgroup partial sums of x_j^H (H^H H) x_j = ||H x_j||^2, summed here in
// a fixed order, so W is written exactly once.
//
// Decomposition: a workgroup of 4 waves covers 128 antennas x (32*NJ) columns
// of W; wave w owns antennas [32w, 32w+32) of the block and NJ 32-column tiles.
// beta_pow * X for the block's columns is staged in LDS once. On
// v_mfma_f32_32x32x2_f32 the two k slots carry users k = s and k = s + K/2, so
// each lane half reads one user's antenna column of H, coalesced along m.
#include "device_util.hpp"

namespace jacpcg {
namespace {

template <int KT, int NJ, bool VEC>
__global__ __launch_bounds__(256) void precoder_f32_kernel(PrecoderLaunch e) {
  constexpr int KP = KT * 32;
  constexpr int KH = KT * 16;
  constexpr int NC = 32 * NJ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jl = lane & 31, half = lane >> 5;
  const int nmb = (e.M + 127) / 128;
  const int ncw = (e.nrhs + NC - 1) / NC;
  const int per = nmb * ncw;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / per;
  const int rem = L - b * per;
  const int mb = rem / ncw, cw = rem - mb * ncw;
  const int K = e.K;

  __shared__ float2 Xs[KP][NC];

  float fs = 0.f;
  for (int c = 0; c < e.ncb; ++c) fs += e.fpart[(int64_t)b * e.ncb + c];
  const float beta = fs > 0.f ? sqrtf(e.power / fs) : 0.f;
  if (e.beta_out && mb == 0 && cw == 0 && threadIdx.x == 0) e.beta_out[b] = beta;

  const float2* Xb = e.X + (int64_t)b * e.stride_x;
  for (int idx = threadIdx.x; idx < KP * NC; idx += 256) {
    const int jj = idx % NC, k = idx / NC;
    const int j = cw * NC + jj;
    float2 v = make_float2(0.f, 0.f);
    if (k < K && j < e.nrhs) {
      v = Xb[(int64_t)j * e.ldx + k];
      v.x *= beta;
      v.y *= beta;
    }
    Xs[k][jj] = v;
  }
  __syncthreads();

  const int m0 = mb * 128 + w * 32;
  const int mrow = m0 + jl;
  const bool mvalid = mrow < e.M;
  const int klim = max(0, min(KH, K - half * KH));
  const float2* hcol = e.H + (int64_t)b * e.stride_h + (int64_t)(half * KH) * e.ldh + (mvalid ? mrow : 0);

  floatx16 wr[NJ], wi[NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) {
    wr[t] = zero16();
    wi[t] = zero16();
  }
  for (int s0 = 0; s0 < KH; s0 += 8) {
    float2 h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int s = s0 + q;
      h[q] = (mvalid && s < klim) ? hcol[(int64_t)s * e.ldh] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        const float2 xv = Xs[half * KH + s0 + q][t * 32 + jl];
        wr[t] = mfma32(h[q].x, xv.x, wr[t]);
        wr[t] = mfma32(h[q].y, -xv.y, wr[t]);
        wi[t] = mfma32(h[q].x, xv.y, wi[t]);
        wi[t] = mfma32(h[q].y, xv.x, wi[t]);
      }
    }
  }

  float2* Wb = e.W + (int64_t)b * e.stride_w;
#pragma unroll
  for (int t = 0; t < NJ; ++t) {
    const int j = cw * NC + t * 32 + jl;
    if (j >= e.nrhs) continue;
    float2* wc = Wb + (int64_t)j * e.ldw;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int m = m0 + 8 * g + 4 * half;
      if (VEC && m + 4 <= e.M) {
        float4* dst = reinterpret_cast<float4*>(wc + m);
        dst[0] = make_float4(wr[t][4 * g + 0], wi[t][4 * g + 0], wr[t][4 * g + 1], wi[t][4 * g + 1]);
        dst[1] = make_float4(wr[t][4 * g + 2], wi[t][4 * g + 2], wr[t][4 * g + 3], wi[t][4 * g + 3]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (m + q < e.M) wc[m + q] = make_float2(wr[t][4 * g + q], wi[t][4 * g + q]);
      }
    }
  }
}

template <int KT>
hipError_t launch_kt(const PrecoderLaunch& e, hipStream_t s) {
  const int nmb = (e.M + 127) / 128;
  const bool vec = ((uintptr_t)e.W % 16 == 0) && (e.ldw % 2 == 0) && (e.stride_w % 2 == 0);
  // Two column tiles per wave halve the reads of H; LDS caps it at K <= 128.
  if constexpr (KT <= 4) {
    if (e.nrhs > 32) {
      const int grid = e.batch * nmb * ((e.nrhs + 63) / 64);
      if (vec)
        hipLaunchKernelGGL((precoder_f32_kernel<KT, 2, true>), dim3(grid), dim3(256), 0, s, e);
      else
        hipLaunchKernelGGL((precoder_f32_kernel<KT, 2, false>), dim3(grid), dim3(256), 0, s, e);
      return hipGetLastError();
    }
  }
  {
    const int grid = e.batch * nmb * ((e.nrhs + 31) / 32);
    if (vec)
      hipLaunchKernelGGL((precoder_f32_kernel<KT, 1, true>), dim3(grid), dim3(256), 0, s, e);
    else
      hipLaunchKernelGGL((precoder_f32_kernel<KT, 1, false>), dim3(grid), dim3(256), 0, s, e);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_precoder(const PrecoderLaunch& e, hipStream_t s) {
  if (e.batch == 0) return hipSuccess;
  switch ((e.K + 31) / 32) {
    case 1: return launch_kt<1>(e, s);
    case 2: return launch_kt<2>(e, s);
    case 3: return launch_kt<3>(e, s);
    case 4: return launch_kt<4>(e, s);
    case 5: return launch_kt<5>(e, s);
    case 6: return launch_kt<6>(e, s);
    case 7: return launch_kt<7>(e, s);
    case 8: return launch_kt<8>(e, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace jacpcg
