// Matrix-core peak probe: register-only loops of independent MFMA chains for
// the instruction shapes the kernels use (FP32 32x32x2, BF16 32x32x16, FP64
// 16x16x4) and the int8 32x32x32 shape, timed with HIP events. The measured
// rates are the ceilings the kernels' matrix-core utilisation is read against.
#include <hip/hip_runtime.h>

#include "../../include/jacpcg.h"
#include "device_util.hpp"
#include "session.hpp"

namespace jacpcg {
namespace {

typedef int int32x16 __attribute__((ext_vector_type(16)));
typedef int int32x4 __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;   // independent accumulators per wave
constexpr int kPeakIters = 1024;

// Each kind runs kPeakIters x kChains MFMAs per wave on register operands; the
// accumulators are reduced into one value per lane and stored, so nothing is
// dead code.
__global__ __launch_bounds__(256) void peak_f32_kernel(float* out, float seed) {
  floatx16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = zero16();
  const float a = seed + threadIdx.x * 1e-7f, b = seed - threadIdx.x * 1e-7f;
  for (int i = 0; i < kPeakIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][threadIdx.x & 15];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void peak_bf16_kernel(float* out, float seed) {
  floatx16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = zero16();
  u32x4 a, b;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    a[e] = pack_bf16x2(seed + e, seed - e + threadIdx.x * 1e-3f);
    b[e] = pack_bf16x2(seed * 0.5f + e, seed + threadIdx.x * 1e-3f);
  }
  for (int i = 0; i < kPeakIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = mfma_bf16(a, b, acc[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][threadIdx.x & 15];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void peak_f64_kernel(float* out, float seed) {
  doublex4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c][0] = acc[c][1] = acc[c][2] = acc[c][3] = 0.0;
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
  for (int i = 0; i < kPeakIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][threadIdx.x & 3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

__global__ __launch_bounds__(256) void peak_i8_kernel(float* out, float seed) {
  int32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0;
  const int s8 = (int)seed;
  int32x4 av, bv;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    av[e] = (s8 + e + (int)threadIdx.x) & 0x3f3f3f3f;
    bv[e] = (s8 * 3 + e) & 0x3f3f3f3f;
  }
  for (int i = 0; i < kPeakIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc[c], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][threadIdx.x & 15];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

}  // namespace
}  // namespace jacpcg

using namespace jacpcg;

extern "C" int jacpcg_mfma_peaks(jacpcg_session* s, void* stream, double* tflops) {
  if (!s || !tflops) return set_error(JACPCG_E_INVALID_ARG, "session and output must not be NULL");
  if (hipSetDevice(s->device) != hipSuccess) return set_error(JACPCG_E_HIP, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) return set_error(JACPCG_E_HIP, "device properties");
  // Two 4-wave workgroups per compute unit: two waves per SIMD, each with
  // eight independent accumulation chains.
  const int grid = prop.multiProcessorCount * 2;
  float* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)grid * 256 * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(JACPCG_E_OUT_OF_MEMORY, "probe output allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // flops per MFMA instruction per wave: 2 m n k
  const double per_mfma[4] = {2.0 * 32 * 32 * 2, 2.0 * 32 * 32 * 16, 2.0 * 16 * 16 * 4, 2.0 * 32 * 32 * 32};
  int rc = JACPCG_OK;
  for (int kind = 0; kind < 4 && rc == JACPCG_OK; ++kind) {
    auto launch = [&] {
      switch (kind) {
        case 0: hipLaunchKernelGGL(peak_f32_kernel, dim3(grid), dim3(256), 0, st, out, 1.0f); break;
        case 1: hipLaunchKernelGGL(peak_bf16_kernel, dim3(grid), dim3(256), 0, st, out, 1.0f); break;
        case 2: hipLaunchKernelGGL(peak_f64_kernel, dim3(grid), dim3(256), 0, st, out, 1.0f); break;
        default: hipLaunchKernelGGL(peak_i8_kernel, dim3(grid), dim3(256), 0, st, out, 1.0f); break;
      }
    };
    launch();  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 5; ++r) launch();
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
      rc = set_error(JACPCG_E_HIP, "probe kernel failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double mfmas = 5.0 * grid * 4 /* waves */ * kPeakIters * kChains;
    tflops[kind] = mfmas * per_mfma[kind] / (ms * 1e-3) / 1e12;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return rc;
}
