// FP64 side of the path: widening of FP32 solutions (more kernels of the
// FP64-residual refinement live here).
#include "device_util.hpp"

namespace jacpcg {
namespace {

__global__ void widen_kernel(const float2* __restrict__ X, int64_t ldx, int64_t stride_x, int K, int n,
                             double2* __restrict__ out) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * n) return;
  const int j = idx / K, i = idx - j * K;
  const float2 v = X[(int64_t)b * stride_x + (int64_t)j * ldx + i];
  out[(int64_t)b * K * n + idx] = make_double2(v.x, v.y);
}

}  // namespace

hipError_t launch_widen(const float2* X, int64_t ldx, int64_t stride_x, int batch, int K, int n, double2* out,
                        hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3((K * n + 255) / 256, batch), dim3(256), 0, s, X, ldx, stride_x, K, n, out);
  return hipGetLastError();
}

}  // namespace jacpcg
