// FP64 side of the path: the FP64 Gram A64 = H^H H + xi I (from the same
// complex64 channel, widened exactly), the refinement residual R = B - A64 X64
// with its column norms, and the FP64 accumulation X64 += scale * E of the
// FP32 correction solves. Iterative refinement is not in the paper; it wins
// back the accuracy the FP32 (or split-BF16) Gram and the FP32 solve lose.
//
// v_mfma_f64_16x16x4_f64 layout: A-operand lane l holds A[l%16][l/16],
// B-operand B[l/16][l%16], result register r of lane l is D[l/16 + 4r][l%16].
// The four k slots carry two complex terms as (Re, Im) pairs.
#include "device_util.hpp"

namespace jacpcg {
namespace {

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 zero4d() {
  doublex4 z;
  z[0] = z[1] = z[2] = z[3] = 0.0;
  return z;
}

__device__ __forceinline__ void upper_tile16(int t, int nt, int& ti, int& tj) {
  int i = 0;
  while (t >= nt - i) {
    t -= nt - i;
    ++i;
  }
  ti = i;
  tj = i + t;
}

// One workgroup per (instance, 16x16 tile of the upper triangle); 4 waves split
// the antennas, partial tiles summed in LDS in wave order.
__global__ __launch_bounds__(256) void gram64_kernel(Gram64Launch g) {
  const int nt = (g.K + 15) >> 4;
  const int ntiles = nt * (nt + 1) / 2;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / ntiles;
  int ti, tj;
  upper_tile16(L - b * ntiles, nt, ti, tj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, li = lane & 15;
  const int slot_m = q >> 1, comp = q & 1;
  const float2* Hb = g.H + (int64_t)b * g.stride_h;
  const int ui = ti * 16 + li, uj = tj * 16 + li;
  const bool vi = ui < g.K, vj = uj < g.K;
  const float2* hi = Hb + (int64_t)(vi ? ui : 0) * g.ldh;
  const float2* hj = Hb + (int64_t)(vj ? uj : 0) * g.ldh;
  const int chunk = ((g.M + 4 * 8 - 1) / (4 * 8)) * 8;
  const int m0 = wave * chunk;
  const int m1 = min(g.M, m0 + chunk);

  doublex4 accR = zero4d(), accI = zero4d();
  for (int m = m0; m < m1; m += 8) {
    float2 a[4], c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int mm = m + 2 * u + slot_m;
      a[u] = (vi && mm < m1) ? hi[mm] : make_float2(0.f, 0.f);
      c[u] = (vj && mm < m1) ? hj[mm] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double av = comp ? (double)a[u].y : (double)a[u].x;
      const double br = comp ? (double)c[u].y : (double)c[u].x;
      const double bi = comp ? -(double)c[u].x : (double)c[u].y;
      accR = mfma64(av, br, accR);
      accI = mfma64(av, bi, accI);
    }
  }

  __shared__ double red[4][2][4][64];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    red[wave][0][r][lane] = accR[r];
    red[wave][1][r][lane] = accI[r];
  }
  __syncthreads();
  // element (i, j) of the tile: lane j + 16*(i%4), register i/4
  auto tile = [&](int i, int j, double& re, double& im) {
    const int l = j + 16 * (i & 3), r = i >> 2;
    re = 0.0;
    im = 0.0;
    for (int w = 0; w < 4; ++w) {
      re += red[w][0][r][l];
      im += red[w][1][r][l];
    }
  };
  const bool same = ti == tj;
  double2* Ab = g.A64 + (int64_t)b * g.K * g.K;
  const int e = threadIdx.x;  // 256 threads, one tile element each
  const int i = e >> 4, j = e & 15;
  const int gi = ti * 16 + i, gj = tj * 16 + j;
  if (gi < g.K && gj < g.K) {
    double re, im;
    if (!same || i < j) {
      tile(i, j, re, im);
    } else if (i > j) {
      tile(j, i, re, im);
      im = -im;
    } else {
      tile(i, i, re, im);
      re += g.xi;
      im = 0.0;
    }
    Ab[(int64_t)gi * g.K + gj] = make_double2(re, im);
  }
  if (!same) {
    const int mi = tj * 16 + i, mj = ti * 16 + j;
    if (mi < g.K && mj < g.K) {
      double re, im;
      tile(j, i, re, im);
      Ab[(int64_t)mi * g.K + mj] = make_double2(re, -im);
    }
  }
}

// R = B - A64 X64 for one instance and 16 columns per workgroup (B = I when
// `identity`). Wave w owns row tiles w, w+4, ... Per column: ||r_j||^2, the
// FP32 right-hand side r_j / ||r_j|| of the next correction solve, and
// Re x_j^H (A64 - xi I) x_j = ||H x_j||^2 (FP64, no cancellation problem).
constexpr int kResMaxRowTiles = 4;  // K <= 256: 16 row tiles over 4 waves

__global__ __launch_bounds__(256) void residual64_kernel(ResidualLaunch r) {
  const int n16 = (r.nrhs + 15) >> 4;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / n16, cb = L - b * n16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, li = lane & 15;
  const int slot_k = q >> 1, comp = q & 1;
  const int K = r.K;
  const int j = cb * 16 + li;
  const bool jv = j < r.nrhs;
  const double2* Ab = r.A64 + (int64_t)b * K * K;
  const double2* Xb = r.X64 + (int64_t)b * K * r.nrhs;
  const int ntr = (K + 15) >> 4;

  doublex4 qr[kResMaxRowTiles], qi[kResMaxRowTiles];
#pragma unroll
  for (int t = 0; t < kResMaxRowTiles; ++t) {
    qr[t] = zero4d();
    qi[t] = zero4d();
    const int rt = w + 4 * t;
    if (rt >= ntr) continue;
    const int ia = rt * 16 + li;  // A-operand row
    for (int k0 = 0; k0 < K; k0 += 2) {
      const int kk = k0 + slot_k;
      const double2 a = (ia < K && kk < K) ? Ab[(int64_t)ia * K + kk] : make_double2(0.0, 0.0);
      const double2 x = (jv && kk < K) ? Xb[(int64_t)j * K + kk] : make_double2(0.0, 0.0);
      const double av = comp ? a.y : a.x;
      qr[t] = mfma64(av, comp ? -x.y : x.x, qr[t]);
      qi[t] = mfma64(av, comp ? x.x : x.y, qi[t]);
    }
  }
  // Own rows of the result: rt*16 + q + 4*reg, column j.
  double nr = 0.0, quad = 0.0;
  double rre[kResMaxRowTiles][4], rim[kResMaxRowTiles][4];
#pragma unroll
  for (int t = 0; t < kResMaxRowTiles; ++t) {
    const int rt = w + 4 * t;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int i = rt * 16 + q + 4 * g;
      rre[t][g] = 0.0;
      rim[t][g] = 0.0;
      if (rt >= ntr || i >= K || !jv) continue;
      double2 bv = make_double2(0.0, 0.0);
      if (r.B) {
        const float2 bf = r.B[(int64_t)b * r.ldb_stride + (int64_t)j * r.ldb + i];  // caller's B
        bv = make_double2(bf.x, bf.y);
      } else if (i == j) {
        bv.x = 1.0;
      }
      rre[t][g] = bv.x - qr[t][g];
      rim[t][g] = bv.y - qi[t][g];
      nr += rre[t][g] * rre[t][g] + rim[t][g] * rim[t][g];
      const double2 x = Xb[(int64_t)j * K + i];
      quad += x.x * qr[t][g] + x.y * qi[t][g] - r.xi * (x.x * x.x + x.y * x.y);
    }
  }
  // column sums: the 4 lane groups of a wave, then the 4 waves (fixed order)
  nr += __shfl_xor(nr, 16);
  nr += __shfl_xor(nr, 32);
  quad += __shfl_xor(quad, 16);
  quad += __shfl_xor(quad, 32);
  __shared__ double cs[2][4][16];
  if (q == 0) {
    cs[0][w][li] = nr;
    cs[1][w][li] = quad;
  }
  __syncthreads();
  nr = cs[0][0][li] + cs[0][1][li] + cs[0][2][li] + cs[0][3][li];
  const double sc = sqrt(nr);
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
#pragma unroll
  for (int t = 0; t < kResMaxRowTiles; ++t) {
    const int rt = w + 4 * t;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int i = rt * 16 + q + 4 * g;
      if (rt < ntr && i < K && jv)
        r.R32[(int64_t)b * K * r.nrhs + (int64_t)j * K + i] =
            make_float2((float)(rre[t][g] * inv), (float)(rim[t][g] * inv));
    }
  }
  if (w == 0 && q == 0 && jv) r.scale[(int64_t)b * r.nrhs + j] = sc;
  if (threadIdx.x == 0) {
    double s = 0.0, s2 = 0.0;
    for (int c = 0; c < 16; ++c) {
      s += cs[0][0][c] + cs[0][1][c] + cs[0][2][c] + cs[0][3][c];
      s2 += cs[1][0][c] + cs[1][1][c] + cs[1][2][c] + cs[1][3][c];
    }
    r.rnorm2[L] = s;
    r.quad[L] = s2;
  }
}

__global__ void accumulate_kernel(AccumulateLaunch a) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.K * a.nrhs) return;
  const int j = idx / a.K;
  const int64_t o = (int64_t)b * a.K * a.nrhs + idx;
  const float2 e = a.E[o];
  double2 x;
  if (a.first) {
    x = make_double2(e.x, e.y);
  } else {
    const double s = a.scale[(int64_t)b * a.nrhs + j];
    x = a.X64[o];
    x.x += s * (double)e.x;
    x.y += s * (double)e.y;
  }
  a.X64[o] = x;
  if (a.X32) a.X32[o] = make_float2((float)x.x, (float)x.y);
}

__global__ void widen_kernel(const float2* __restrict__ X, int64_t ldx, int64_t stride_x, int K, int n,
                             double2* __restrict__ out) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * n) return;
  const int j = idx / K, i = idx - j * K;
  const float2 v = X[(int64_t)b * stride_x + (int64_t)j * ldx + i];
  out[(int64_t)b * K * n + idx] = make_double2(v.x, v.y);
}

// Deterministic pseudo-random complex values (hash of the index), for
// autotuning runs on synthetic data.
__global__ void fill_synthetic_kernel(float2* __restrict__ H, size_t n, uint32_t seed) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)i * 2654435761u ^ seed;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const float a = (float)(h & 0xffff) / 65536.0f - 0.5f;
  const float b = (float)(h >> 16) / 65536.0f - 0.5f;
  H[i] = make_float2(a, b);
}

// Zero rows [row0, row0 + nrows) x columns [col0, col0 + ncols) of a batch of
// column-major matrices (ld, stride): the zero blocks of a block precoder.
__global__ void zero_block_kernel(float2* __restrict__ G, int64_t ld, int64_t stride, int row0, int nrows, int col0,
                                  int ncols, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t per = (int64_t)nrows * ncols;
  const int64_t b = i / per, e = i - b * per;
  const int c = (int)(e / nrows), r = (int)(e - (int64_t)c * nrows);
  G[b * stride + (int64_t)(col0 + c) * ld + row0 + r] = make_float2(0.f, 0.f);
}

}  // namespace

hipError_t launch_zero_block(float2* G, int64_t ld, int64_t stride, int batch, int row0, int nrows, int col0,
                             int ncols, hipStream_t s) {
  const int64_t total = (int64_t)batch * nrows * ncols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_block_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G, ld, stride, row0,
                     nrows, col0, ncols, total);
  return hipGetLastError();
}

hipError_t launch_fill_synthetic(float2* H, size_t n, uint32_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_synthetic_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, H, n, seed);
  return hipGetLastError();
}

hipError_t launch_gram64(const Gram64Launch& g, hipStream_t s) {
  if (g.batch == 0) return hipSuccess;
  const int nt = (g.K + 15) / 16;
  hipLaunchKernelGGL(gram64_kernel, dim3(nt * (nt + 1) / 2 * g.batch), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualLaunch& r, hipStream_t s) {
  if (r.batch == 0) return hipSuccess;
  if (r.K > 16 * 4 * kResMaxRowTiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(residual64_kernel, dim3(r.batch * ((r.nrhs + 15) / 16)), dim3(256), 0, s, r);
  return hipGetLastError();
}

int residual_workgroups_per_instance(int nrhs) { return (nrhs + 15) / 16; }

hipError_t launch_accumulate(const AccumulateLaunch& a, hipStream_t s) {
  if (a.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(accumulate_kernel, dim3((a.K * a.nrhs + 255) / 256, a.batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_widen(const float2* X, int64_t ldx, int64_t stride_x, int batch, int K, int n, double2* out,
                        hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3((K * n + 255) / 256, batch), dim3(256), 0, s, X, ldx, stride_x, K, n, out);
  return hipGetLastError();
}

}  // namespace jacpcg
