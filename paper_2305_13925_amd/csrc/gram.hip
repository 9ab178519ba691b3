// Regularised Gram matrix A = H^H H + xi I_K (eq. 7 of the paper: P_i) on the
// gfx950 matrix cores, FP32 accumulation.
//
// Work decomposition: one workgroup per (instance, 32x32 tile of the upper
// triangle of A). Its waves split the antenna range M into contiguous chunks;
// the partial tiles are summed in LDS in a fixed wave order (deterministic,
// no atomics) and written out together with the conjugate mirror tile, so A is
// exactly Hermitian with an exactly real diagonal.
//
// Complex arithmetic on the real MFMA (v_mfma_f32_32x32x2_f32): for antenna m
// the two k slots of one MFMA carry the real and imaginary parts,
//   A-operand  (row i, slot 0/1) = (Re h_im, Im h_im)
//   B-operand for Re A (slot 0/1) = (Re h_jm, Im h_jm)   -> Re h_i Re h_j + Im h_i Im h_j
//   B-operand for Im A (slot 0/1) = (Im h_jm, -Re h_jm)  -> Re h_i Im h_j - Im h_i Re h_j
// which is conj(h_im) h_jm split into real and imaginary parts.
#include "device_util.hpp"

namespace jacpcg {
namespace {

__device__ __forceinline__ void upper_tile(int t, int nt, int& ti, int& tj) {
  int i = 0;
  while (t >= nt - i) {
    t -= nt - i;
    ++i;
  }
  ti = i;
  tj = i + t;
}

// Load 8 consecutive complex entries row[m .. m+7], zero past `mend` or when the
// row is padding. VEC: 16-byte aligned row and m multiple of 8.
template <bool VEC>
__device__ __forceinline__ void load8(const float2* __restrict__ row, int m, int mend, bool valid,
                                      float2 (&v)[8]) {
  if (VEC && valid && m + 8 <= mend) {
    const float4* p = reinterpret_cast<const float4*>(row + m);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = p[q];
      v[2 * q] = make_float2(t.x, t.y);
      v[2 * q + 1] = make_float2(t.z, t.w);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (valid && m + e < mend) ? row[m + e] : make_float2(0.f, 0.f);
  }
}

constexpr int kGramMaxWaves = 8;

template <bool VEC>
__global__ __launch_bounds__(512) void gram_f32_kernel(GramLaunch g) {
  const int nt = (g.K + 31) >> 5;
  const int ntiles = nt * (nt + 1) / 2;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / ntiles;
  int ti, tj;
  upper_tile(L - b * ntiles, nt, ti, tj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int half = lane >> 5, li = lane & 31;
  const float2* Hb = g.H + (int64_t)b * g.stride_h;
  const int ui = ti * 32 + li, uj = tj * 32 + li;
  const bool vi = ui < g.K, vj = uj < g.K;
  const float2* hi = Hb + (int64_t)(vi ? ui : 0) * g.ldh;
  const float2* hj = Hb + (int64_t)(vj ? uj : 0) * g.ldh;
  const bool same = (ti == tj);

  const int chunk = ((g.M + nw * 8 - 1) / (nw * 8)) * 8;
  const int m0 = wave * chunk;
  const int m1 = min(g.M, m0 + chunk);

  floatx16 accR = zero16(), accI = zero16();
  for (int m = m0; m < m1; m += 8) {
    float2 a[8], c[8];
    load8<VEC>(hi, m, m1, vi, a);
    if (same) {
#pragma unroll
      for (int e = 0; e < 8; ++e) c[e] = a[e];
    } else {
      load8<VEC>(hj, m, m1, vj, c);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float av = half ? a[e].y : a[e].x;
      const float br = half ? c[e].y : c[e].x;
      const float bi = half ? -c[e].x : c[e].y;
      accR = mfma32(av, br, accR);
      accI = mfma32(av, bi, accI);
    }
  }

  // Fixed-order cross-wave sum through LDS.
  // red[w][0|1][r][lane]: nw * 2 * 16 * 64 floats of dynamic LDS.
  extern __shared__ float red_dyn[];
  float(*red)[2][16][64] = reinterpret_cast<float(*)[2][16][64]>(red_dyn);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    red[wave][0][r][lane] = accR[r];
    red[wave][1][r][lane] = accI[r];
  }
  __syncthreads();

  // Tile element (i, j) sits in lane j + 32*((i>>2)&1), register 4*(i>>3) + (i&3).
  auto tile = [&](int i, int j, float& re, float& im) {
    const int l = j + 32 * ((i >> 2) & 1), r = 4 * (i >> 3) + (i & 3);
    re = 0.f;
    im = 0.f;
    for (int w = 0; w < nw; ++w) {
      re += red[w][0][r][l];
      im += red[w][1][r][l];
    }
  };

  float2* Ab = g.A + (int64_t)b * g.stride_a;
  for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
    const int i = e >> 5, j = e & 31;
    const int gi = ti * 32 + i, gj = tj * 32 + j;
    if (gi < g.K && gj < g.K) {
      float re, im;
      if (!same || i < j) {
        tile(i, j, re, im);
      } else if (i > j) {
        tile(j, i, re, im);  // Hermitian mirror inside a diagonal tile
        im = -im;
      } else {
        tile(i, i, re, im);
        if (g.gdiag) g.gdiag[(int64_t)b * g.K + gi] = re;
        re += g.xi;
        im = 0.f;
        if (g.diag) g.diag[(int64_t)b * g.K + gi] = re;
      }
      Ab[(int64_t)gi * g.lda + gj] = make_float2(re, im);
    }
    if (!same) {
      // Mirror tile (tj, ti): row tj*32 + i, column ti*32 + j holds conj(T[j][i]).
      const int mi = tj * 32 + i, mj = ti * 32 + j;
      if (mi < g.K && mj < g.K) {
        float re, im;
        tile(j, i, re, im);
        Ab[(int64_t)mi * g.lda + mj] = make_float2(re, -im);
      }
    }
  }
}

}  // namespace

hipError_t launch_gram(const GramLaunch& g, hipStream_t s) {
  if (g.batch == 0) return hipSuccess;
  if (g.precision != 0) return hipErrorNotSupported;
  const int nt = (g.K + 31) / 32;
  const int ntiles = nt * (nt + 1) / 2;
  int waves = g.m_split > 0 ? g.m_split : 4;
  if (waves > kGramMaxWaves) waves = kGramMaxWaves;
  const dim3 grid((unsigned)(ntiles * g.batch)), block(64 * waves);
  const bool vec = ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);
  const size_t lds = (size_t)waves * 2 * 16 * 64 * sizeof(float);
  if (vec)
    hipLaunchKernelGGL(gram_f32_kernel<true>, grid, block, lds, s, g);
  else
    hipLaunchKernelGGL(gram_f32_kernel<false>, grid, block, lds, s, g);
  return hipGetLastError();
}

}  // namespace jacpcg
