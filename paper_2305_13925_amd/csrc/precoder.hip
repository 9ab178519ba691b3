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
#include <algorithm>

#include "device_util.hpp"

namespace jacpcg {
namespace {

// beta_pow = sqrt(P / ||H X||_F^2) from the per-workgroup partial sums of the
// solve (fixed order); 0 when H X = 0.
// Per-instance solver status from its ncb per-workgroup statuses, by
// severity: BREAKDOWN over NOT_CONVERGED over OK.
__device__ __forceinline__ int instance_status(const PrecoderLaunch& e, int b) {
  int s = kStatusOk;
  for (int c = 0; c < e.ncb; ++c) {
    const int v = e.wg_status[(int64_t)b * e.ncb + c];
    if (v == kStatusBreakdown) s = kStatusBreakdown;
    else if (v == kStatusNotConverged && s == kStatusOk) s = kStatusNotConverged;
  }
  if (e.ref_scale && s == kStatusOk) {
    for (int j = 0; j < e.nrhs; ++j)
      if (!(e.ref_scale[(int64_t)b * e.nrhs + j] <= e.ref_tol)) s = kStatusNotConverged;
  }
  return s;
}

__device__ __forceinline__ float power_factor(const PrecoderLaunch& e, int b) {
  if (e.fpart64) {
    double fs = 0.0;
    for (int c = 0; c < e.ncb64; ++c) fs += e.fpart64[(int64_t)b * e.ncb64 + c];
    return fs > 0.0 ? (float)sqrt((double)e.power / fs) : 0.f;
  }
  float fs = 0.f;
  for (int c = 0; c < e.ncb; ++c) fs += e.fpart[(int64_t)b * e.ncb + c];
  return fs > 0.f ? sqrtf(e.power / fs) : 0.f;
}

template <int KT, int NJ, bool VEC>
__global__ __launch_bounds__(256) void precoder_f32_kernel(PrecoderLaunch e) {
  constexpr int KP = KT * 32;
  constexpr int KH = KT * 16;
  constexpr int NC = 32 * NJ;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int jl = lane & 31, half = lane >> 5;
  const int nmb = (e.M + 127) / 128;
  const int ncw = (e.nrhs + NC - 1) / NC;
  const int per = nmb * ncw;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  // Instances are taken last first: the Gram launch just before this one read
  // the channels in increasing order, so the last ones it read are the likeliest
  // still to sit in the Infinity Cache (256 MB, shared by all XCDs).
  const int bq = L / per;
  const int b = e.batch - 1 - bq;
  const int rem = L - bq * per;
  const int mb = rem / ncw, cw = rem - mb * ncw;
  const int K = e.K;

  __shared__ float2 Xs[KP][NC];

  const float beta = power_factor(e, b);
  if (mb == 0 && cw == 0 && threadIdx.x == 0) {
    if (e.beta_out) e.beta_out[b] = beta;
    if (e.status) e.status[b] = instance_status(e, b);
  }

  gptr<const float2> Xb = as_global(e.X + (int64_t)b * e.stride_x);
  for (int idx = threadIdx.x; idx < KP * NC; idx += 256) {
    const int jj = idx % NC, k = idx / NC;
    const int j = cw * NC + jj;
    float2 v = make_float2(0.f, 0.f);
    if (k < K && j < e.nrhs) {
      v = ld2(Xb + (int64_t)j * e.ldx + k);
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
  gptr<const float2> hcol = as_global(e.H_ptrs ? e.H_ptrs[b] : e.H + (int64_t)b * e.stride_h) + (int64_t)(half * KH) * e.ldh +
                           (mvalid ? mrow : 0);

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
      h[q] = (mvalid && s < klim) ? ld2(hcol + (int64_t)s * e.ldh) : make_float2(0.f, 0.f);
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

  gptr<float2> Wb = as_global(e.W_ptrs ? e.W_ptrs[b] : e.W + (int64_t)b * e.stride_w);
#pragma unroll
  for (int t = 0; t < NJ; ++t) {
    const int j = cw * NC + t * 32 + jl;
    if (j >= e.nrhs) continue;
    gptr<float2> wc = Wb + (int64_t)j * e.ldw;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int m = m0 + 8 * g + 4 * half;
      if (VEC && m + 4 <= e.M) {
        gptr<float4> dst = reinterpret_cast<gptr<float4>>(wc + m);
        st4_nt(dst, wr[t][4 * g + 0], wi[t][4 * g + 0], wr[t][4 * g + 1], wi[t][4 * g + 1]);
        st4_nt(dst + 1, wr[t][4 * g + 2], wi[t][4 * g + 2], wr[t][4 * g + 3], wi[t][4 * g + 3]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (m + q < e.M) st2_nt(wc + m + q, wr[t][4 * g + q], wi[t][4 * g + q]);
      }
    }
  }
}

template <int KT>
hipError_t launch_kt(const PrecoderLaunch& e, hipStream_t s) {
  const int nmb = (e.M + 127) / 128;
  const bool vec = !e.no_vec && ((uintptr_t)e.W % 16 == 0) && (e.ldw % 2 == 0) && (e.stride_w % 2 == 0);
  // Two column tiles per wave halve the reads of H; LDS caps it at K <= 128.
  if constexpr (KT <= 4) {
    if (e.nrhs > 32 && e.nj != 1) {
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


// Split-BF16 precoder (FP32-class accuracy with NS = 3). It computes the
// transpose W^T = X^T H^T so that the MFMA result puts consecutive antennas in
// consecutive lanes and every W store is a coalesced 256-byte row segment.
// Real-plane formulation on v_mfma_f32_32x32x16_bf16: the 16 k slots are 16
// users of one component (lane half c holds users k0+8c .. k0+8c+7):
//   Re W[m,j] = sum_k Re X[k,j] Re H[m,k] + Im X[k,j] (-Im H[m,k])
//   Im W[m,j] = sum_k Re X[k,j] Im H[m,k] + Im X[k,j]   Re H[m,k]
// beta_pow X is split into bf16 parts once per workgroup (Re and Im planes in
// LDS); H is split on the fly and its negated Im plane is shared by all column
// tiles, so no other operand shuffling is needed.
// Active user steps per chunk of the sparse epilogue's LDS split of beta_pow X
// (its LDS is sized for this many steps, not for all of K).
constexpr int kVrSteps = 4;

// Index of the n-th set bit of a step mask (the last set bit when n is past
// the end, 0 for an empty mask); wave-uniform arguments, scalar work.
__device__ __forceinline__ int nth_active(unsigned act, int n) {
  int last = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if ((act >> s) & 1u) {
      if (n == 0) return s;
      --n;
      last = s;
    }
  }
  return last;
}

// With one column tile per wave at 64 < K <= 128 the kernel is held to 168
// registers, three waves per SIMD (170 unconstrained, which allowed two): more
// waves in flight overlap the channel reads with the products (K = 128,
// 256 x (M=4096): 0.73 -> 0.66 ms).
// VR: visibility-region sparse variant (one antenna block per workgroup):
// only the user steps whose 32-user block has a span reaching this block's
// antennas are computed (the others hold zero channel entries here).
// NW waves per workgroup, one 32-antenna tile each: blocks of 32 NW antennas.
template <int NS, int KT, int NJ, bool FULL, bool VR, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu((KT == 3 || KT == 4) && NJ == 1 ? 3 : 1))) void precoder_bf16_kernel(PrecoderLaunch e) {
  constexpr int BLK = 32 * NW;
  constexpr int KP = KT * 32;
  constexpr int K8 = KP / 8;  // groups of 8 users (one lane half of one step)
  constexpr int NC = 32 * NJ;
  // LDS rows of the split of beta_pow X: every group of 8 users, or for the
  // sparse variant the active steps of one chunk (kVrSteps steps, 2 rows each).
  constexpr int K8X = VR ? 2 * kVrSteps : K8;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int jl = lane & 31, half = lane >> 5;
  // A workgroup covers `mt` consecutive blocks of BLK antennas (one 32-antenna
  // tile per wave and block), so its split of beta_pow X is reused mt times.
  const int mt = e.mtiles;
  const int nblk = (e.M + BLK - 1) / BLK;
  const int nmb = (nblk + mt - 1) / mt;
  const int ncw = (e.nrhs + NC - 1) / NC;
  const int per = nmb * ncw;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  // Instances are taken last first: the Gram launch just before this one read
  // the channels in increasing order, so the last ones it read are the likeliest
  // still to sit in the Infinity Cache (256 MB, shared by all XCDs).
  const int bq = L / per;
  const int b = e.batch - 1 - bq;
  const int rem = L - bq * per;
  const int mb = rem / ncw, cw = rem - mb * ncw;
  const int blk0 = mb * mt, blk1 = min(nblk, blk0 + mt);
  const int K = e.K;

  extern __shared__ u32x4 xs_dyn[];  // [2 planes][NS][K8X][NC]
  auto XS = [&](int plane, int s, int k8, int j) -> u32x4& {
    return xs_dyn[(((size_t)plane * NS + s) * K8X + k8) * NC + j];
  };

  gptr<const float2> Hb = as_global(e.H_ptrs ? e.H_ptrs[b] : e.H + (int64_t)b * e.stride_h);
  // Channel values of global step gs (step gs % S of block blk0 + gs / S): the
  // lane's antenna row, users 8 * (2 * step + half) .. +7. Steps past the last
  // block reload the last one, so every load can be issued unconditionally.
  constexpr int S = K8 / 2;
  static_assert(S <= 16, "step masks hold 16 steps");
  unsigned act = (S >= 32) ? ~0u : ((1u << S) - 1u);
  int nact = S;
  if constexpr (VR) {
    const int m_lo = blk0 * BLK, m_hi = min(e.M, m_lo + BLK);
    act = 0;
    for (int c = 0; c < KT; ++c) {
      const int2 sp = e.tile_span[(int64_t)b * KT + c];
      if (sp.y > m_lo && sp.x < m_hi) act |= 3u << (2 * c);  // steps 2c, 2c+1: users 32c .. 32c+31
    }
    act = __builtin_amdgcn_readfirstlane(act);
    nact = __popc(act);
  }
  auto issue = [&](int gs, float (&hr)[8], float (&hi)[8]) {
    int blk, st;
    if constexpr (VR) {
      blk = blk0;
      st = nth_active(act, gs);
    } else {
      blk = blk0 + gs / S;
      st = gs % S;
      if (blk >= blk1) {
        blk = blk1 - 1;
        st = S - 1;
      }
    }
    const int mrow = blk * BLK + w * 32 + jl;
    const bool v = FULL || mrow < e.M;
    gptr<const float2> hc = Hb + (v ? mrow : 0);
    const int k8 = 2 * st + half;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = 8 * k8 + u;
      const float2 h = (FULL || (v && k < K)) ? ld2(hc + (int64_t)k * e.ldh) : make_float2(0.f, 0.f);
      hr[u] = h.x;
      hi[u] = h.y;
    }
  };
  // Two steps in flight per wave, issued before the X preamble so that their
  // latency overlaps it.
  float hrA[8], hiA[8], hrB[8], hiB[8];
  issue(0, hrA, hiA);
  issue(1, hrB, hiB);

  const float beta = power_factor(e, b);
  if (mb == 0 && cw == 0 && threadIdx.x == 0) {
    if (e.beta_out) e.beta_out[b] = beta;
    if (e.status) e.status[b] = instance_status(e, b);
  }

  gptr<const float2> Xb = as_global(e.X + (int64_t)b * e.stride_x);
  // beta_pow X, users 8 k8 .. 8 k8 + 7 of column tile entry jj, split into
  // LDS row r.
  auto split_x = [&](int k8, int r, int jj) {
    const int j = cw * NC + jj;
    float re[8], im[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = 8 * k8 + u;
      float2 x = make_float2(0.f, 0.f);
      if (FULL || (k < K && j < e.nrhs)) x = ld2(Xb + (int64_t)j * e.ldx + k);
      re[u] = beta * x.x;
      im[u] = beta * x.y;
    }
    u32x4 pr[NS], pi[NS];
    split8<NS>(re, pr);
    split8<NS>(im, pi);
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      XS(0, q, r, jj) = pr[q];
      XS(1, q, r, jj) = pi[q];
    }
  };
  if constexpr (!VR) {
    for (int idx = threadIdx.x; idx < K8 * NC; idx += 64 * NW) split_x(idx / NC, idx / NC, idx % NC);
    __syncthreads();
  }

  gptr<float2> Wbase = as_global(e.W_ptrs ? e.W_ptrs[b] : e.W + (int64_t)b * e.stride_w);
  floatx16 wr[NJ], wi[NJ];
  // One step: split the staged users, refill the stage with the step two
  // ahead, then the products of this step's 8 users (per lane half) with the
  // split of beta_pow X in LDS row k8.
  auto compute = [&](float (&hr)[8], float (&hi)[8], int k8, int gs_next) {
    u32x4 Hr[NS], Hi[NS], Hn[NS];
    split8<NS>(hr, Hr);
    split8<NS>(hi, Hi);
    issue(gs_next, hr, hi);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) Hn[q][c] = neg_bf16x2(Hi[q][c]);
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      u32x4 Xr[NS], Xi[NS];
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        Xr[q] = XS(0, q, k8, t * 32 + jl);
        Xi[q] = XS(1, q, k8, t * 32 + jl);
      }
      split_mma<NS>(Xr, Hr, wr[t]);
      split_mma<NS>(Xi, Hn, wr[t]);
      split_mma<NS>(Xr, Hi, wi[t]);
      split_mma<NS>(Xi, Hr, wi[t]);
    }
  };
  int gs = 0;
#pragma unroll 1
  for (int blk = blk0; blk < blk1; ++blk) {
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      wr[t] = zero16();
      wi[t] = zero16();
    }
    if constexpr (VR) {
      // Active steps in chunks of kVrSteps: the chunk's split of beta_pow X
      // goes to LDS, then its products.
#pragma unroll 1
      for (int c0 = 0; c0 < nact; c0 += kVrSteps) {
        const int c1 = min(nact, c0 + kVrSteps);
        if (c0 > 0) __syncthreads();  // the previous chunk's products have read the split
        for (int idx = threadIdx.x; idx < 2 * (c1 - c0) * NC; idx += 64 * NW) {
          const int r = idx / NC;
          split_x(2 * nth_active(act, c0 + (r >> 1)) + (r & 1), r, idx % NC);
        }
        __syncthreads();
#pragma unroll 1
        for (int i = c0; i < c1; i += 2) {
          compute(hrA, hiA, 2 * (i - c0) + half, i + 2);
          if (i + 1 < c1) compute(hrB, hiB, 2 * (i + 1 - c0) + half, i + 3);
        }
      }
    } else if constexpr (KT > 4) {
      // Fully unrolled over the block's steps: as a loop, the compiler copied
      // the staged channel values into the loop-carried registers at the back
      // edge and waited there for every load in flight, including the ones
      // just issued for the steps ahead. (At K <= 128 the rolled loop fits
      // three waves per SIMD, which gains more.)
#pragma unroll
      for (int st = 0; st < S; st += 2, gs += 2) {
        compute(hrA, hiA, 2 * st + half, gs + 2);
        compute(hrB, hiB, 2 * st + 2 + half, gs + 3);
      }
    } else {
#pragma unroll 1
      for (int st = 0; st < S; st += 2, gs += 2) {
        compute(hrA, hiA, 2 * st + half, gs + 2);
        compute(hrB, hiB, 2 * st + 2 + half, gs + 3);
      }
    }
    const int m = blk * BLK + w * 32 + jl;
    if (FULL || m < e.M) {
      gptr<float2> Wb = Wbase + m;
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = cw * NC + t * 32 + d32_row(r, half);
          if (FULL || j < e.nrhs) st2_nt(Wb + (int64_t)j * e.ldw, wr[t][r], wi[t][r]);
        }
      }
    }
  }
}

template <int NS, int KT, int NJ>
hipError_t launch_bf16_nj(const PrecoderLaunch& e, hipStream_t s) {
  // Beyond K = 128 the split of beta_pow X (2 NS K/8 32 NJ 16-byte entries)
  // leaves room for one workgroup per compute unit, so the workgroup has 8
  // waves (two per SIMD) sharing it, over blocks of 256 antennas.
  constexpr int NW = KT > 4 ? 8 : 4;
  // The sparse variant sizes its LDS for kVrSteps active steps, which leaves
  // room for more than one workgroup per compute unit at any K: 4 waves.
  constexpr int NWV = 4;
  const bool vr = e.tile_span != nullptr && KT > 2;
  const int BLK = 32 * (vr ? NWV : NW);
  const int nblk = (e.M + BLK - 1) / BLK;
  PrecoderLaunch p = e;
  // Blocks of BLK antennas per workgroup: enough to amortise the split of X,
  // few enough to keep several workgroups per compute unit busy. The sparse
  // variant takes one block per workgroup (its user steps depend on it).
  if (vr)
    p.mtiles = 1;
  else if (p.mtiles <= 0)
    p.mtiles = nblk >= 8 ? 2 : 1;
  p.mtiles = std::min(p.mtiles, nblk);
  const int nmb = (nblk + p.mtiles - 1) / p.mtiles;
  const size_t lds = (size_t)2 * NS * (vr ? 2 * kVrSteps : KT * 4) * 32 * NJ * 16;
  // FULL: every user, antenna and column of every tile is in range (no masks).
  const bool full = (e.K == KT * 32) && (e.M % BLK == 0) && (e.nrhs % (32 * NJ) == 0);
  const int grid = e.batch * nmb * ((e.nrhs + 32 * NJ - 1) / (32 * NJ));
  auto k = full ? (vr ? precoder_bf16_kernel<NS, KT, NJ, true, true, NWV> : precoder_bf16_kernel<NS, KT, NJ, true, false, NW>)
                : (vr ? precoder_bf16_kernel<NS, KT, NJ, false, true, NWV> : precoder_bf16_kernel<NS, KT, NJ, false, false, NW>);
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * (vr ? NWV : NW)), lds, s, p);
  return hipGetLastError();
}

template <int NS, int KT>
hipError_t launch_bf16_kt(const PrecoderLaunch& e, hipStream_t s) {
  // Two column tiles per wave share each split of H (default up to K = 64;
  // the tuner may choose either for K <= 128).
  if constexpr (KT <= 4) {
    const bool two = e.nj == 2 || (e.nj == 0 && KT <= 2);
    if (e.nrhs > 32 && two) return launch_bf16_nj<NS, KT, 2>(e, s);
  }
  return launch_bf16_nj<NS, KT, 1>(e, s);
}
}  // namespace

hipError_t launch_precoder(const PrecoderLaunch& e, hipStream_t s) {
  if (e.batch == 0) return hipSuccess;
  if (e.split == 3) {
    switch ((e.K + 31) / 32) {
      case 1: return launch_bf16_kt<3, 1>(e, s);
      case 2: return launch_bf16_kt<3, 2>(e, s);
      case 3: return launch_bf16_kt<3, 3>(e, s);
      case 4: return launch_bf16_kt<3, 4>(e, s);
      case 5: return launch_bf16_kt<3, 5>(e, s);
      case 6: return launch_bf16_kt<3, 6>(e, s);
      case 7: return launch_bf16_kt<3, 7>(e, s);
      case 8: return launch_bf16_kt<3, 8>(e, s);
      default: return hipErrorInvalidValue;
    }
  }
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
