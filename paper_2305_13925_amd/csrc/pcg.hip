// Jacobi-preconditioned conjugate gradient (Sec. III-B, eq. 21, Algorithm 1 with
// the standard PCG step length of Step 3) for a batch of K x K Hermitian
// positive definite systems A X = B with many right-hand sides, as one
// persistent launch: every iteration runs inside the kernel.
//
// Decomposition: the columns of B are independent PCG solves that share A, so a
// workgroup owns (instance b, block of 32 right-hand sides) and all of its
// iterations. KT = ceil(K/32) waves; wave w owns rows [32w, 32w+32) of the
// solution, residual and direction for the block's 32 columns, held in
// registers in the 32x32 MFMA result layout. The direction block P (K x 32)
// lives in LDS and is the B-operand of the per-iteration product Q = A P.
//
// Q = A P on v_mfma_f32_32x32x2_f32: the two k slots of one MFMA carry the
// complex terms k = s (slot 0) and k = s + K/2 (slot 1), so each lane walks one
// contiguous half-row of A. Per step four real MFMAs form
//   Re Q += Re A Re P - Im A Im P,   Im Q += Re A Im P + Im A Re P.
// For K <= 64 each wave keeps its 32 rows of A in registers for the whole
// solve; larger K streams the rows from L2 every iteration.
//
// Per iteration and column j (reductions are shuffles + LDS, fixed order):
//   gamma_j = Re p_j^H q_j;  alpha_j = rho_j / gamma_j
//   x_j += alpha_j p_j;  r_j -= alpha_j q_j
//   stop when ||r_j|| <= tol ||b_j||  (tol = 0: fixed iteration count)
//   z_j = D^{-1} r_j;  rho'_j = Re r_j^H z_j;  p_j = z_j + (rho'_j / rho_j) p_j
// gamma_j < 0 or non-finite flags a breakdown and freezes the column;
// gamma_j = 0 (p_j = 0 for HPD A: the residual underflowed) ends it as converged.
//
// Optional final pass for the precoder's power normalisation: with G = H^H H
// (A with its diagonal replaced by diag(H^H H), passed in `gdiag`), every
// workgroup writes sum over its columns of x_j^H G x_j = ||H X||_F^2 part,
// computed without subtracting xi from A (no cancellation when xi >> ||h||^2).
#include "device_util.hpp"

namespace jacpcg {
namespace {

// Sum of one float per column over the two lane halves and all waves; every
// lane receives the total of its column. One barrier.
template <int KT, int NS>
__device__ __forceinline__ void col_reduce(float (&v)[NS], float (*red)[KT][32], int w, int jl, int half) {
#pragma unroll
  for (int q = 0; q < NS; ++q) v[q] += __shfl_xor(v[q], 32);
  if (half == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) red[q][w][jl] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    float t = 0.f;
#pragma unroll
    for (int ww = 0; ww < KT; ++ww) t += red[q][ww][jl];
    v[q] = t;
  }
}

// Q = A' P, A' the wave's 32 rows of A (with the diagonal entry zeroed when
// `zero_diag`), P from LDS.
template <int KT, bool AREG>
__device__ __forceinline__ void apply_a(floatx16& qr, floatx16& qi, const float* ar, const float* ai,
                                        const float2* __restrict__ arow, int klim, bool zero_diag, int diag_s,
                                        const float2 (*Psh)[32], int half, int jl) {
  constexpr int KH = KT * 16;
  qr = zero16();
  qi = zero16();
  if constexpr (AREG) {
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      const float2 pv = Psh[half * KH + s][jl];
      const float a_r = (zero_diag && s == diag_s) ? 0.f : ar[s];
      const float a_i = (zero_diag && s == diag_s) ? 0.f : ai[s];
      qr = mfma32(a_r, pv.x, qr);
      qr = mfma32(a_i, -pv.y, qr);
      qi = mfma32(a_r, pv.y, qi);
      qi = mfma32(a_i, pv.x, qi);
    }
  } else {
    for (int s0 = 0; s0 < KH; s0 += 8) {
      float2 av[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int s = s0 + e;
        av[e] = (s < klim && !(zero_diag && s == diag_s)) ? arow[s] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 pv = Psh[half * KH + s0 + e][jl];
        qr = mfma32(av[e].x, pv.x, qr);
        qr = mfma32(av[e].y, -pv.y, qr);
        qi = mfma32(av[e].x, pv.y, qi);
        qi = mfma32(av[e].y, pv.x, qi);
      }
    }
  }
}

// Visibility-region sparse variant (K > 64, A streamed from L2): the two k
// slots of one MFMA carry the adjacent columns k = 2s and 2s + 1, so the 16
// steps of a 32-column block of A stay inside that block, and blocks that are
// structurally zero for this wave's rows (bit c of `mask` clear: the users'
// visibility regions do not overlap, so A is exactly zero there) are skipped.
template <int KT>
__device__ __forceinline__ void apply_a_vr(floatx16& qr, floatx16& qi, const float2* __restrict__ arow, bool rowvalid,
                                           int K, int ia, bool zero_diag, unsigned mask, const float2 (*Psh)[32],
                                           int half, int jl) {
  qr = zero16();
  qi = zero16();
  for (int c = 0; c < KT; ++c) {
    if (!((mask >> c) & 1u)) continue;  // wave-uniform
    for (int s0 = 16 * c; s0 < 16 * c + 16; s0 += 8) {
      float2 av[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 2 * (s0 + e) + half;
        av[e] = (rowvalid && k < K && !(zero_diag && k == ia)) ? arow[k] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 pv = Psh[2 * (s0 + e) + half][jl];
        qr = mfma32(av[e].x, pv.x, qr);
        qr = mfma32(av[e].y, -pv.y, qr);
        qi = mfma32(av[e].x, pv.y, qi);
        qi = mfma32(av[e].y, pv.x, qi);
      }
    }
  }
}

// Split-BF16 variant of the product (K > 64, dense, A streamed from L2): the
// direction block lives in LDS as three-part bf16 planes PB[comp][part][k8][j]
// (entry: the 8 bf16 of rows 8 k8 .. 8 k8 + 7 of column j, the B operand of
// v_mfma_f32_32x32x16_bf16), and each lane splits the 8 entries of its row of A
// that one 16-row step needs (k = 16 s + 8 half ..), so
//   Re Q += Re A Re P + (-Im A) Im P,   Im Q += Re A Im P + Im A Re P
// take four split products of six bf16 MFMAs each (FP32-class: the dropped
// part products are at most ~2^-24 of the terms).
template <int NS>
__device__ __forceinline__ void split4(const float (&x)[4], uint32_t (&parts)[NS][2]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float a = x[2 * q], b = x[2 * q + 1];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const uint32_t pk = pack_bf16x2(a, b);
      parts[t][q] = pk;
      if (t + 1 < NS) {
        a -= bf16_lo(pk);
        b -= bf16_hi(pk);
      }
    }
  }
}

// Store this wave's rows of a block (result layout) as the bf16 planes.
template <int KT>
__device__ __forceinline__ void store_planes(const float (&vr)[16], const float (&vi)[16], u32x4* PB, int w,
                                             int half, int jl) {
  constexpr int K8 = KT * 4;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float xr4[4] = {vr[4 * g], vr[4 * g + 1], vr[4 * g + 2], vr[4 * g + 3]};
    const float xi4[4] = {vi[4 * g], vi[4 * g + 1], vi[4 * g + 2], vi[4 * g + 3]};
    uint32_t pr[3][2], pi[3][2];
    split4<3>(xr4, pr);
    split4<3>(xi4, pi);
    const int k8 = 4 * w + g;  // rows 8 k8 + 4 half .. + 3 of the plane entry
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      uint2* er = reinterpret_cast<uint2*>(&PB[((0 * 3 + t) * K8 + k8) * 32 + jl]);
      uint2* ei = reinterpret_cast<uint2*>(&PB[((1 * 3 + t) * K8 + k8) * 32 + jl]);
      er[half] = make_uint2(pr[t][0], pr[t][1]);
      ei[half] = make_uint2(pi[t][0], pi[t][1]);
    }
  }
}

template <int KT>
__device__ __forceinline__ void apply_a_spl(floatx16& qr, floatx16& qi, const float2* __restrict__ arow, bool rowvalid,
                                            int K, int ia, bool zero_diag, const u32x4* PB, int half, int jl) {
  constexpr int K8 = KT * 4;
  constexpr int NSTEP = KT * 2;  // 16 rows of P per step
  qr = zero16();
  qi = zero16();
  float2 av[2][8];
  auto load = [&](int st, float2 (&v)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * st + 8 * half + e;
      v[e] = (rowvalid && k < K && !(zero_diag && k == ia)) ? arow[k] : make_float2(0.f, 0.f);
    }
  };
  load(0, av[0]);
#pragma unroll
  for (int st = 0; st < NSTEP; ++st) {
    float2(&cur)[8] = av[st & 1];
    if (st + 1 < NSTEP) load(st + 1, av[(st + 1) & 1]);
    // Re A's products first, then Im A's, so that few operands are live at
    // once (the solver state takes most of the registers).
    u32x4 Pr[3], Pi[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      Pr[t] = PB[((0 * 3 + t) * K8 + 2 * st + half) * 32 + jl];
      Pi[t] = PB[((1 * 3 + t) * K8 + 2 * st + half) * 32 + jl];
    }
    {
      float re[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) re[e] = cur[e].x;
      u32x4 Ar[3];
      split8<3>(re, Ar);
      split_mma<3>(Ar, Pr, qr);
      split_mma<3>(Ar, Pi, qi);
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      float im[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) im[e] = cur[e].y;
      u32x4 Ai[3];
      split8<3>(im, Ai);
      split_mma<3>(Ai, Pr, qi);
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) Ai[t][c] = neg_bf16x2(Ai[t][c]);
      split_mma<3>(Ai, Pi, qr);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Sparse form of the split-BF16 product: only the 32-column blocks of A that
// can hold nonzeros in this wave's rows (bit c of `mask`) are taken, two
// 16-row steps each, with both steps' entries loaded before the products.
template <int KT>
__device__ __forceinline__ void apply_a_spl_vr(floatx16& qr, floatx16& qi, const float2* __restrict__ arow,
                                               bool rowvalid, int K, int ia, bool zero_diag, unsigned mask,
                                               const u32x4* PB, int half, int jl) {
  constexpr int K8 = KT * 4;
  qr = zero16();
  qi = zero16();
  for (int c = 0; c < KT; ++c) {
    if (!((mask >> c) & 1u)) continue;  // wave-uniform
    float2 av[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * c + 16 * h + 8 * half + e;
        av[h][e] = (rowvalid && k < K && !(zero_diag && k == ia)) ? arow[k] : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int st = 2 * c + h;
      u32x4 Pr[3], Pi[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        Pr[t] = PB[((0 * 3 + t) * K8 + 2 * st + half) * 32 + jl];
        Pi[t] = PB[((1 * 3 + t) * K8 + 2 * st + half) * 32 + jl];
      }
      {
        float re[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) re[e] = av[h][e].x;
        u32x4 Ar[3];
        split8<3>(re, Ar);
        split_mma<3>(Ar, Pr, qr);
        split_mma<3>(Ar, Pi, qi);
      }
      {
        float im[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) im[e] = av[h][e].y;
        u32x4 Ai[3];
        split8<3>(im, Ai);
        split_mma<3>(Ai, Pr, qi);
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) Ai[t][q] = neg_bf16x2(Ai[t][q]);
        split_mma<3>(Ai, Pi, qr);
      }
    }
  }
}

// Two waves per SIMD (the register budget of 256 per lane) let one workgroup's
// reductions overlap another's products.
template <int KT, bool AREG, bool VRS, bool SPL = false>
__global__ __launch_bounds__(KT * 64) __attribute__((amdgpu_waves_per_eu(2))) void pcg_f32_kernel(PcgLaunch p) {
  static_assert(!(VRS && AREG), "the sparse variant streams A");
  static_assert(!SPL || !AREG, "the split-BF16 product is for streamed A");
  constexpr int KP = KT * 32;
  constexpr int KH = KT * 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jl = lane & 31, half = lane >> 5;
  const int ncb = (p.nrhs + 31) >> 5;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / ncb, cb = L - b * ncb;
  const int K = p.K;
  const int j = cb * 32 + jl;
  const bool jvalid = j < p.nrhs;

  // The direction block P, and before it (K <= 64) the staging tile of A.
  // The direction block P; before it (K <= 64) the staging tile of 32 rows of
  // A, after it the staging tile of X (32 columns of KP + 1 entries).
  constexpr int kLdsP = SPL ? 6 * (KP / 8) * 32 * 16 : KP * 32 * (int)sizeof(float2);
  constexpr int kLdsA = AREG ? 32 * KP * (int)sizeof(float2) : 0;
  constexpr int kLdsX = 32 * (KP + 1) * (int)sizeof(float2);
  constexpr int kLds = kLdsA > kLdsX ? kLdsA : (kLdsX > kLdsP ? kLdsX : kLdsP);
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kLds];
  float2(*Psh)[32] = reinterpret_cast<float2(*)[32]>(lds_raw);
  u32x4* PB = reinterpret_cast<u32x4*>(lds_raw);  // SPL: the bf16 planes of P
  __shared__ float red[3][KT][32];

  const bool chunked = p.st.vec != nullptr;
  // A workgroup that already finished in an earlier chunk has nothing to do.
  if (chunked && !p.first && p.st.done[L]) return;
  // Gated columns (refinement corrections): only columns whose residual
  // missed the tolerance are solved; a block with none leaves X untouched.
  // Every wave holds all 32 columns, so the test is workgroup-uniform.
  bool gate_on = true;
  if (p.col_gate) {
    gate_on = jvalid && !(p.col_gate[(int64_t)b * p.nrhs + j] <= p.gate_tol);
    if (!__any(gate_on)) return;
  }

  const float2* Ab = p.A + (int64_t)b * p.stride_a;
  // A-operand row of this lane and its contiguous half-row.
  const int ia = w * 32 + jl;
  const int klim = (ia < K) ? max(0, min(KH, K - half * KH)) : 0;
  const float2* arow = Ab + (int64_t)(ia < K ? ia : 0) * p.lda + half * KH;
  const int diag_s = ia - half * KH;  // step holding A[ia][ia] in this lane, if in [0, KH)
  // Sparse variant: the 32-column blocks of A that can hold nonzeros in this
  // wave's rows (spans overlap; the diagonal block always, for xi).
  unsigned vr_mask = 0;
  if constexpr (VRS) {
    const int2 sw = p.tile_span[(int64_t)b * KT + w];
    for (int c = 0; c < KT; ++c) {
      const int2 sc = p.tile_span[(int64_t)b * KT + c];
      if (c == w || min(sw.y, sc.y) > max(sw.x, sc.x)) vr_mask |= 1u << c;
    }
    vr_mask = __builtin_amdgcn_readfirstlane(vr_mask);
  }
  const float2* arow_full = Ab + (int64_t)(ia < K ? ia : 0) * p.lda;

  float ar[AREG ? KH : 1], ai[AREG ? KH : 1];
  float dinv[16];  // Jacobi preconditioner D^{-1} on the rows owned in the result layout
  if constexpr (AREG) {
    // K <= 64: the workgroup reads A once with coalesced loads (consecutive
    // threads take consecutive columns of a row), all loads in flight at once,
    // and passes it through LDS 32 rows at a time (the rows of one wave; the
    // tile is the memory of P): entry (i, k) of the pass at i * KP + (k ^ i),
    // so that the lanes of one read below (32 rows, one column) hit distinct
    // banks; zero outside K x K. Wave w takes its half-rows and the diagonal
    // entries of its rows from pass w.
    float2* At = reinterpret_cast<float2*>(lds_raw);
    constexpr int kPer = 32 * KP / (KT * 64);  // entries per thread and pass
    float2 av[KT][kPer];
#pragma unroll
    for (int q = 0; q < KT; ++q)
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * KT * 64;
        const int i = q * 32 + e / KP, k = e % KP;
        av[q][u] = (i < K && k < K) ? Ab[(int64_t)i * p.lda + k] : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      if (q > 0) __syncthreads();  // wave q - 1 has read the previous pass
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * KT * 64;
        const int i = e / KP, k = e % KP;
        At[i * KP + (k ^ i)] = av[q][u];
      }
      __syncthreads();
      if (w == q) {
#pragma unroll
        for (int s = 0; s < KH; ++s) {
          const float2 v = At[jl * KP + ((half * KH + s) ^ jl)];
          ar[s] = v.x;
          ai[s] = v.y;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int il = d32_row(r, half), i = w * 32 + il;
          const float d = p.precond_none ? 1.f : At[il * KP + (i ^ il)].x;  // entry (i, i)
          dinv[r] = (i < K) ? 1.f / d : 0.f;
        }
      }
    }
    __syncthreads();  // the tile is read; its memory becomes P
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = w * 32 + d32_row(r, half);
      float d = 0.f;
      if (i < K) d = p.precond_none ? 1.f : Ab[(int64_t)i * p.lda + i].x;
      dinv[r] = (i < K) ? 1.f / d : 0.f;
    }
  }

  float xr[16], xim[16], rr[16], ri[16], pr[16], pim[16];
  float rho = 0.f, bb = 0.f, rres = 0.f;
  int it = 0, t0 = 0;
  bool active = false, conv = false, brk = false;

  constexpr int kVecPerArray = KT * 16 * 64;
  float* stv = chunked ? p.st.vec + (int64_t)L * 6 * kVecPerArray : nullptr;
  float* stc = chunked ? p.st.col + (int64_t)L * 8 * 32 : nullptr;

  if (!chunked || p.first) {
    const float2* Bb = p.B ? p.B + (int64_t)b * p.stride_b : nullptr;
    float part[2] = {0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = w * 32 + d32_row(r, half);
      float2 bv = make_float2(0.f, 0.f);
      if (i < K && jvalid) {
        if (Bb)
          bv = Bb[(int64_t)j * p.ldb + i];
        else
          bv = make_float2(i == j ? 1.f : 0.f, 0.f);
      }
      xr[r] = 0.f;
      xim[r] = 0.f;
      rr[r] = bv.x;
      ri[r] = bv.y;
      pr[r] = dinv[r] * bv.x;
      pim[r] = dinv[r] * bv.y;
      const float n2 = bv.x * bv.x + bv.y * bv.y;
      part[0] += n2;
      part[1] += dinv[r] * n2;
    }
    col_reduce<KT, 2>(part, red, w, jl, half);
    bb = part[0];
    rho = part[1];
    rres = bb;
    active = jvalid && bb > 0.f && gate_on;
    conv = true;  // reset below for columns that must iterate
    if (active) conv = false;
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = w * 16 * 64 + r * 64 + lane;
      xr[r] = stv[0 * kVecPerArray + o];
      xim[r] = stv[1 * kVecPerArray + o];
      rr[r] = stv[2 * kVecPerArray + o];
      ri[r] = stv[3 * kVecPerArray + o];
      pr[r] = stv[4 * kVecPerArray + o];
      pim[r] = stv[5 * kVecPerArray + o];
    }
    rho = stc[0 * 32 + jl];
    bb = stc[1 * 32 + jl];
    rres = stc[2 * 32 + jl];
    it = (int)stc[3 * 32 + jl];
    active = stc[4 * 32 + jl] != 0.f;
    conv = stc[5 * 32 + jl] != 0.f;
    brk = stc[6 * 32 + jl] != 0.f;
    t0 = (int)stc[7 * 32 + 0];
  }

  if constexpr (SPL) {
    store_planes<KT>(pr, pim, PB, w, half, jl);
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) Psh[w * 32 + d32_row(r, half)][jl] = make_float2(pr[r], pim[r]);
  }

  // FP32 range guard: below ||r|| = 2^-40 ||b|| an FP32 iterate no longer
  // changes (the update is far under its rounding) while p^H A p heads for
  // underflow, so such a column ends as converged even with tol = 0.
  const float tol2 = fmaxf(p.tol * p.tol, 0x1p-80f);
  const int tend = chunked ? min(p.max_iter, t0 + p.chunk) : p.max_iter;
  int t = t0;
  while (t < tend) {
    if (!__any(active)) break;  // identical in every wave: workgroup-uniform
    ++t;
    __syncthreads();  // P visible to all waves
    floatx16 qr, qi;
    if constexpr (VRS && SPL)
      apply_a_spl_vr<KT>(qr, qi, arow_full, ia < K, K, ia, false, vr_mask, PB, half, jl);
    else if constexpr (VRS)
      apply_a_vr<KT>(qr, qi, arow_full, ia < K, K, ia, false, vr_mask, Psh, half, jl);
    else if constexpr (SPL)
      apply_a_spl<KT>(qr, qi, arow_full, ia < K, K, ia, false, PB, half, jl);
    else
      apply_a<KT, AREG>(qr, qi, ar, ai, arow, klim, false, diag_s, Psh, half, jl);

    float g[1] = {0.f};
#pragma unroll
    for (int r = 0; r < 16; ++r) g[0] += pr[r] * qr[r] + pim[r] * qi[r];
    col_reduce<KT, 1>(g, red, w, jl, half);
    const float gamma = g[0];
    if (active) {
      if (!isfinite(gamma) || gamma < 0.f) {
        brk = true;  // A not numerically HPD
        active = false;
      } else if (gamma == 0.f) {
        conv = true;  // p = 0: the residual underflowed to zero, nothing left to solve
        active = false;
      }
    }
    const float alpha = active ? rho / gamma : 0.f;
    if (active) it = t;
    float s2[2] = {0.f, 0.f};
    if (active) {  // frozen columns keep x and r untouched (0 * NaN would not)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        xr[r] += alpha * pr[r];
        xim[r] += alpha * pim[r];
        rr[r] -= alpha * qr[r];
        ri[r] -= alpha * qi[r];
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float n2 = rr[r] * rr[r] + ri[r] * ri[r];
      s2[0] += n2;
      s2[1] += dinv[r] * n2;
    }
    col_reduce<KT, 2>(s2, red + 1, w, jl, half);
    if (active) {
      rres = s2[0];
      // Converged by the stop rule, or the residual underflowed: r^H D^{-1} r = 0
      // with D > 0 only for r = 0 (and the next beta would be 0/0).
      if (s2[0] <= tol2 * bb || s2[1] == 0.f) {
        active = false;
        conv = true;
      }
    }
    if (active) {
      const float beta = s2[1] / rho;
      rho = s2[1];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        pr[r] = dinv[r] * rr[r] + beta * pr[r];
        pim[r] = dinv[r] * ri[r] + beta * pim[r];
      }
    }
    if constexpr (SPL) {
      store_planes<KT>(pr, pim, PB, w, half, jl);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) Psh[w * 32 + d32_row(r, half)][jl] = make_float2(pr[r], pim[r]);
    }
  }

  const bool finished = !__any(active) || t >= p.max_iter;
  if (chunked && !finished) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = w * 16 * 64 + r * 64 + lane;
      stv[0 * kVecPerArray + o] = xr[r];
      stv[1 * kVecPerArray + o] = xim[r];
      stv[2 * kVecPerArray + o] = rr[r];
      stv[3 * kVecPerArray + o] = ri[r];
      stv[4 * kVecPerArray + o] = pr[r];
      stv[5 * kVecPerArray + o] = pim[r];
    }
    if (w == 0 && half == 0) {
      stc[0 * 32 + jl] = rho;
      stc[1 * 32 + jl] = bb;
      stc[2 * 32 + jl] = rres;
      stc[3 * 32 + jl] = (float)it;
      stc[4 * 32 + jl] = active ? 1.f : 0.f;
      stc[5 * 32 + jl] = conv ? 1.f : 0.f;
      stc[6 * 32 + jl] = brk ? 1.f : 0.f;
      if (jl == 0) stc[7 * 32 + 0] = (float)t;
    }
    if (threadIdx.x == 0) p.st.done[L] = 0;
    return;
  }

  // ---- final outputs --------------------------------------------------------
  // X through LDS: column jl of the block at jl * (KP + 1) (distinct banks for
  // the 32 lanes of one register), then stored with consecutive threads on
  // consecutive rows of a column.
  float2* Xb = p.X + (int64_t)b * p.stride_x;
  {
    float2* Xt = reinterpret_cast<float2*>(lds_raw);
    __syncthreads();  // every wave is done with P
#pragma unroll
    for (int r = 0; r < 16; ++r) Xt[jl * (KP + 1) + w * 32 + d32_row(r, half)] = make_float2(xr[r], xim[r]);
    __syncthreads();
    const int ncol = min(32, p.nrhs - cb * 32);
    for (int e = threadIdx.x; e < ncol * K; e += KT * 64) {
      const int jc = e / K, i = e - jc * K;
      Xb[(int64_t)(cb * 32 + jc) * p.ldx + i] = Xt[jc * (KP + 1) + i];
    }
  }
  int col_status = kStatusOk;
  if (brk)
    col_status = kStatusBreakdown;
  else if (p.tol > 0.f && !conv)
    col_status = kStatusNotConverged;
  if (w == 0 && half == 0 && jvalid) {
    if (p.iters) p.iters[(int64_t)b * p.nrhs + j] = it;
    if (p.relres) p.relres[(int64_t)b * p.nrhs + j] = bb > 0.f ? sqrtf(rres / bb) : 0.f;
  }
  if (p.wg_status) {
    const bool anyb = __any(brk);
    const bool anyn = __any(col_status == kStatusNotConverged);
    if (threadIdx.x == 0) p.wg_status[L] = anyb ? kStatusBreakdown : (anyn ? kStatusNotConverged : kStatusOk);
  }

  if (p.gdiag) {
    // ||H X||^2 contribution of this block: x_j^H (A - diag(A) + diag(H^H H)) x_j.
    __syncthreads();
    if constexpr (SPL) {
      store_planes<KT>(xr, xim, PB, w, half, jl);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) Psh[w * 32 + d32_row(r, half)][jl] = make_float2(xr[r], xim[r]);
    }
    __syncthreads();
    floatx16 yr, yi;
    if constexpr (VRS && SPL)
      apply_a_spl_vr<KT>(yr, yi, arow_full, ia < K, K, ia, true, vr_mask, PB, half, jl);
    else if constexpr (VRS)
      apply_a_vr<KT>(yr, yi, arow_full, ia < K, K, ia, true, vr_mask, Psh, half, jl);
    else if constexpr (SPL)
      apply_a_spl<KT>(yr, yi, arow_full, ia < K, K, ia, true, PB, half, jl);
    else
      apply_a<KT, AREG>(yr, yi, ar, ai, arow, klim, true, diag_s, Psh, half, jl);
    float q[1] = {0.f};
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = w * 32 + d32_row(r, half);
      const float gd = (i < K) ? p.gdiag[(int64_t)b * K + i] : 0.f;
      q[0] += xr[r] * yr[r] + xim[r] * yi[r] + gd * (xr[r] * xr[r] + xim[r] * xim[r]);
    }
    col_reduce<KT, 1>(q, red, w, jl, half);
    __shared__ float colsum[32];
    if (w == 0 && half == 0) colsum[jl] = q[0];
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int c = 0; c < 32; ++c) s += colsum[c];
      p.fpart[L] = s;
    }
  }
  if (chunked && threadIdx.x == 0) p.st.done[L] = 1;
}

__global__ void status_reduce_kernel(const int32_t* __restrict__ wg, int ncb, int batch, int32_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  int s = kStatusOk;
  for (int c = 0; c < ncb; ++c) {
    const int v = wg[(int64_t)b * ncb + c];
    if (v == kStatusBreakdown) s = kStatusBreakdown;
    else if (v == kStatusNotConverged && s == kStatusOk) s = kStatusNotConverged;
  }
  out[b] = s;
}

template <int KT, bool AREG>
hipError_t launch_kt(const PcgLaunch& p, int grid, hipStream_t s) {
  if constexpr (!AREG) {
    if (p.tile_span) {
      if constexpr (KT >= 3) {
        if (p.a_source != 2) {  // split-BF16 products (the default above K = 64)
          hipLaunchKernelGGL((pcg_f32_kernel<KT, false, true, true>), dim3(grid), dim3(KT * 64), 0, s, p);
          return hipGetLastError();
        }
      }
      hipLaunchKernelGGL((pcg_f32_kernel<KT, false, true>), dim3(grid), dim3(KT * 64), 0, s, p);
      return hipGetLastError();
    }
    if constexpr (KT >= 3) {
      if (p.a_source != 2) {  // split-BF16 products (the default above K = 64)
        hipLaunchKernelGGL((pcg_f32_kernel<KT, false, false, true>), dim3(grid), dim3(KT * 64), 0, s, p);
        return hipGetLastError();
      }
    }
  }
  hipLaunchKernelGGL((pcg_f32_kernel<KT, AREG, false>), dim3(grid), dim3(KT * 64), 0, s, p);
  return hipGetLastError();
}

}  // namespace

int pcg_workgroups(int batch, int K, int nrhs) {
  (void)K;
  return batch * ((nrhs + 31) / 32);
}

size_t pcg_state_floats_per_wg(int K) {
  const int kt = (K + 31) / 32;
  return (size_t)6 * kt * 16 * 64;
}

hipError_t launch_pcg(const PcgLaunch& p, hipStream_t s, int* wg_count_out) {
  const int grid = pcg_workgroups(p.batch, p.K, p.nrhs);
  if (wg_count_out) *wg_count_out = grid;
  if (grid == 0) return hipSuccess;
  const int kt = (p.K + 31) / 32;
  // K <= 64: each wave keeps its rows of A in registers, unless the tuned
  // choice streams them from L2 (FP32 products). Above K = 64 the rows are
  // streamed with split-BF16 products, unless the choice is FP32 products or
  // the spans of the sparse variant apply.
  const bool regs = p.a_source != 2;
  switch (kt) {
    case 1: return regs ? launch_kt<1, true>(p, grid, s) : launch_kt<1, false>(p, grid, s);
    case 2: return regs ? launch_kt<2, true>(p, grid, s) : launch_kt<2, false>(p, grid, s);
    case 3: return launch_kt<3, false>(p, grid, s);
    case 4: return launch_kt<4, false>(p, grid, s);
    case 5: return launch_kt<5, false>(p, grid, s);
    case 6: return launch_kt<6, false>(p, grid, s);
    case 7: return launch_kt<7, false>(p, grid, s);
    case 8: return launch_kt<8, false>(p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_status_reduce(const int32_t* wg_status, int ncb, int batch, int32_t* status, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(status_reduce_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, wg_status, ncb, batch,
                     status);
  return hipGetLastError();
}

}  // namespace jacpcg
