// FP64 side of the path: the FP64 Gram A64 = H^H H + xi I (from the same
// complex64 channel, widened exactly) and the refinement step (FP64
// accumulation X64 += ||r|| E of the FP32 correction solves, the residual
// R = I - A64 X64 and its column norms). Iterative refinement is not in the paper; it wins
// back the accuracy the FP32 (or split-BF16) Gram and the FP32 solve lose.
//
// v_mfma_f64_16x16x4_f64 layout: A-operand lane l holds A[l%16][l/16],
// B-operand B[l/16][l%16], result register r of lane l is D[l/16 + 4r][l%16].
// The four k slots carry two complex terms as (Re, Im) pairs.
#include <type_traits>

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

// One workgroup per (instance, 64 x 64 block of the upper block triangle of A).
// Wave w owns block rows 16w .. 16w+15 against all 64 block columns (four
// 16 x 16 tiles, so no reduction across waves); in a diagonal block the tiles
// wholly below the diagonal are not formed. The channel rows of the block
// pass through LDS 16 antennas at a time, widened to FP64 once as they are
// stored. Each entry conj(h_i) h_j = (a - ib)(c + id) takes three real
// products instead of four (Gauss's method):
//   t1 = a c,  t2 = b d,  t3 = (a - b)(c + d);
//   Re A_ij = t1 + t2,  Im A_ij = (t3 - t1) + t2 = a d - b c,
// each summed over the antennas on its own accumulator, the four k slots of
// one MFMA carrying four antennas. The row operand is stored as (a, b, a - b)
// triples and the column operand as (c, d, c + d), so every MFMA operand is
// a single LDS read. Im A_ij picks up rounding of the size of the terms'
// magnitudes, the same order as the four-product sum's; the diagonal's
// imaginary part is set to exactly zero.
// Global loads are coalesced 16-byte loads one stage ahead (into registers)
// of the products.
constexpr int kG64Rows = 64;  // block edge
constexpr int kG64Ant = 16;   // antennas per stage
constexpr int kG64Pitch = 3 * kG64Ant + 1;  // doubles per operand row (+1: bank spread)

__global__ __launch_bounds__(256) void gram64_kernel(Gram64Launch g) {
  const int nb = (g.K + kG64Rows - 1) / kG64Rows;
  const int nblk = nb * (nb + 1) / 2;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  // Split mode: workgroup (instance, block, antenna chunk), chunk innermost.
  const bool split = g.partial != nullptr && g.msplit > 1;
  const int S = split ? g.msplit : 1;
  const int item = L / S, chunk = L - item * S;
  const int b = item / nblk;
  int bi, bj;
  upper_tile16(item - b * nblk, nb, bi, bj);
  const bool same = bi == bj;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, li = lane & 15;
  const float2* Hb = g.H + (int64_t)b * g.stride_h;
  const bool vec = ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);

  // Row operand (block rows i) and column operand (block columns j); a
  // diagonal block loads its rows once and stores both operands from them.
  __shared__ double HsA[kG64Rows][kG64Pitch];
  __shared__ double HsB[kG64Rows][kG64Pitch];

  // Stage loads: each thread moves 2 x 16 bytes per operand (row = e / 8,
  // antennas 2 (e % 8) and 2 (e % 8) + 1 of the stage).
  float4 st[2][2];
  auto load_stage = [&](int m) {
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      if (op == 1 && same) break;  // block-uniform
      const int blk = op == 0 ? bi : bj;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int row = e >> 3, a2 = 2 * (e & 7);
        const int k = blk * kG64Rows + row, mm = m + a2;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < g.K) {
          const float2* src = Hb + (int64_t)k * g.ldh + mm;
          if (vec && mm + 2 <= g.M) {
            v = *reinterpret_cast<const float4*>(src);
          } else {
            if (mm < g.M) {
              v.x = src[0].x;
              v.y = src[0].y;
            }
            if (mm + 1 < g.M) {
              v.z = src[1].x;
              v.w = src[1].y;
            }
          }
        }
        st[op][u] = v;
      }
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int row = e >> 3, a2 = 2 * (e & 7);
      const float4 v = st[0][u];
      double* d = &HsA[row][3 * a2];
      d[0] = (double)v.x;
      d[1] = (double)v.y;
      d[2] = (double)v.x - (double)v.y;
      d[3] = (double)v.z;
      d[4] = (double)v.w;
      d[5] = (double)v.z - (double)v.w;
      const float4 c = same ? v : st[1][u];
      double* f = &HsB[row][3 * a2];
      f[0] = (double)c.x;
      f[1] = (double)c.y;
      f[2] = (double)c.x + (double)c.y;
      f[3] = (double)c.z;
      f[4] = (double)c.w;
      f[5] = (double)c.z + (double)c.w;
    }
  };

  doublex4 t1[4], t2[4], t3[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    t1[c] = zero4d();
    t2[c] = zero4d();
    t3[c] = zero4d();
  }
  // The products of one stage for NT tiles (row tile R[t] of the row operand,
  // column tile C[t] of the column operand). Called with compile-time tile
  // lists, so every LDS offset is static and every product is unconditional.
  auto products = [&](auto nt_tag, const int (&R)[4], const int (&C)[4]) {
    constexpr int NT = decltype(nt_tag)::value;
#pragma unroll  // the operands of the four steps are loaded ahead
    for (int p = 0; p < kG64Ant / 4; ++p) {
      const int ant = 4 * p + q;  // k slot q
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const double* ra = &HsA[16 * R[c] + li][3 * ant];
        const double* cb = &HsB[16 * C[c] + li][3 * ant];
        t1[c] = mfma64(ra[0], cb[0], t1[c]);
        t2[c] = mfma64(ra[1], cb[1], t2[c]);
        t3[c] = mfma64(ra[2], cb[2], t3[c]);
      }
    }
  };
  // Tiles of each wave. Off the diagonal: row tile w against the four column
  // tiles. On it: the ten upper tiles (r <= c) dealt 3, 3, 2, 2 over the waves,
  // so no tile below the diagonal is formed.
  constexpr int kDiagR[4][4] = {{0, 0, 0, 0}, {0, 1, 1, 0}, {1, 2, 0, 0}, {2, 3, 0, 0}};
  constexpr int kDiagC[4][4] = {{0, 1, 2, 0}, {3, 1, 2, 0}, {3, 2, 0, 0}, {3, 3, 0, 0}};
  const int offR[4] = {w, w, w, w};
  constexpr int offC[4] = {0, 1, 2, 3};
  const int ntile = same ? (w < 2 ? 3 : 2) : 4;
  auto stage = [&]() {
    if (!same) {
      products(std::integral_constant<int, 4>{}, offR, offC);
    } else {
      switch (w) {  // wave-uniform
        case 0: products(std::integral_constant<int, 3>{}, kDiagR[0], kDiagC[0]); break;
        case 1: products(std::integral_constant<int, 3>{}, kDiagR[1], kDiagC[1]); break;
        case 2: products(std::integral_constant<int, 2>{}, kDiagR[2], kDiagC[2]); break;
        default: products(std::integral_constant<int, 2>{}, kDiagR[3], kDiagC[3]); break;
      }
    }
  };
  // Antenna range: all of M, or with visibility-region spans the overlap of
  // the row block's and the column block's ranges (each the union of its two
  // 32-user blocks' spans), widened to whole stages (antennas outside a user's
  // span hold zeros). An empty overlap leaves the block exactly zero.
  int mb = 0, me = g.M;
  if (g.tile_span) {
    const int nt = (g.K + 31) >> 5;
    auto range64 = [&](int blk, int& lo, int& hi) {
      lo = g.M;
      hi = 0;
      for (int t = 2 * blk; t < min(2 * blk + 2, nt); ++t) {
        const int2 sp = g.tile_span[(int64_t)b * nt + t];
        if (sp.y > sp.x) {
          lo = min(lo, sp.x);
          hi = max(hi, sp.y);
        }
      }
    };
    int lo0, hi0, lo1, hi1;
    range64(bi, lo0, hi0);
    range64(bj, lo1, hi1);
    const int lo = max(lo0, lo1), hi = min(hi0, hi1);
    mb = hi > lo ? (lo / kG64Ant) * kG64Ant : 0;
    me = hi > lo ? min(g.M, hi) : 0;
  }
  if (split) {  // this chunk of the antennas (whole stages)
    const int cs = ((g.M + S - 1) / S + kG64Ant - 1) / kG64Ant * kG64Ant;
    mb = max(mb, chunk * cs);
    me = min(me, (chunk + 1) * cs);
    if (me <= mb) me = mb;
  }
  const int nst = (me - mb + kG64Ant - 1) / kG64Ant;
  load_stage(mb);
  store_stage();
  __syncthreads();
  for (int s2 = 0; s2 < nst; ++s2) {
    if (s2 + 1 < nst) load_stage(mb + (s2 + 1) * kG64Ant);
    stage();
    __syncthreads();  // every wave is done with this stage
    if (s2 + 1 < nst) {
      store_stage();
      __syncthreads();
    }
  }

  // Element (row q + 4r, column li) of a tile sits in register r. Each entry
  // strictly above the diagonal of A is written with its conjugate mirror, the
  // diagonal gets xi and an exactly zero imaginary part; entries below the
  // diagonal of a diagonal tile are left to their mirror. In split mode the
  // formed tiles go to this chunk's partial block instead.
  const int wq = min(w, 3);
  if (split) {
    double2* Pb = g.partial + (int64_t)L * kG64Rows * kG64Rows;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= ntile) continue;
      const int tr = same ? kDiagR[wq][c] : w;
      const int tc = same ? kDiagC[wq][c] : c;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Pb[(16 * tr + q + 4 * r) * kG64Rows + 16 * tc + li] =
            make_double2(t1[c][r] + t2[c][r], (t3[c][r] - t1[c][r]) + t2[c][r]);
    }
    return;
  }
  double2* Ab = g.A64 + (int64_t)b * g.K * g.K;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= ntile) continue;
    const int tr = same ? kDiagR[wq][c] : w;
    const int tc = same ? kDiagC[wq][c] : c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = bi * kG64Rows + 16 * tr + q + 4 * r;
      const int gj = bj * kG64Rows + 16 * tc + li;
      if (gi >= g.K || gj >= g.K || gi > gj) continue;
      const double re = t1[c][r] + t2[c][r], im = (t3[c][r] - t1[c][r]) + t2[c][r];
      if (gi == gj) {
        Ab[(int64_t)gi * g.K + gj] = make_double2(re + g.xi, 0.0);
      } else {
        Ab[(int64_t)gi * g.K + gj] = make_double2(re, im);
        Ab[(int64_t)gj * g.K + gi] = make_double2(re, -im);
      }
    }
  }
}

// Sum of the antenna chunks' partial blocks in chunk order (fixed, so the
// result does not depend on scheduling), written like gram64_kernel's blocks:
// entries above the diagonal with their conjugate mirror, xi on the diagonal.
// One workgroup per (instance, block); the sums pass through LDS, half a
// block at a time, so the mirror is written along its rows too.
__global__ __launch_bounds__(256) void gram64_reduce_kernel(Gram64Launch g) {
  const int nb = (g.K + kG64Rows - 1) / kG64Rows;
  const int nblk = nb * (nb + 1) / 2;
  const int item = blockIdx.x;
  const int b = item / nblk;
  int bi, bj;
  upper_tile16(item - b * nblk, nb, bi, bj);
  const double2* P = g.partial + (int64_t)item * g.msplit * kG64Rows * kG64Rows;
  double2* Ab = g.A64 + (int64_t)b * g.K * g.K;
  constexpr int kHalf = kG64Rows / 2;
  __shared__ double2 T[kHalf][kG64Rows + 1];
  for (int h = 0; h < 2; ++h) {
    if (h > 0) __syncthreads();  // the first half's mirror has read T
    for (int e = threadIdx.x; e < kHalf * kG64Rows; e += 256) {
      const int il = e / kG64Rows, j = e - il * kG64Rows;
      const int i = h * kHalf + il;
      const int gi = bi * kG64Rows + i, gj = bj * kG64Rows + j;
      double re = 0.0, im = 0.0;
      for (int c = 0; c < g.msplit; ++c) {
        const double2 v = P[(int64_t)c * kG64Rows * kG64Rows + i * kG64Rows + j];
        re += v.x;
        im += v.y;
      }
      T[il][j] = make_double2(re, im);
      if (gi >= g.K || gj >= g.K || gi > gj) continue;
      Ab[(int64_t)gi * g.K + gj] = gi == gj ? make_double2(re + g.xi, 0.0) : make_double2(re, im);
    }
    __syncthreads();
    // Mirror of this half: rows gj of A, columns gi (consecutive threads on
    // consecutive gi).
    for (int e = threadIdx.x; e < kHalf * kG64Rows; e += 256) {
      const int j = e / kHalf, il = e - j * kHalf;
      const int gi = bi * kG64Rows + h * kHalf + il, gj = bj * kG64Rows + j;
      if (gi >= gj || gj >= g.K) continue;
      const double2 v = T[il][j];
      Ab[(int64_t)gj * g.K + gi] = make_double2(v.x, -v.y);
    }
  }
}

// One step of iterative refinement for one instance and 16 right-hand-side
// columns of B = I (workgroup of 4 waves):
//   1. X64 of the block's columns: at step 0 the first FP32 solution widened
//      exactly; at a later step X64 += ||r_j|| E_j for every column j whose
//      residual at the previous step missed the tolerance (E_j solves
//      A E_j = r_j / ||r_j|| in FP32). The rounded X64 goes back to X32 for the
//      precoder. A block whose columns had all converged returns at once:
//      its X, residual and partial sums stand from the step that ran last.
//   2. R = I - A64 X64 in FP64 on the matrix cores; per column ||r_j||, the
//      FP32 right-hand side r_j / ||r_j|| of the next correction solve; per
//      workgroup sum_j ||r_j||^2 and sum_j Re x_j^H (A64 - xi I) x_j =
//      sum_j ||H x_j||^2 (FP64, the power factor of the precoder).
// X64 of the block sits in LDS as the B-operand. A64 is exactly Hermitian,
// so the A-operand entry A[i][k] is read as conj(A[k][i]): the 16 lanes of one
// k slot then load 256 contiguous bytes of row k. Wave w owns the RT
// consecutive row tiles from w RT; k is outermost, so its row tiles' products
// are independent accumulation chains, and the A entries are loaded four
// steps ahead of the products.
template <int RT>
__global__ __launch_bounds__(256) void refine_step_kernel(RefineStepLaunch r) {
  constexpr int KM = 64 * RT;  // largest K of this variant
  const int n16 = (r.nrhs + 15) >> 4;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / n16, cb = L - b * n16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, li = lane & 15;
  const int slot_k = q >> 1, comp = q & 1;
  const int K = r.K;
  const int j0 = cb * 16;
  const int ncol = min(16, r.nrhs - j0);
  const int64_t xo = (int64_t)b * K * r.nrhs;
  double* scale = r.scale + (int64_t)b * r.nrhs;

  if (r.step > 0) {
    bool need = false;
    for (int c = 0; c < ncol; ++c) need |= !(scale[j0 + c] <= r.tol);  // NaN keeps refining
    if (!need) return;
  }

  // X64 of the block's columns; entries K .. KM - 1 stay zero, so the
  // products of steps past K add nothing.
  __shared__ double2 Xs[16][KM + 1];
  for (int e = threadIdx.x; e < 16 * KM; e += 256) {
    const int jj = e / KM, i = e - jj * KM;
    double2 x = make_double2(0.0, 0.0);
    if (jj < ncol && i < K) {
      const int64_t o = xo + (int64_t)(j0 + jj) * K + i;
      if (r.step == 0) {
        const float2 v = r.X32[o];
        x = make_double2(v.x, v.y);
        r.X64[o] = x;
      } else {
        x = r.X64[o];
        const double sc = scale[j0 + jj];
        if (!(sc <= r.tol)) {
          const float2 ev = r.E32[o];
          x.x += sc * (double)ev.x;
          x.y += sc * (double)ev.y;
          r.X64[o] = x;
          r.X32[o] = make_float2((float)x.x, (float)x.y);
        }
      }
    }
    Xs[jj][i] = x;
  }
  if (threadIdx.x == 0 && r.steps) r.steps[L] = r.step;
  __syncthreads();

  gptr<const double2> Ab = as_global(r.A64 + (int64_t)b * K * K);
  const int ntr = (K + 15) >> 4;
  doublex4 qr[RT], qi[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    qr[t] = zero4d();
    qi[t] = zero4d();
  }
  // With a = A[kk][i] (so A[i][kk] = conj(a)) and the B-operand x[comp] of
  // column j at step kk, the k slots comp = 0, 1 of two products give
  //   Re (A x)_i = a.x Re x + a.y Im x    (A-operand a[comp])
  //   Im (A x)_i = -a.y Re x + a.x Im x   (A-operand (-a.y, a.x)[comp])
  // so each operand is one 8-byte load with no select: the second one reads
  // component 1 - comp and flips its sign bit in slot 0. Loads are
  // unconditional (indices clamped into A): rows past K are never written and
  // steps past K meet zeros of X.
  gptr<const double> Ad = reinterpret_cast<gptr<const double>>(Ab);
  int ia_c[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) ia_c[t] = min((w * RT + t) * 16 + li, K - 1);
  const uint32_t sign2 = comp ? 0u : 0x80000000u;
  auto load_a = [&](int k0, double (&d1)[RT], double (&d2)[RT]) {
    const int kk = min(k0 + slot_k, K - 1);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int64_t o = 2 * ((int64_t)kk * K + ia_c[t]);
      d1[t] = Ad[o + comp];
      d2[t] = Ad[o + 1 - comp];
    }
  };
  const double* xrow = &Xs[li][0].x + comp;
  // One complex step pair k0: operands from the staged values, then the stage
  // is refilled with step k0 + 2 * kStages (clamped into A, so past the end it
  // reloads a valid row and the join never waits), then the products.
  constexpr int kStages = 4;
  auto step = [&](double (&a1)[RT], double (&a2)[RT], int k0) {
    const double xv = xrow[2 * (k0 + slot_k)];
    double b2[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const uint64_t u = __builtin_bit_cast(uint64_t, a2[t]) ^ ((uint64_t)sign2 << 32);
      b2[t] = __builtin_bit_cast(double, u);
    }
    double c1[RT];  // the stage is refilled before the products
#pragma unroll
    for (int t = 0; t < RT; ++t) c1[t] = a1[t];
    load_a(k0 + 2 * kStages, a1, a2);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    // Every row tile is formed (rows beyond K give discarded rows): a branch
    // around the products, though wave-uniform, makes the compiler move the
    // accumulators between register files around each one.
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      qr[t] = mfma64(c1[t], xv, qr[t]);
      qi[t] = mfma64(b2[t], xv, qi[t]);
    }
  };
  // Range of k the wave's rows meet: all of it, or with visibility-region
  // spans the wave's own 32-user blocks (xi on the diagonal) and every block
  // whose span overlaps the hull of theirs (A64[i][k] - xi delta_ik is exactly
  // zero when users i and k share no antenna), as one range of whole blocks.
  int klo = 0, khi = K;
  if (r.tile_span) {
    const int nt = (K + 31) >> 5;
    const int2* sp = r.tile_span + (int64_t)b * nt;
    const int rb0 = min(nt - 1, (w * RT * 16) >> 5);
    const int rb1 = max(rb0 + 1, min(nt, ((w + 1) * RT * 16 + 31) >> 5));
    int ulo = 1 << 30, uhi = -1;
    for (int t = rb0; t < rb1; ++t)
      if (sp[t].y > sp[t].x) {
        ulo = min(ulo, sp[t].x);
        uhi = max(uhi, sp[t].y);
      }
    int tlo = rb0, thi = rb1 - 1;
    for (int t = 0; t < nt; ++t)
      if (sp[t].y > sp[t].x && sp[t].y > ulo && sp[t].x < uhi) {
        tlo = min(tlo, t);
        thi = max(thi, t);
      }
    klo = 32 * tlo;
    khi = min(32 * (thi + 1), KM);
  }
  double st1[kStages][RT], st2[kStages][RT];
#pragma unroll
  for (int u = 0; u < kStages; ++u) {
    load_a(klo + 2 * u, st1[u], st2[u]);
    __builtin_amdgcn_sched_barrier(0);  // stages issued in order: stage 0 arrives first
  }
  for (int k0 = klo; k0 < khi; k0 += 2 * kStages) {
#pragma unroll
    for (int u = 0; u < kStages; ++u) step(st1[u], st2[u], k0 + 2 * u);
  }

  // Own rows of the result: rt*16 + q + 4*g, column j0 + li.
  const bool jv = li < ncol;
  double nr = 0.0, quad = 0.0;
  double rre[RT][4], rim[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int rt = w * RT + t;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int i = rt * 16 + q + 4 * g;
      rre[t][g] = 0.0;
      rim[t][g] = 0.0;
      if (rt >= ntr || i >= K || !jv) continue;
      rre[t][g] = (i == j0 + li ? 1.0 : 0.0) - qr[t][g];
      rim[t][g] = -qi[t][g];
      nr += rre[t][g] * rre[t][g] + rim[t][g] * rim[t][g];
      const double2 x = Xs[li][i];
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
  for (int t = 0; t < RT; ++t) {
    const int rt = w * RT + t;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int i = rt * 16 + q + 4 * g;
      if (rt < ntr && i < K && jv)
        r.R32[xo + (int64_t)(j0 + li) * K + i] = make_float2((float)(rre[t][g] * inv), (float)(rim[t][g] * inv));
    }
  }
  if (w == 0 && q == 0 && jv) scale[j0 + li] = sc;
  if (threadIdx.x == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < 16; ++c) {
      s1 += cs[0][0][c] + cs[0][1][c] + cs[0][2][c] + cs[0][3][c];
      s2 += cs[1][0][c] + cs[1][1][c] + cs[1][2][c] + cs[1][3][c];
    }
    r.rnorm2[L] = s1;
    r.quad[L] = s2;
  }
}

// The FP32 system matrix of the refined path: A64 rounded once to FP32 (more
// accurate than any FP32-accumulated Gram), and diag(H^H H) = Re A64_ii - xi
// for the solver's power partials.
__global__ void narrow_gram_kernel(const double2* __restrict__ A64, int K, double xi, float2* __restrict__ A,
                                   int64_t lda, int64_t stride_a, float* __restrict__ gdiag) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * K) return;
  const int i = idx / K, j = idx - i * K;
  const double2 v = A64[(int64_t)b * K * K + idx];
  A[(int64_t)b * stride_a + (int64_t)i * lda + j] = make_float2((float)v.x, (float)v.y);
  if (i == j && gdiag) gdiag[(int64_t)b * K + i] = (float)(v.x - xi);
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
  const int nb = (g.K + kG64Rows - 1) / kG64Rows;
  const int items = nb * (nb + 1) / 2 * g.batch;
  if (g.partial && g.msplit > 1) {
    hipLaunchKernelGGL(gram64_kernel, dim3((unsigned)(items * g.msplit)), dim3(256), 0, s, g);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram64_reduce_kernel, dim3((unsigned)items), dim3(256), 0, s, g);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(gram64_kernel, dim3((unsigned)items), dim3(256), 0, s, g);
  return hipGetLastError();
}

int gram64_antenna_chunks(int K, int batch, bool spans) {
  // Above K = 128 a batch has few 64 x 64 blocks of unequal work (diagonal
  // blocks form 10 of their 16 tiles) for the compute units; four antenna
  // chunks per block even out the load. Above K = 64 the same when the batch
  // has fewer than 512 blocks (idle compute units), and two chunks with more:
  // two workgroups fit a compute unit, so 768 blocks (256 instances of
  // K = 128) would run in one and a half rounds. Not with spans (sparse
  // blocks).
  if (spans || K <= kG64Rows) return 1;
  const int nb = (K + kG64Rows - 1) / kG64Rows;
  const long items = (long)batch * (nb * (nb + 1) / 2);
  return (K > 2 * kG64Rows || items < 512) ? 4 : 2;
}

hipError_t launch_narrow_gram(const double2* A64, int K, int batch, double xi, float2* A, int64_t lda,
                              int64_t stride_a, float* gdiag, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  const dim3 grid((unsigned)((K * K + 255) / 256), (unsigned)batch);
  hipLaunchKernelGGL(narrow_gram_kernel, grid, dim3(256), 0, s, A64, K, xi, A, lda, stride_a, gdiag);
  return hipGetLastError();
}

hipError_t launch_refine_step(const RefineStepLaunch& r, hipStream_t s) {
  if (r.batch == 0) return hipSuccess;
  const dim3 grid((unsigned)(r.batch * refine_workgroups_per_instance(r.nrhs)));
  if (r.K <= 64)
    hipLaunchKernelGGL(refine_step_kernel<1>, grid, dim3(256), 0, s, r);
  else if (r.K <= 128)
    hipLaunchKernelGGL(refine_step_kernel<2>, grid, dim3(256), 0, s, r);
  else if (r.K <= 256)
    hipLaunchKernelGGL(refine_step_kernel<4>, grid, dim3(256), 0, s, r);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int refine_workgroups_per_instance(int nrhs) { return (nrhs + 15) / 16; }

hipError_t launch_widen(const float2* X, int64_t ldx, int64_t stride_x, int batch, int K, int n, double2* out,
                        hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3((K * n + 255) / 256, batch), dim3(256), 0, s, X, ldx, stride_x, K, n, out);
  return hipGetLastError();
}

}  // namespace jacpcg
