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
__device__ __forceinline__ void load8(gptr<const float2> row, int m, int mend, bool valid, float2 (&v)[8]) {
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

constexpr int kGramMaxWaves = 8;

// Panels: tile row ti of the upper triangle cut into groups of up to two tiles.
__host__ __device__ inline int panels_per_instance(int nt) {
  int n = 0;
  for (int ti = 0; ti < nt; ++ti) n += (nt - ti + 1) / 2;
  return n;
}

__device__ __forceinline__ void panel_tiles(int p, int nt, int& ti, int& tj0, int& ntj) {
  for (ti = 0; ti < nt; ++ti) {
    const int np = (nt - ti + 1) / 2;
    if (p < np) break;
    p -= np;
  }
  tj0 = ti + 2 * p;
  ntj = min(2, nt - tj0);
}

// Antenna range of a tile (or a panel of tiles) of an instance. Without spans
// it is [0, M). With visibility-region spans it is the overlap of the row
// block's span with the column blocks' spans, widened to multiples of `align`
// (antennas outside a user's span hold zeros, so a wider range changes
// nothing); an empty overlap gives an empty range (the tile is zero).
__device__ __forceinline__ void tile_range(const GramLaunch& g, int b, int ti, int tj0, int ntj, int align, int& mb,
                                           int& me) {
  mb = 0;
  me = g.M;
  if (!g.tile_span) return;
  const int nt = (g.K + 31) >> 5;
  const int2 si = g.tile_span[(int64_t)b * nt + ti];
  int lo = g.M, hi = 0;
  for (int t = 0; t < ntj; ++t) {
    const int2 sj = g.tile_span[(int64_t)b * nt + tj0 + t];
    const int l = max(si.x, sj.x), h = min(si.y, sj.y);
    if (h > l) {
      lo = min(lo, l);
      hi = max(hi, h);
    }
  }
  if (hi <= lo) {
    mb = me = 0;
    return;
  }
  mb = (lo / align) * align;
  me = min(g.M, ((hi + align - 1) / align) * align);
}

// 4 consecutive complex entries row[m .. m+3] as 8 floats (re, im, ...), zero
// past `mend` or for a padding row.
template <bool VEC>
__device__ __forceinline__ void load4c(gptr<const float2> row, int m, int mend, bool valid, float (&v)[8]) {
  if (VEC && valid && m + 4 <= mend) {
    gptr<const float4> p = reinterpret_cast<gptr<const float4>>(row + m);
    const float4 a = ld4(p), c = ld4(p + 1);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float2 t = (valid && m + e < mend) ? ld2(row + m + e) : make_float2(0.f, 0.f);
      v[2 * e] = t.x;
      v[2 * e + 1] = t.y;
    }
  }
}

// Sum the waves' partial tiles (fixed wave order) and write tile (ti, tj) of A
// plus its conjugate mirror; the diagonal tile is mirrored inside itself and
// gets xi added to an exactly real diagonal. `red` holds nw * 2 * 16 * 64
// floats of LDS.
__device__ void reduce_and_write_tile(const GramLaunch& g, float* red_raw, const floatx16& accR,
                                      const floatx16& accI, int b, int ti, int tj, int wave, int nw, int lane) {
  float(*red)[2][16][64] = reinterpret_cast<float(*)[2][16][64]>(red_raw);
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
  const bool same = (ti == tj);
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
  gptr<const float2> Hb = as_global(g.H_ptrs ? g.H_ptrs[b] : g.H + (int64_t)b * g.stride_h);
  const int ui = ti * 32 + li, uj = tj * 32 + li;
  const bool vi = ui < g.K, vj = uj < g.K;
  gptr<const float2> hi = Hb + (int64_t)(vi ? ui : 0) * g.ldh;
  gptr<const float2> hj = Hb + (int64_t)(vj ? uj : 0) * g.ldh;
  const bool same = (ti == tj);

  int mb, me;
  tile_range(g, b, ti, tj, 1, 8, mb, me);
  const int chunk = ((me - mb + nw * 8 - 1) / (nw * 8)) * 8;
  const int m0 = mb + wave * chunk;
  const int m1 = min(me, m0 + chunk);

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

  extern __shared__ float red_dyn[];
  reduce_and_write_tile(g, red_dyn, accR, accI, b, ti, tj, wave, nw, lane);
}

// FP32 Gram for K > 64 without antenna spans: one workgroup (4 waves) per
// (instance, 64 x 64 block of the upper block triangle); wave w forms the
// 32 x 32 tile (w / 2, w % 2) of the block over the whole antenna range (on a
// diagonal block the tile below the diagonal is formed and not written). The
// block's channel rows pass through LDS 16 antennas at a time, stored as
// (-Im, Re, Im) triples (row operand) and (Re, Im) pairs (column operand), so
// that with the two k slots of v_mfma_f32_32x32x2_f32 carrying one antenna
//   Re A_ij += (Re h_i, Im h_i).(Re h_j, Im h_j)
//   Im A_ij += (-Im h_i, Re h_i).(Re h_j, Im h_j)
// and every operand is one LDS read. Each channel value is loaded once per
// block from global memory (the tile-per-workgroup kernel above reads each
// row once per tile it meets, with twice the loads per product).
constexpr int kG32Ant = 16;
constexpr int kG32PitchA = 3 * kG32Ant + 1;  // floats per row operand row (+1: bank spread)
constexpr int kG32PitchB = 2 * kG32Ant + 1;

// Split mode (partial set, msplit > 1): one workgroup per (instance, block,
// antenna chunk), chunk innermost; each chunk is a run of whole stages and its
// tiles go to a partial block that gram_f32_reduce_kernel sums.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gram_f32_block_kernel(GramLaunch g) {
  const int nb = (g.K + 63) >> 6;
  const int nblk = nb * (nb + 1) / 2;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const bool split = g.partial != nullptr && g.msplit > 1;
  const int S = split ? g.msplit : 1;
  const int item = L / S, chunk = L - item * S;
  const int b = item / nblk;
  int bi, bj;
  upper_tile(item - b * nblk, nb, bi, bj);
  const bool same = bi == bj;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kk = lane >> 5, li = lane & 31;
  const int ti = w >> 1, tj = w & 1;
  gptr<const float2> Hb = as_global(g.H_ptrs ? g.H_ptrs[b] : g.H + (int64_t)b * g.stride_h);
  const bool vec = !g.no_vec && ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);

  __shared__ float HsA[64][kG32PitchA];
  __shared__ float HsB[64][kG32PitchB];
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
        const int k = blk * 64 + row, mm = m + a2;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < g.K) {
          gptr<const float2> src = Hb + (int64_t)k * g.ldh + mm;
          if (vec && mm + 2 <= g.M) {
            v = ld4(reinterpret_cast<gptr<const float4>>(src));
          } else {
            if (mm < g.M) {
              const float2 t = ld2(src);
              v.x = t.x;
              v.y = t.y;
            }
            if (mm + 1 < g.M) {
              const float2 t = ld2(src + 1);
              v.z = t.x;
              v.w = t.y;
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
      float* d = &HsA[row][3 * a2];
      d[0] = -v.y;
      d[1] = v.x;
      d[2] = v.y;
      d[3] = -v.w;
      d[4] = v.z;
      d[5] = v.w;
      if (!same) {
        const float4 c = st[1][u];
        float* f = &HsB[row][2 * a2];
        f[0] = c.x;
        f[1] = c.y;
        f[2] = c.z;
        f[3] = c.w;
      }
    }
  };

  // Four accumulator pairs take the stage's antennas in turn (p % 4), so each
  // FP32 chain sums a quarter of the antennas (and four independent chains
  // keep the matrix core busy); they are added in a fixed order at the end.
  constexpr int kChains = 4;
  floatx16 accR[kChains], accI[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    accR[c] = zero16();
    accI[c] = zero16();
  }
  const float* ra = &HsA[32 * ti + li][0];
  const float* rb = same ? &HsA[32 * tj + li][1] : &HsB[32 * tj + li][0];
  const int pb = same ? 3 : 2;  // column operand stride per antenna (block-uniform)
  // Antenna range: all of M, or this chunk's whole stages.
  int mb = 0, me = g.M;
  if (split) {
    const int cs = ((g.M + S - 1) / S + kG32Ant - 1) / kG32Ant * kG32Ant;
    mb = min(g.M, chunk * cs);
    me = min(g.M, mb + cs);
  }
  const int nst = (me - mb + kG32Ant - 1) / kG32Ant;
  load_stage(mb);
  store_stage();
  __syncthreads();
  for (int s2 = 0; s2 < nst; ++s2) {
    if (s2 + 1 < nst) load_stage(mb + (s2 + 1) * kG32Ant);
#pragma unroll
    for (int p = 0; p < kG32Ant; ++p) {
      const float a_plain = ra[3 * p + 1 + kk];
      const float a_rot = ra[3 * p + kk];
      const float bv = rb[pb * p + kk];
      accR[p % kChains] = mfma32(a_plain, bv, accR[p % kChains]);
      accI[p % kChains] = mfma32(a_rot, bv, accI[p % kChains]);
    }
    __syncthreads();  // every wave is done with this stage
    if (s2 + 1 < nst) {
      store_stage();
      __syncthreads();
    }
  }

  // Write-out from the accumulators: element (i, j) of the tile is register
  // 4 (i / 8) + i % 4 of lane j + 32 ((i / 4) % 2). Entries above the diagonal
  // of A are written with their conjugate mirror; a diagonal entry gets xi
  // and an exactly zero imaginary part; a tile below the diagonal is skipped.
  const int gti = 2 * bi + ti, gtj = 2 * bj + tj;
  if (gti > gtj) return;
  const floatx16 sumR = (accR[0] + accR[1]) + (accR[2] + accR[3]);
  const floatx16 sumI = (accI[0] + accI[1]) + (accI[2] + accI[3]);
  if (split) {
    float2* Pb = g.partial + (int64_t)L * 64 * 64;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * kk + (r & 3);
      Pb[(32 * ti + i) * 64 + 32 * tj + li] = make_float2(sumR[r], sumI[r]);
    }
    return;
  }
  float2* Ab = g.A + (int64_t)b * g.stride_a;
  const int j = li, gj = gtj * 32 + j;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * kk + (r & 3);
    const int gi = gti * 32 + i;
    if (gi >= g.K || gj >= g.K || gi > gj) continue;
    const float re = sumR[r], im = sumI[r];
    if (gi == gj) {
      if (g.gdiag) g.gdiag[(int64_t)b * g.K + gi] = re;
      if (g.diag) g.diag[(int64_t)b * g.K + gi] = re + g.xi;
      Ab[(int64_t)gi * g.lda + gj] = make_float2(re + g.xi, 0.f);
    } else {
      Ab[(int64_t)gi * g.lda + gj] = make_float2(re, im);
      Ab[(int64_t)gj * g.lda + gi] = make_float2(re, -im);
    }
  }
}

// Sum of the antenna chunks' partial blocks in chunk order (fixed, so the
// result does not depend on scheduling), written as gram_f32_block_kernel
// writes its blocks: mirror above the diagonal, xi on the diagonal, diag and
// gdiag. One workgroup per (instance, block); the sums pass through LDS so the
// mirror is written along its rows too.
__global__ __launch_bounds__(256) void gram_f32_reduce_kernel(GramLaunch g) {
  const int nb = (g.K + 63) >> 6;
  const int nblk = nb * (nb + 1) / 2;
  const int item = blockIdx.x;
  const int b = item / nblk;
  int bi, bj;
  upper_tile(item - b * nblk, nb, bi, bj);
  const float2* P = g.partial + (int64_t)item * g.msplit * 64 * 64;
  float2* Ab = g.A + (int64_t)b * g.stride_a;
  __shared__ float2 T[64][65];
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    const int gi = bi * 64 + i, gj = bj * 64 + j;
    float re = 0.f, im = 0.f;
    for (int c = 0; c < g.msplit; ++c) {
      const float2 v = P[(int64_t)c * 64 * 64 + e];
      re += v.x;
      im += v.y;
    }
    T[i][j] = make_float2(re, im);
    if (gi >= g.K || gj >= g.K || gi > gj) continue;
    if (gi == gj) {
      if (g.gdiag) g.gdiag[(int64_t)b * g.K + gi] = re;
      if (g.diag) g.diag[(int64_t)b * g.K + gi] = re + g.xi;
      Ab[(int64_t)gi * g.lda + gj] = make_float2(re + g.xi, 0.f);
    } else {
      Ab[(int64_t)gi * g.lda + gj] = make_float2(re, im);
    }
  }
  __syncthreads();
  // Mirror: row gj of A, columns gi, consecutive threads on consecutive gi.
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int j = e >> 6, i = e & 63;
    const int gi = bi * 64 + i, gj = bj * 64 + j;
    if (gi >= gj || gj >= g.K) continue;
    const float2 v = T[i][j];
    Ab[(int64_t)gj * g.lda + gi] = make_float2(v.x, -v.y);
  }
}

// Split-BF16 Gram: one workgroup per (instance, panel of up to two tiles of one
// tile row), so the split of the row block's users is shared by both tiles.
// Real-plane formulation on v_mfma_f32_32x32x16_bf16: the 16 k slots are 16
// antennas (lane half c holds antennas m+8c .. m+8c+7) of one component, and
//   Re A_ij = sum_m Re h_im Re h_jm + Im h_im Im h_jm
//   Im A_ij = sum_m Re h_im Im h_jm + (-Im h_im) Re h_jm
// so each tile takes four split products per 16 antennas and the only extra
// work is one negation of the row block's imaginary plane, shared by the panel.
template <int NS, bool VEC>
__global__ __launch_bounds__(256) void gram_bf16_kernel(GramLaunch g) {
  const int nt = (g.K + 31) >> 5;
  const int npanel = panels_per_instance(nt);
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / npanel;
  int ti, tj0, ntj;
  panel_tiles(L - b * npanel, nt, ti, tj0, ntj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int half = lane >> 5, li = lane & 31;
  gptr<const float2> Hb = as_global(g.H_ptrs ? g.H_ptrs[b] : g.H + (int64_t)b * g.stride_h);
  const int ui = ti * 32 + li;
  const bool vi = ui < g.K;
  gptr<const float2> hi = Hb + (int64_t)(vi ? ui : 0) * g.ldh;
  // Tile t of the panel is (ti, tj0 + t); both tiles are always formed, each
  // from its own column block of users (a diagonal tile loads the row block a
  // second time; the second tile of a one-tile panel reads zeros and is not
  // written). Products under a branch, even a workgroup-uniform one, make the
  // compiler copy the accumulators between register files around each of them.
  bool vx[2];
  gptr<const float2> hx[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ux = (tj0 + q) * 32 + li;
    vx[q] = (q < ntj) && ux < g.K;
    hx[q] = Hb + (int64_t)(vx[q] ? ux : 0) * g.ldh;
  }

  int mb, me;
  tile_range(g, b, ti, tj0, ntj, 16, mb, me);
  const int chunk = ((me - mb + nw * 16 - 1) / (nw * 16)) * 16;
  const int m0 = mb + wave * chunk;
  const int m1 = min(me, m0 + chunk);

  floatx16 accR[2], accI[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    accR[t] = zero16();
    accI[t] = zero16();
  }
  auto load = [&](gptr<const float2> row, bool valid, int m, float (&re)[8], float (&im)[8]) {
    const int mm = m + 8 * half;
    if (VEC && valid && mm + 8 <= m1) {
      gptr<const float4> p = reinterpret_cast<gptr<const float4>>(row + mm);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 t = ld4(p + q);
        re[2 * q] = t.x;
        im[2 * q] = t.y;
        re[2 * q + 1] = t.z;
        im[2 * q + 1] = t.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 t = (valid && mm + e < m1) ? ld2(row + mm + e) : make_float2(0.f, 0.f);
        re[e] = t.x;
        im[e] = t.y;
      }
    }
  };
  for (int m = m0; m < m1; m += 16) {
    float ri[8], ii[8], rx[2][8], ix[2][8];
    load(hi, vi, m, ri, ii);
#pragma unroll
    for (int q = 0; q < 2; ++q) load(hx[q], vx[q], m, rx[q], ix[q]);
    u32x4 Ar[NS], Ai[NS], An[NS];
    split8<NS>(ri, Ar);
    split8<NS>(ii, Ai);
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) An[q][e] = neg_bf16x2(Ai[q][e]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      u32x4 Xr[NS], Xi[NS];
      split8<NS>(rx[q], Xr);
      split8<NS>(ix[q], Xi);
      floatx16& aR = accR[q];
      floatx16& aI = accI[q];
      split_mma<NS>(Ar, Xr, aR);
      split_mma<NS>(Ai, Xi, aR);
      split_mma<NS>(Ar, Xi, aI);
      split_mma<NS>(An, Xr, aI);
    }
  }

  extern __shared__ float red_dyn[];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t >= ntj) break;
    if (t > 0) __syncthreads();  // previous tile's write-out has read the buffer
    reduce_and_write_tile(g, red_dyn, accR[t], accI[t], b, ti, tj0 + t, wave, nw, lane);
  }
}


// Split-BF16 Gram for K <= 64: one workgroup per instance; each wave takes
// every nw-th 16-antenna step, splits each of the (at most two) user blocks
// once per step and forms all upper tiles (0,0), (0,1), (1,1) from those
// splits, so the split work per MFMA is a third of the panel kernel's. The
// next step's channel values are loaded before the products.
// EXACT: M is a multiple of 16 and the rows are 16-byte aligned, so every
// lane's 8 antennas are in range and the loads need no per-lane branch (rows
// past K repeat user 0; they feed only entries of A that are never written).
template <int NS, int NT, bool EXACT>
__global__ __launch_bounds__(256) void gram_bf16_small_kernel(GramLaunch g) {
  constexpr int NTILE = NT * (NT + 1) / 2;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int nw = blockDim.x >> 6;
  const int half = lane >> 5, li = lane & 31;
  gptr<const float2> Hb = as_global(g.H_ptrs ? g.H_ptrs[b] : g.H + (int64_t)b * g.stride_h);
  bool vu[NT];
  gptr<const float2> row[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int u = q * 32 + li;
    vu[q] = u < g.K;
    row[q] = Hb + (int64_t)(vu[q] ? u : 0) * g.ldh;
  }
  const int mstep = nw * 16;
  const int m0 = wave * 16;
  const int m1 = g.M;
  const bool vec = !g.no_vec && ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);

  floatx16 accR[NTILE], accI[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    accR[t] = zero16();
    accI[t] = zero16();
  }
  auto load = [&](int q, int m, float (&re)[8], float (&im)[8]) {
    const int mm = m + 8 * half;
    if (EXACT || (vec && vu[q] && mm + 8 <= m1)) {
      gptr<const float4> p = reinterpret_cast<gptr<const float4>>(row[q] + mm);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float4 t = ld4(p + c);
        re[2 * c] = t.x;
        im[2 * c] = t.y;
        re[2 * c + 1] = t.z;
        im[2 * c + 1] = t.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 t = (vu[q] && mm + e < m1) ? ld2(row[q] + mm + e) : make_float2(0.f, 0.f);
        re[e] = t.x;
        im[e] = t.y;
      }
    }
  };
  // One 16-antenna step from staged values: split, refill the stage with the
  // step `ahead` steps later (unconditionally: past the end it reloads the
  // current step, so no join has to wait for the load), then the products of
  // every upper tile.
  auto step = [&](float (&re)[NT][8], float (&im)[NT][8], int m, int ahead) {
    u32x4 Pr[NT][NS], Pi[NT][NS];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      split8<NS>(re[q], Pr[q]);
      split8<NS>(im[q], Pi[q]);
    }
    const int mnext = (m + ahead * mstep < m1) ? m + ahead * mstep : m;
#pragma unroll
    for (int q = 0; q < NT; ++q) load(q, mnext, re[q], im[q]);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    int t = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      u32x4 An[NS];
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
        for (int e = 0; e < 4; ++e) An[s2][e] = neg_bf16x2(Pi[a][s2][e]);
#pragma unroll
      for (int c = a; c < NT; ++c, ++t) {
        split_mma<NS>(Pr[a], Pr[c], accR[t]);
        split_mma<NS>(Pi[a], Pi[c], accR[t]);
        split_mma<NS>(Pr[a], Pi[c], accI[t]);
        split_mma<NS>(An, Pr[c], accI[t]);
      }
    }
  };
  if constexpr (EXACT) {
    // M is a multiple of 2 * mstep: two stages, each refilled two steps ahead.
    float reA[NT][8], imA[NT][8], reB[NT][8], imB[NT][8];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      load(q, m0, reA[q], imA[q]);
      load(q, m0 + mstep, reB[q], imB[q]);
    }
    for (int m = m0; m < m1; m += 2 * mstep) {
      step(reA, imA, m, 2);
      step(reB, imB, m + mstep, 2);
    }
  } else {
    float re[NT][8], im[NT][8];
    if (m0 < m1) {
#pragma unroll
      for (int q = 0; q < NT; ++q) load(q, m0, re[q], im[q]);
    }
    for (int m = m0; m < m1; m += mstep) step(re, im, m, 1);
  }

  extern __shared__ float red_dyn[];
  int t = 0;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int c = a; c < NT; ++c, ++t) {
      if (t > 0) __syncthreads();  // previous tile's write-out has read the buffer
      reduce_and_write_tile(g, red_dyn, accR[t], accI[t], b, a, c, wave, nw, lane);
    }
}

// Split-BF16 Gram for K > 64 without antenna spans: the 32-user blocks are
// taken in pairs and there is one workgroup per (instance, pair p <= pair q).
// A diagonal workgroup (p = q) splits the pair's two blocks and forms their
// three upper tiles, as the K <= 64 kernel does for its two blocks; an
// off-diagonal one splits the four blocks of pairs p and q and forms the 2 x 2
// tiles between them. Every upper tile is formed once, each block's split
// feeds two or three tiles, and a channel row is read by as many workgroups
// as there are pairs. Waves take every nw-th 16-antenna step; staged loads run
// two steps ahead when M is a multiple of 32 nw (EXACT), else one.
template <int NS, bool EXACT, bool DIAG>
__device__ __forceinline__ void gram_pair_body(const GramLaunch& g, gptr<const float2> Hb, int b, int p, int q,
                                               float* red) {
  constexpr int NB = DIAG ? 2 : 4;     // blocks loaded and split
  constexpr int NTILE = DIAG ? 3 : 4;  // tiles formed
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int half = lane >> 5, li = lane & 31;
  // loaded block n -> block of A
  auto blk = [&](int n) { return n < 2 ? 2 * p + n : 2 * q + n - 2; };
  // tile t -> (row, column) among the loaded blocks
  auto trow = [](int t) { return DIAG ? (t < 2 ? 0 : 1) : (t >> 1); };
  auto tcol = [](int t) { return DIAG ? (t == 0 ? 0 : 1) : 2 + (t & 1); };
  bool vu[NB];
  gptr<const float2> row[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    const int u = blk(n) * 32 + li;
    vu[n] = u < g.K;
    row[n] = Hb + (int64_t)(vu[n] ? u : 0) * g.ldh;
  }
  const int mstep = nw * 16;
  const int m0 = wave * 16;
  const int m1 = g.M;
  const bool vec = !g.no_vec && ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);

  floatx16 accR[NTILE], accI[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    accR[t] = zero16();
    accI[t] = zero16();
  }
  auto load = [&](int n, int m, float (&re)[8], float (&im)[8]) {
    const int mm = m + 8 * half;
    if (EXACT || (vec && vu[n] && mm + 8 <= m1)) {
      gptr<const float4> ptr = reinterpret_cast<gptr<const float4>>(row[n] + mm);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float4 t = ld4(ptr + c);
        re[2 * c] = t.x;
        im[2 * c] = t.y;
        re[2 * c + 1] = t.z;
        im[2 * c + 1] = t.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 t = (vu[n] && mm + e < m1) ? ld2(row[n] + mm + e) : make_float2(0.f, 0.f);
        re[e] = t.x;
        im[e] = t.y;
      }
    }
  };
  auto step = [&](float (&re)[NB][8], float (&im)[NB][8], int m, int ahead) {
    u32x4 Pr[NB][NS], Pi[NB][NS], An[2][NS];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      split8<NS>(re[n], Pr[n]);
      split8<NS>(im[n], Pi[n]);
    }
    const int mnext = (m + ahead * mstep < m1) ? m + ahead * mstep : m;
#pragma unroll
    for (int n = 0; n < NB; ++n) load(n, mnext, re[n], im[n]);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
        for (int e = 0; e < 4; ++e) An[a][s2][e] = neg_bf16x2(Pi[a][s2][e]);
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      const int a = trow(t), c = tcol(t);
      split_mma<NS>(Pr[a], Pr[c], accR[t]);
      split_mma<NS>(Pi[a], Pi[c], accR[t]);
      split_mma<NS>(Pr[a], Pi[c], accI[t]);
      split_mma<NS>(An[a], Pr[c], accI[t]);
    }
  };
  if constexpr (EXACT) {
    float reA[NB][8], imA[NB][8], reB[NB][8], imB[NB][8];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      load(n, m0, reA[n], imA[n]);
      load(n, m0 + mstep, reB[n], imB[n]);
    }
    for (int m = m0; m < m1; m += 2 * mstep) {
      step(reA, imA, m, 2);
      step(reB, imB, m + mstep, 2);
    }
  } else {
    float re[NB][8], im[NB][8];
    if (m0 < m1) {
#pragma unroll
      for (int n = 0; n < NB; ++n) load(n, m0, re[n], im[n]);
    }
    for (int m = m0; m < m1; m += mstep) step(re, im, m, 1);
  }
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    if (t > 0) __syncthreads();  // previous tile's write-out has read the buffer
    reduce_and_write_tile(g, red, accR[t], accI[t], b, blk(trow(t)), blk(tcol(t)), wave, nw, lane);
  }
}

__host__ __device__ inline int pair_groups_per_instance(int nt) {
  const int np = (nt + 1) / 2;
  return np * (np + 1) / 2;
}

template <int NS, bool EXACT>
__global__ __launch_bounds__(256) void gram_bf16_pair_kernel(GramLaunch g) {
  const int npp = pair_groups_per_instance((g.K + 31) >> 5);
  const int np = (((g.K + 31) >> 5) + 1) / 2;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int b = L / npp;
  int p, q;
  upper_tile(L - b * npp, np, p, q);
  gptr<const float2> Hb = as_global(g.H_ptrs ? g.H_ptrs[b] : g.H + (int64_t)b * g.stride_h);
  extern __shared__ float red_dyn[];
  if (p == q)  // workgroup-uniform
    gram_pair_body<NS, EXACT, true>(g, Hb, b, p, q, red_dyn);
  else
    gram_pair_body<NS, EXACT, false>(g, Hb, b, p, q, red_dyn);
}

}  // namespace

hipError_t launch_gram(const GramLaunch& g, hipStream_t s) {
  if (g.batch == 0) return hipSuccess;
  if (g.precision < 0 || g.precision > 2) return hipErrorNotSupported;
  const int nt = (g.K + 31) / 32;
  int waves = g.m_split > 0 ? g.m_split : 4;
  if (waves > kGramMaxWaves) waves = kGramMaxWaves;
  const dim3 block(64 * waves);
  const bool vec = !g.no_vec && ((uintptr_t)g.H % 16 == 0) && (g.ldh % 2 == 0) && (g.stride_h % 2 == 0);
  const size_t lds = (size_t)waves * 2 * 16 * 64 * sizeof(float);
  if (g.precision == 0 && nt > 2 && !g.tile_span) {
    const int nb = (g.K + 63) / 64;
    const int items = nb * (nb + 1) / 2 * g.batch;
    if (g.partial && g.msplit > 1) {
      hipLaunchKernelGGL(gram_f32_block_kernel, dim3((unsigned)(items * g.msplit)), dim3(256), 0, s, g);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(gram_f32_reduce_kernel, dim3((unsigned)items), dim3(256), 0, s, g);
    } else {
      hipLaunchKernelGGL(gram_f32_block_kernel, dim3((unsigned)items), dim3(256), 0, s, g);
    }
  } else if (g.precision == 0) {
    const dim3 grid((unsigned)(nt * (nt + 1) / 2 * g.batch));
    if (vec)
      hipLaunchKernelGGL(gram_f32_kernel<true>, grid, block, lds, s, g);
    else
      hipLaunchKernelGGL(gram_f32_kernel<false>, grid, block, lds, s, g);
  } else {
    // The split kernel is compiled for at most 256 threads (register budget).
    const int wb = waves > 4 ? 4 : waves;
    const dim3 block(64 * wb);
    const size_t lds = (size_t)wb * 2 * 16 * 64 * sizeof(float);
    if (nt <= 2) {
      const dim3 grid1((unsigned)g.batch);
      const bool exact = vec && (g.M % (32 * wb) == 0);
      auto pick = [&](auto k_exact, auto k_any) {
        if (exact)
          hipLaunchKernelGGL(k_exact, grid1, block, lds, s, g);
        else
          hipLaunchKernelGGL(k_any, grid1, block, lds, s, g);
      };
      if (g.precision == 1) {
        if (nt == 1)
          pick(gram_bf16_small_kernel<2, 1, true>, gram_bf16_small_kernel<2, 1, false>);
        else
          pick(gram_bf16_small_kernel<2, 2, true>, gram_bf16_small_kernel<2, 2, false>);
      } else {
        if (nt == 1)
          pick(gram_bf16_small_kernel<3, 1, true>, gram_bf16_small_kernel<3, 1, false>);
        else
          pick(gram_bf16_small_kernel<3, 2, true>, gram_bf16_small_kernel<3, 2, false>);
      }
      return hipGetLastError();
    }
    if (!g.tile_span) {
      const dim3 gridp((unsigned)(pair_groups_per_instance(nt) * g.batch));
      const bool exact = vec && (g.M % (32 * wb) == 0);
      if (g.precision == 1) {
        if (exact)
          hipLaunchKernelGGL((gram_bf16_pair_kernel<2, true>), gridp, block, lds, s, g);
        else
          hipLaunchKernelGGL((gram_bf16_pair_kernel<2, false>), gridp, block, lds, s, g);
      } else {
        if (exact)
          hipLaunchKernelGGL((gram_bf16_pair_kernel<3, true>), gridp, block, lds, s, g);
        else
          hipLaunchKernelGGL((gram_bf16_pair_kernel<3, false>), gridp, block, lds, s, g);
      }
      return hipGetLastError();
    }
    const dim3 grid((unsigned)(panels_per_instance(nt) * g.batch));
    if (g.precision == 1) {
      if (vec)
        hipLaunchKernelGGL((gram_bf16_kernel<2, true>), grid, block, lds, s, g);
      else
        hipLaunchKernelGGL((gram_bf16_kernel<2, false>), grid, block, lds, s, g);
    } else {
      if (vec)
        hipLaunchKernelGGL((gram_bf16_kernel<3, true>), grid, block, lds, s, g);
      else
        hipLaunchKernelGGL((gram_bf16_kernel<3, false>), grid, block, lds, s, g);
    }
  }
  return hipGetLastError();
}

int gram_antenna_chunks(int K, int batch, int precision, bool spans) {
  // The FP32 block kernel without spans. Above K = 128: 64 instances of
  // K = 256 give 640 workgroups for 768 slots (2.5 per compute unit), so the
  // compute units holding three set the time; four antenna chunks per block
  // give ten equal workgroups per compute unit. Above K = 64 with fewer than
  // 512 blocks in the batch, the chunks fill idle compute units; with every
  // block resident at once (256 instances of K = 128) they only add the sums.
  const int nb = (K + 63) / 64;
  const long items = (long)batch * (nb * (nb + 1) / 2);
  return (precision == 0 && !spans && (K > 128 || (K > 64 && items < 512))) ? 4 : 1;
}

}  // namespace jacpcg
