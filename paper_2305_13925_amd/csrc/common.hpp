// Shared declarations of the gfx950 kernels and the host runtime of libjacpcg.
//
// Matrix-core conventions used by every kernel (gfx950, wave64):
//   v_mfma_f32_32x32x2_f32   A-operand: lane l holds A[l%32][l/32]
//                            B-operand: lane l holds B[l/32][l%32]
//                            result reg r of lane l is D[8*(r/4) + 4*(l/32) + r%4][l%32]
//   v_mfma_f32_32x32x16_bf16 A-operand: lane l holds A[l%32][8*(l/32) + e], e < 8
//                            B-operand: lane l holds B[8*(l/32) + e][l%32]; result as above
//   v_mfma_f64_16x16x4_f64   A-operand: lane l holds A[l%16][l/16]
//                            B-operand: lane l holds B[l/16][l%16]
//                            result reg r of lane l is D[l/16 + 4*r][l%16]
// Complex products are formed from real MFMAs; the k dimension of one MFMA
// carries either the (re, im) parts of one complex term or two different
// complex terms, as documented in each kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jacpcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxK = 256;
constexpr int kMaxNrhs = 256;

// Row (within a 32x32 tile) of result register r in lane l of a 32x32 MFMA.
__host__ __device__ constexpr int d32_row(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }

// Severity order of per-instance statuses: BREAKDOWN > NOT_CONVERGED > OK.
constexpr int kStatusOk = 0;
constexpr int kStatusNotConverged = 1;
constexpr int kStatusBreakdown = -5;

// ---------------------------------------------------------------------------
// Launch descriptors (host -> kernels). Pointers are device pointers.
// ---------------------------------------------------------------------------
struct GramLaunch {
  const float2* H; int64_t ldh, stride_h;
  const float2* const* H_ptrs;  // nullable: per-instance channel pointers (ld ldh) instead of H + b * stride_h
  int batch, M, K;
  float xi;
  float2* A; int64_t lda, stride_a;
  float* diag;      // batch x K, Re diag(A) (nullable)
  float* gdiag;     // batch x K, diag(H^H H) without xi (nullable)
  int precision;    // 0 fp32, 1 bf16x3, 2 bf16x6
  int m_split;      // waves per workgroup that split the antenna range (tuned)
  int no_vec;       // 1: some channel pointer or ldh does not allow 16-byte loads
  const int2* tile_span;  // nullable: per (instance, 32-user block) antenna span [x, y) outside which
                          // every user of the block has a zero channel; tiles use only the overlap
  int msplit;             // FP32 Gram above K = 64 with partial: the antenna range in msplit chunks
  float2* partial;        // batch x blocks x msplit x 64 x 64 partial blocks (nullable)
};

// Per-workgroup resumable PCG state for chunked launches.
struct PcgState {
  float* vec;       // per WG: 6 arrays (x, r, p; re/im) of KT*16*64 floats
  float* col;       // per WG: 8 x 32 floats of per-column scalars
  int32_t* done;    // per WG: 1 when the WG has finished all its columns
};

struct PcgLaunch {
  const float2* A; int64_t lda, stride_a;
  const float2* B; int64_t ldb, stride_b;   // NULL => identity
  float2* X; int64_t ldx, stride_x;
  int batch, K, nrhs;
  float tol;                                // 0 => fixed max_iter
  int max_iter;
  int precond_none;
  int32_t* iters; float* relres;            // batch x nrhs (nullable)
  int32_t* wg_status;                       // per workgroup worst status (nullable)
  const float* gdiag;                       // nullable: enables the ||H X||^2 pass
  float* fpart;                             // per workgroup sum_j x_j^H G x_j
  PcgState st;                              // chunked mode when st.vec != NULL
  int chunk;                                // iterations in this launch (chunked mode)
  int first;                                // chunked mode: 1 on the first launch
  const int2* tile_span;                    // nullable: user-block antenna spans (as GramLaunch); tiles of A
                                            // whose blocks' spans are disjoint are zero and skipped (K > 64)
  const double* col_gate;                   // nullable: batch x nrhs; column j is solved only when
  double gate_tol;                          //   col_gate[j] > gate_tol (or NaN); other columns give x = 0
  int a_source;                             // where A is kept and how its products are formed: 0 default
                                            //   (registers up to K = 64; above, streamed from L2 with split-
                                            //   BF16 products, FP32 products with spans), 1 registers
                                            //   (K <= 64), 2 streamed from L2 with FP32 products, 3 streamed
                                            //   with split-BF16 products (K > 64 without spans; else as 0)
};

struct PrecoderLaunch {
  const float2* H; int64_t ldh, stride_h;
  const float2* const* H_ptrs;  // nullable: per-instance channel pointers
  float2* const* W_ptrs;        // nullable: per-instance precoder pointers (ld ldw)
  const float2* X; int64_t ldx, stride_x;
  float2* W; int64_t ldw, stride_w;
  int batch, M, K, nrhs;
  const float* fpart; int ncb;              // per instance: ncb partial ||H X||^2 terms
  float power;
  float* beta_out;                          // batch (nullable)
  int split;                                // 0: FP32 MFMA; 3: split-BF16 (3 parts, six products)
  const double* fpart64; int ncb64;         // nullable: FP64 ||H X||^2 partials (refined path)
  int no_vec;                               // 1: some precoder pointer or ldw does not allow 16-byte stores
  int nj;                                   // column tiles per wave: 0 = default rule, 1 or 2 = tuned choice
  int mtiles;                               // split-BF16: antenna blocks (128, or 256 beyond K = 128) per workgroup (0 = default rule)
  const int2* tile_span;                    // nullable (split-BF16, K > 64): user-block antenna spans; user
                                            // blocks whose span misses a workgroup's antennas are skipped
  const int32_t* wg_status;                 // nullable: the solver's per-workgroup statuses (ncb per instance),
  int32_t* status;                          // reduced here into the per-instance status (no separate launch)
  const double* ref_scale;                  // nullable (refined path): batch x nrhs final ||r_j||; a column
  double ref_tol;                           //   above ref_tol (or NaN) makes the instance NOT_CONVERGED
};

struct Gram64Launch {
  const float2* H; int64_t ldh, stride_h;
  int batch, M, K;
  double xi;
  double2* A64;                             // batch x K x K row-major, ld K
  const int2* tile_span;                    // nullable: per (instance, 32-user block) antenna spans (as
                                            // GramLaunch); a block uses only the overlap of its spans
  int msplit;                               // >= 2 with partial: the antenna range in msplit chunks
  double2* partial;                         // batch x blocks x msplit x 64 x 64 partial blocks (nullable)
};

// One refinement step (B = I): X64 += ||r_j|| E_j for the columns that missed
// the tolerance at the previous step (step 0: X64 = X32 widened), then
// R = I - A64 X64 and its column norms.
struct RefineStepLaunch {
  const double2* A64;                       // batch x K x K row-major, ld K, exactly Hermitian
  double2* X64;                             // batch x nrhs x K (column-major K x nrhs, ld K)
  float2* X32;                              // same layout: the first solve's X (step 0), then X64 rounded
  const float2* E32;                        // same layout: the previous step's corrections (step > 0)
  int batch, K, nrhs;
  int step;
  double xi;
  double tol;                               // column j is converged when ||r_j|| <= tol
  float2* R32;                              // same layout: r_j / ||r_j|| (next correction RHS)
  double* scale;                            // batch x nrhs: ||r_j|| (read as the previous step's at entry)
  double* rnorm2;                           // per workgroup: sum_j ||r_j||^2
  double* quad;                             // per workgroup: sum_j Re x_j^H (A64 - xi I) x_j
  int32_t* steps;                           // per workgroup: last step that ran (nullable)
  const int2* tile_span;                    // nullable: per (instance, 32-user block) antenna spans; rows
                                            // of A64 meet only the column blocks whose spans overlap theirs
};

// Visibility-region spans: per user the antenna range [first, end) outside
// which its channel is zero, and per 32-user block the hull of its users'.
struct SpanLaunch {
  const float2* H; int64_t ldh, stride_h;   // scanned when user_span_in is NULL
  const int32_t* user_span_in;              // nullable: batch x K x 2 (first, end) given by the caller
  int batch, M, K;
  int2* tile_span;                          // batch x ceil(K/32)
};

// Precoder evaluation (eqs. 8-10): C = H^H W, per-user SINR, sum rate.
struct EvalLaunch {
  const float2* H; int64_t ldh, stride_h;
  const float2* W; int64_t ldw, stride_w;
  int batch, M, K;
  float sigma2;
  float2* C;                                // workspace: batch x K x K row-major, C[k][j] = h_k^H w_j
  float* sinr;                              // batch x K
  float* se;                                // batch (nullable): sum_k log2(1 + SINR_k)
};

// Kernel launchers (defined in the .hip files). All return hipError_t of the
// launch itself.
hipError_t launch_gram(const GramLaunch& g, hipStream_t s);
hipError_t launch_pcg(const PcgLaunch& p, hipStream_t s, int* wg_count_out);
int pcg_workgroups(int batch, int K, int nrhs);
size_t pcg_state_floats_per_wg(int K);
hipError_t launch_status_reduce(const int32_t* wg_status, int ncb, int batch, int32_t* status, hipStream_t s);
hipError_t launch_precoder(const PrecoderLaunch& e, hipStream_t s);
hipError_t launch_gram64(const Gram64Launch& g, hipStream_t s);
int gram64_antenna_chunks(int K, int batch, bool spans);  // antenna chunks of the FP64 Gram (1: unsplit)
int gram_antenna_chunks(int K, int batch, int precision, bool spans);  // the same for the FP32 Gram
hipError_t launch_narrow_gram(const double2* A64, int K, int batch, double xi, float2* A, int64_t lda,
                              int64_t stride_a, float* gdiag, hipStream_t s);
hipError_t launch_refine_step(const RefineStepLaunch& r, hipStream_t s);
int refine_workgroups_per_instance(int nrhs);
hipError_t launch_zero_block(float2* G, int64_t ld, int64_t stride, int batch, int row0, int nrows, int col0,
                             int ncols, hipStream_t s);
hipError_t launch_fill_synthetic(float2* H, size_t n, uint32_t seed, hipStream_t s);
hipError_t launch_eval(const EvalLaunch& e, hipStream_t s);
hipError_t launch_spans(const SpanLaunch& sl, hipStream_t s);
hipError_t launch_widen(const float2* X, int64_t ldx, int64_t stride_x, int batch, int K, int n,
                        double2* out, hipStream_t s);

}  // namespace jacpcg
