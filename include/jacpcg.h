/*
 * jacpcg.h -- C ABI of libjacpcg.so: the RZF precoder computed by
 * Jacobi-preconditioned conjugate gradient, on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Xu et al., "Jac-PCG Based Low-Complexity Precoding for
 * Extremely Large-Scale MIMO Systems":
 *   - regularised Gram A = H^H H + xi I_K               (Sec. II, eq. 7: P_i)
 *   - Jacobi-preconditioned CG on A X = B, C = diag(A)  (Sec. III-B, eq. 21,
 *                                                        Algorithm 1)
 *   - precoder W = beta_pow H X, beta_pow = sqrt(P_tx / ||H X||_F^2)
 *                                                       (eq. 7, the power factor
 *                                                        after it, and eq. 15)
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) pairs: jacpcg_c64 has the
 *     storage of torch.complex64 / std::complex<float>, jacpcg_c128 that of
 *     complex128.
 *   - Matrix pointers are DEVICE pointers owned by the caller; the library never
 *     frees them. Host pointers are marked "host".
 *   - H (M x K per instance) is column-major: H[k * ldh + m] is antenna m of
 *     user k (each user's channel vector h_k is contiguous), ldh >= M.
 *   - A (K x K) is row-major with both triangles stored: A[i * lda + j] = A_ij,
 *     lda >= K. A is Hermitian, so the row-major and column-major readings
 *     differ only by conjugation.
 *   - B, X (K x nrhs) and W (M x nrhs) are column-major: X[j * ldx + i].
 *   - Batches are strided: instance b of a matrix starts at ptr + b * stride
 *     (strides in elements of the pointee type).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *     is enqueued asynchronously on it; outputs are valid after the stream is
 *     synchronised, unless the entry point says it synchronises.
 *   - The calls of one session share its workspace. A call on another stream
 *     than the session's previous call first makes its stream wait for that
 *     call's work, so a caller may alternate streams without synchronising.
 *   - Every call returns a status code. Argument errors are detected on the
 *     host before any device work and leave outputs untouched; the detail is
 *     available from jacpcg_last_error() on the calling thread.
 *   - Sizes: 1 <= K <= 256, 1 <= M, 1 <= nrhs <= 256, batch >= 0 (0 = no-op).
 */
#ifndef JACPCG_H
#define JACPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jacpcg_session jacpcg_session;
typedef struct { float re, im; } jacpcg_c64;
typedef struct { double re, im; } jacpcg_c128;

/* Status codes. Positive: warnings, outputs are valid. Negative: errors. */
enum {
  JACPCG_OK = 0,
  JACPCG_NOT_CONVERGED = 1,   /* some column missed `tol` within max_iter (Step 2 stop rule) */
  JACPCG_NOT_READY = 2,       /* request still in flight */
  JACPCG_E_INVALID_ARG = -1,
  JACPCG_E_UNSUPPORTED = -2,
  JACPCG_E_NO_DEVICE = -3,
  JACPCG_E_OUT_OF_MEMORY = -4,
  JACPCG_E_BREAKDOWN = -5,    /* p^H A p < 0 or non-finite: A not numerically HPD (eq. 18) */
  JACPCG_E_HIP = -6,
  JACPCG_E_BUDGET = -7,       /* request can never fit the session's HBM budget */
  JACPCG_E_CANCELLED = -8,
  JACPCG_E_TIMEOUT = -9
};

/* Gram precision (jacpcg_gram, rzf_precoder `precision`). */
enum {
  JACPCG_GRAM_FP32 = 0,       /* FP32 MFMA, FP32 accumulation */
  JACPCG_GRAM_BF16X3 = 1,     /* split BF16 hi+lo, products hi*hi + hi*lo + lo*hi, FP32 accumulation */
  JACPCG_GRAM_BF16X6 = 2,     /* split BF16 hi+mid+lo (exact split of FP32), six products, FP32 accumulation */
  JACPCG_GRAM_FP64_ROUNDED = 3, /* with JACPCG_REFINE_FP64 only: the FP64 Gram of the refinement,
                                   rounded once to FP32 (no separate FP32 Gram launch) */
  JACPCG_REFINE_FP64 = 0x100  /* rzf_precoder only: FP64-residual iterative refinement of X */
};

/* jacpcg_solve / rzf_precoder `flags` (bitwise or). */
enum {
  JACPCG_PRECOND_JACOBI = 0,  /* C = diag(A) (eq. 21) */
  JACPCG_PRECOND_NONE = 1,    /* C = I: plain CG, the method the paper compares against */
  JACPCG_EPILOGUE_FP32 = 0x10 /* rzf_precoder*: form W = beta H X with FP32 MFMA instead of the
                                 default split-BF16 products (three exact bf16 parts, six
                                 products, FP32 accumulation: FP32-class accuracy) */
};

/* Kernel phases timed when profiling is on (jacpcg_session_set_profiling). */
enum {
  JACPCG_PHASE_GRAM = 0,
  JACPCG_PHASE_SOLVE = 1,
  JACPCG_PHASE_EPILOGUE = 2,
  JACPCG_PHASE_GRAM64 = 3,
  JACPCG_PHASE_RESIDUAL = 4,
  JACPCG_NUM_PHASES = 5
};

/* ---- session ------------------------------------------------------------ */

/* Create a session on HIP device `device`. hbm_budget_bytes caps the device
 * memory the session may hold for workspaces and admitted requests (0 = no
 * cap). tune_cache_path (host, nullable) names a JSON file of autotuned kernel
 * choices, read at creation and rewritten when new shapes are tuned.
 * Errors: E_INVALID_ARG (out == NULL, device < 0), E_NO_DEVICE (no such HIP
 * device), E_HIP. On success *out owns device resources until destroy. */
int jacpcg_session_create(int device, size_t hbm_budget_bytes, const char* tune_cache_path,
                          jacpcg_session** out);

/* Wait for all work of the session, stop its scheduler and free everything it
 * allocated. NULL is ignored. */
void jacpcg_session_destroy(jacpcg_session* s);

/* Static description of a status code (never NULL). */
const char* jacpcg_status_string(int status);

/* Detail of the last failing call on the calling thread ("" if none). The
 * detail is kept per thread: s (nullable) names the session the caller is
 * asking about, and the text names the failure whichever session it was. */
const char* jacpcg_last_error(const jacpcg_session* s);

/* ABI version: major * 10000 + minor * 100 + patch. */
int jacpcg_version(void);

/* Turn per-phase kernel timing on (1) or off (0). When on, every kernel launch
 * is bracketed by HIP events recorded on the launch stream. */
int jacpcg_session_set_profiling(jacpcg_session* s, int enable);

/* Host arrays of JACPCG_NUM_PHASES: accumulated milliseconds and launch counts
 * of every timed kernel since the last reset (reset != 0 clears them).
 * Synchronises the session's pending events. */
int jacpcg_session_phase_times(jacpcg_session* s, double* ms_out, int64_t* launches_out, int reset);

/* Replay identical rzf_precoder calls (same arguments and buffers, the refined
 * path included; profiling off) from a captured HIP graph: 1 = on (default),
 * 0 = always launch kernel by kernel. Stats, when asked for, are read after
 * the replay. */
int jacpcg_session_set_graphs(jacpcg_session* s, int enable);

/* Autotune the launch choices for one shape: times every value of each knob
 * of jacpcg_tune_set that applies (Gram waves; where the solver keeps A for
 * K <= 64; precoder column tiles and antenna blocks) on `batch` synthetic
 * instances of M x K (device memory from the session workspace), each value
 * as the fastest of five launches, and keeps the fastest value. The fastest
 * choice can differ between batch sizes: pass the batch the calls will use.
 * The choices are saved to the session's tune cache file at destroy.
 * Synchronises `stream`. Choices depend only on the shape, never on the
 * batch, so results stay independent of batch composition. */
int jacpcg_autotune(jacpcg_session* s, void* stream, int batch, int M, int K, int precision, int flags);

/* Matrix-core peaks measured on the session's device: register-only loops of
 * independent MFMA chains (two waves per SIMD on every compute unit), timed
 * with HIP events on `stream`. tflops (host, 4 doubles) receives FP32
 * (32x32x2), BF16 (32x32x16), FP64 (16x16x4) TFLOP/s and int8 (32x32x32)
 * TOP/s. A calibration aid: it allocates a small output buffer and
 * synchronises `stream`. Errors: E_INVALID_ARG (NULL), E_HIP. */
int jacpcg_mfma_peaks(jacpcg_session* s, void* stream, double* tflops);

/* Read or pin one autotuned launch choice. knob names and their values:
 *   "gram_waves"      waves per Gram workgroup splitting the antennas: 2, 4, 8
 *                     (split-BF16 Gram: at most 4); key (M, K, Gram precision)
 *   "precoder_nj"     32-column tiles per precoder wave: 1, 2; key (M, K, split),
 *                     split = 3 for the default split-BF16 epilogue, 0 with
 *                     JACPCG_EPILOGUE_FP32
 *   "precoder_mtiles" antenna blocks per split-BF16 precoder workgroup: 1, 2, 4;
 *                     key (M, K, 3)
 *   "pcg_a_source"    where the solver keeps A and how it forms A P: 1 in
 *                     registers (K <= 64), 2 streamed from L2 with FP32
 *                     products, 3 streamed with split-BF16 products (three
 *                     bf16 parts of A and P, six part products: FP32-class,
 *                     the dropped part products at most ~2^-24 of the terms;
 *                     K > 64 without visibility-region spans, else as the
 *                     default); key (0, K, 0). Default: 1 up to K = 64, 3 above.
 * value 0 restores the kernel's default rule. Choices change the launch and
 * the order of the FP32 sums; the solver's products are FP32 or FP32-class
 * split-BF16 (pcg_a_source 3) and every choice stays within the FP32 bar of
 * the others. jacpcg_tune_set drops the session's captured graphs.
 * Errors: E_INVALID_ARG (NULL, unknown knob, value not a choice of the knob). */
int jacpcg_tune_set(jacpcg_session* s, const char* knob, int M, int K, int variant, int value);
int jacpcg_tune_get(jacpcg_session* s, const char* knob, int M, int K, int variant, int* value);

/* ---- the three steps ---------------------------------------------------- */

/* Regularised Gram (eq. 7): A_b = H_b^H H_b + xi I_K for b < batch.
 * H: column-major M x K (ldh >= M), A: row-major K x K (lda >= K), both
 * triangles written, diagonal exactly real. diag (nullable, batch x K floats,
 * contiguous per instance) receives Re diag(A) = ||h_k||^2 + xi, the Jacobi
 * preconditioner of eq. 21. precision: JACPCG_GRAM_FP32 / _BF16X3 / _BF16X6.
 * Errors: E_INVALID_ARG (NULL H/A, M < 1, K outside [1, 256], xi < 0 or not
 * finite, ldh < M, lda < K, strides too small), E_UNSUPPORTED (precision). */
int jacpcg_gram(jacpcg_session* s, void* stream, int batch, int M, int K,
                const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                float xi, int precision,
                jacpcg_c64* A, int64_t lda, int64_t stride_a,
                float* diag);

/* Jacobi-preconditioned CG (Algorithm 1 with the step length of Step 3, C =
 * diag(A) of eq. 21) on A_b X_b = B_b, every right-hand-side column solved
 * independently from x = 0.
 * A: row-major K x K Hermitian positive definite. B: column-major K x nrhs, or
 * NULL for B = I_K (requires nrhs == K). X: column-major K x nrhs output.
 * tol > 0: column j stops after the first iteration with
 *   ||r_j||_2 <= tol * ||b_j||_2 (recurrence residual; Step 2's rule made
 *   relative); tol == 0 runs exactly max_iter iterations (a column whose
 *   residual falls below 2^-40 ||b_j||, where an FP32 iterate no longer
 *   changes, stops early as converged). One iteration = one A p product.
 * flags: JACPCG_PRECOND_JACOBI (default) or JACPCG_PRECOND_NONE (plain CG).
 * iters (nullable, batch x nrhs int32): iterations done per column.
 * relres (nullable, batch x nrhs float): ||r_j|| / ||b_j|| at the stop.
 * status (nullable, batch int32): per instance OK, NOT_CONVERGED (tol > 0 and a
 *   column did not reach it) or E_BREAKDOWN (p^H A p < 0 or non-finite; that
 *   column keeps its last x). p^H A p = 0 means p = 0 for HPD A, i.e. the
 *   residual vanished: the column stops as converged. A zero column of B gives
 *   x = 0 after 0 iterations.
 * Errors: E_INVALID_ARG (NULL A/X, K or nrhs out of range, B NULL with
 * nrhs != K, tol < 0, max_iter < 0, leading dimensions or strides too small). */
int jacpcg_solve(jacpcg_session* s, void* stream, int batch, int K, int nrhs,
                 const jacpcg_c64* A, int64_t lda, int64_t stride_a,
                 const jacpcg_c64* B, int64_t ldb, int64_t stride_b,
                 jacpcg_c64* X, int64_t ldx, int64_t stride_x,
                 double tol, int max_iter, int flags,
                 int32_t* iters, float* relres, int32_t* status);

/* Per-call summary, filled on the host after the call synchronises. */
typedef struct {
  double max_rel_residual;   /* max over instances/columns of ||b - A x|| / ||b|| (recurrence, FP32) */
  double max_refine_residual;/* refined path: max over instances and columns j of the FP64
                                ||e_j - A64 x_j||_2 at exit, else 0 */
  int32_t max_iters;         /* max PCG iterations over all columns (first solve) */
  int32_t refine_steps;      /* refined path: most correction solves any column took */
  int32_t worst_status;      /* most severe per-instance status */
  int32_t reserved;
  double beta_pow_min, beta_pow_max;
} jacpcg_stats;

/* Whole path: A = H^H H + xi I (Gram in `precision`), X = A^{-1} B with B = I_K
 * by Jacobi-PCG (tol, max_iter as in jacpcg_solve), then W = beta_pow H X with
 * beta_pow = sqrt(power / ||H X||_F^2) per instance (eq. 7 and eq. 15).
 * W: column-major M x K per instance (precoding vector g_k contiguous).
 * precision | JACPCG_REFINE_FP64: iterative refinement of X in FP64 on the
 *   device. A64 = H^H H + xi I is formed in FP64 (FP64 matrix cores) for the
 *   residual only; the FP32 solves use the Gram of the precision bits
 *   (JACPCG_GRAM_FP32, _BF16X3 or _BF16X6), or A64 rounded once to FP32
 *   (JACPCG_GRAM_FP64_ROUNDED). After the first solve, each step computes
 *   R = I - A64 X64 in FP64, and every column j with ||r_j||_2 > refine_tol
 *   takes a correction: A E_j = r_j / ||r_j|| by FP32 Jacobi-PCG (tol,
 *   max_iter), X64 += ||r_j|| E_j. A column stops when ||r_j||_2 <= refine_tol;
 *   at most 16 corrections. The power factor comes from ||H X64||_F^2 in FP64
 *   and W from X64 rounded to FP32. An instance with a column still above
 *   refine_tol after 16 corrections reports NOT_CONVERGED.
 * Above K = 128, and above K = 64 when the batch has fewer than 512 64 x 64
 *   blocks of A (without visibility-region spans), the FP32 Gram and the FP64
 *   Gram of this call sum the antennas in four chunks, added in a fixed order
 *   (session workspace: 4 partial 64 x 64 blocks per block of A); the FP32 A
 *   can then differ from jacpcg_gram's in the last bits. Above K = 64 with
 *   512 or more blocks the FP64 Gram sums two chunks.
 * X_out (nullable): column-major K x K c64 copy of X per instance (ld K,
 *   stride K*K). X64_out (nullable): the same in c128 (the refined X64; the
 *   FP32 solution widened otherwise). flags: as jacpcg_solve.
 * stats (host, nullable): when given, the call synchronises `stream` and fills
 *   it. Without stats no path synchronises (the refined path included).
 * Returns the worst per-instance status when it synchronises, else OK.
 * Non-finite values in an instance's H make its A non-finite: that instance
 *   ends with E_BREAKDOWN within max_iter and its W and X are unspecified; the
 *   other instances are computed exactly as without it (on the refined path
 *   they still stop on their own residuals).
 * Errors: as jacpcg_gram and jacpcg_solve; power <= 0; refine_tol < 0;
 *   E_UNSUPPORTED for JACPCG_GRAM_FP64_ROUNDED without JACPCG_REFINE_FP64. */
int rzf_precoder(jacpcg_session* s, void* stream, int batch, int M, int K,
                 const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                 double xi, double power, double tol, int max_iter, int precision, int flags,
                 double refine_tol,
                 jacpcg_c64* W, int64_t ldw, int64_t stride_w,
                 jacpcg_c64* X_out, jacpcg_c128* X64_out, jacpcg_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): rzf_precoder
 * without refinement, stats, X_out or X64_out, whose workspace (A, diag(H^H H),
 * X, the solver's per-workgroup partials) lives in a fixed device array of the
 * library instead of the session's arena. The call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine, and it records no event.
 * The array holds 96 MiB on each device the library runs on, from the first
 * session on that device until the process ends; a batch needs
 *   2 * batch * K * K * 8 + batch * K * 4 + 2 * batch * ceil(K/32) * 4 bytes
 * (each of the five buffers rounded up to 256 bytes): up to 1529 instances
 * at K = 64, 383 at K = 128, 95 at K = 256.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (other streams, other
 * sessions, other threads) race and give undefined results; the caller orders
 * them. Nothing in the array needs to start at zero.
 * status (device, nullable): batch int32, the per-instance status of
 * jacpcg_solve (OK / NOT_CONVERGED / E_BREAKDOWN).
 * Asynchronous on `stream`; outputs valid after it is synchronised.
 * Every other argument as rzf_precoder.
 * Errors: as rzf_precoder; E_INVALID_ARG when the batch does not fit the
 * array (the message gives both sizes); E_UNSUPPORTED for JACPCG_REFINE_FP64;
 * E_HIP if the array's device address could not be looked up. */
int rzf_precoder_noalloc(jacpcg_session* s, void* stream, int batch, int M, int K,
                         const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                         double xi, double power, double tol, int max_iter, int precision, int flags,
                         jacpcg_c64* W, int64_t ldw, int64_t stride_w, int32_t* status);

/* The same result computed the plain way, one instance at a time: per instance
 * one Gram launch, one launch per PCG iteration (with a host-side convergence
 * check after each when tol > 0), then the precoder launch. The baseline the
 * batched path is measured against. FP32 Gram only, no refinement. */
int rzf_precoder_plain(jacpcg_session* s, void* stream, int batch, int M, int K,
                       const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                       double xi, double power, double tol, int max_iter, int flags,
                       jacpcg_c64* W, int64_t ldw, int64_t stride_w,
                       jacpcg_c64* X_out, jacpcg_stats* stats);

/* rzf_precoder exploiting visibility-region sparsity (Sec. II, eq. 4; the
 * sparsity of P_i noted in Sec. III): user k's channel is zero outside the
 * antenna span [user_span[2k], user_span[2k+1]) of its visibility region, so
 * A_ij = 0 when the spans of users i and j do not overlap. Per 32-user block
 * the hull of its users' spans is formed; each Gram tile contracts only the
 * antennas where its two blocks overlap, and the solver skips the tiles of A
 * whose blocks do not overlap (exact zeros). With JACPCG_REFINE_FP64 the FP64
 * Gram contracts each 64 x 64 block over its blocks' overlap too, and the
 * FP64 residual skips the user blocks a row block does not meet. The skipped
 * terms are exact zeros, so the result is rzf_precoder's up to the summation
 * order.
 * Effective for K > 64 (smaller K runs the dense kernels); most effective
 * with users ordered by the position of their region (A then has a band of
 * nonzero tiles).
 * user_span: device int32, batch x K x 2 (first, end) per user, or NULL to
 *   find each user's first and last nonzero antenna on the device (one read of
 *   H). Channel entries outside a given span are treated as zero.
 * Every other argument as rzf_precoder (X64_out not available). */
int rzf_precoder_vr(jacpcg_session* s, void* stream, int batch, int M, int K,
                    const jacpcg_c64* H, int64_t ldh, int64_t stride_h, const int32_t* user_span,
                    double xi, double power, double tol, int max_iter, int precision, int flags,
                    double refine_tol, jacpcg_c64* W, int64_t ldw, int64_t stride_w,
                    jacpcg_c64* X_out, jacpcg_stats* stats);

/* Per-symbol transmission (eqs. 15-16): for each instance and each of its
 * nsym symbol vectors s (K x 1), w = A^{-1} s by Jacobi-PCG (or plain CG with
 * JACPCG_PRECOND_NONE) on A = H^H H + xi I, and the transmitted vector
 * x = beta_pow H w, with one power factor per instance over its block of
 * symbols: beta_pow = sqrt(power / ||H W||_F^2), W = [w_1 .. w_nsym], so the
 * block carries total power `power` (with S = I_K this is rzf_precoder's W;
 * pass power = nsym * P for an average of P per symbol vector).
 * S: device, column-major K x nsym c64 per instance (ld lds >= K, stride
 *   stride_s >= lds * nsym). x: device output, column-major M x nsym per
 *   instance (ld ldx >= M, stride stride_x >= ldx * nsym). w_out (nullable):
 *   the solutions, column-major K x nsym (ld K, stride K * nsym).
 * precision: JACPCG_GRAM_* only (no refinement: E_UNSUPPORTED); tol, max_iter,
 *   flags and stats as rzf_precoder (per-column iteration counts over the
 *   nsym columns). Errors: as rzf_precoder; nsym < 1; NULL S or x. */
int rzf_transmit(jacpcg_session* s, void* stream, int batch, int M, int K, int nsym,
                 const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                 const jacpcg_c64* S, int64_t lds, int64_t stride_s,
                 double xi, double power, double tol, int max_iter, int precision, int flags,
                 jacpcg_c64* x, int64_t ldx, int64_t stride_x,
                 jacpcg_c64* w_out, jacpcg_stats* stats);

/* Subarray-block RZF (Sec. II, eqs. 2, 6 and 7): three subarrays of M1, Mc
 * and M2 antennas (rows [0, M1), [M1, M1+Mc), [M1+Mc, M)), two user groups of
 * K1 and K2 users (columns [0, K1), [K1, K)); group 1 sees subarrays 1 and c,
 * group 2 sees c and 2, so H has the block form of eq. 2 (the caller's other
 * blocks are never read). Each block is its own RZF problem with its own
 * power factor (eq. 7): G_1 = beta_1 H_1 P_1^{-1} (M1 x K1), G_c =
 * beta_c H_c P_c^{-1} (Mc x K), G_2 = beta_2 H_2 P_2^{-1} (M2 x K2), each of
 * total power `power`; the other two blocks of G are written as zeros (eq. 6).
 * H, G: device, column-major M x K c64 per instance (ld ldh / ldg >= M,
 * strides >= ld * K). Blocks with no rows or no users are skipped.
 * Every other argument as rzf_precoder; stats (when given) combine the three
 * solves (maxima, worst status). Runs as three batched precoder solves on
 * `stream`. Errors: as rzf_precoder; negative sizes; K > 256. */
int rzf_block_precoder(jacpcg_session* s, void* stream, int batch, int M1, int Mc, int M2, int K1, int K2,
                       const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
                       double xi, double power, double tol, int max_iter, int precision, int flags,
                       double refine_tol, jacpcg_c64* G, int64_t ldg, int64_t stride_g,
                       jacpcg_stats* stats);

/* Evaluation of a precoder on its channel (Sec. II, eqs. 8-10): per user k,
 *   SINR_k = |h_k^H g_k|^2 / (sum_{j != k} |h_k^H g_j|^2 + sigma2),
 * and per instance the sum spectral efficiency SE = sum_k log2(1 + SINR_k)
 * (bit/s/Hz), with g_j column j of W. C = H^H W is formed on the FP32 matrix
 * cores (session workspace, K x K per instance); every sum has a fixed order.
 * H, W: device, column-major M x K c64 per instance (as rzf_precoder).
 * sinr (device, nullable): batch x K floats. se (device, nullable): batch
 * floats; at least one of them. Asynchronous on `stream`.
 * Errors: as jacpcg_gram (K <= 256); sigma2 < 0 or non-finite; bad ldw /
 * stride_w; NULL W; both outputs NULL. */
int rzf_sinr(jacpcg_session* s, void* stream, int batch, int M, int K,
             const jacpcg_c64* H, int64_t ldh, int64_t stride_h,
             const jacpcg_c64* W, int64_t ldw, int64_t stride_w,
             double sigma2, float* sinr, float* se);

/* ---- request API: continuous batching ---------------------------------- */

/* One precoder request: n_sub subcarrier instances of one (M, K) shape, each
 * solved as rzf_precoder would (B = I_K; Gram precision JACPCG_GRAM_*, no
 * refinement; flags JACPCG_PRECOND_* | JACPCG_EPILOGUE_FP32).
 * H: device, n_sub instances of column-major M x K complex64 (ld M, stride
 * M*K). W: device output of the same layout. Both buffers are owned by the
 * caller and must stay alive until jacpcg_poll / jacpcg_wait returns a final
 * result for the request.
 * stream: the stream on which the caller writes H (NULL: the default stream).
 * jacpcg_submit records an event on it, and the request's device work waits
 * for that event: H may still be in production when the request is
 * submitted, and work queued on `stream` after the submission is not waited
 * for. W is complete when the result is final. */
typedef struct {
  int M, K, n_sub;
  const jacpcg_c64* H;
  jacpcg_c64* W;
  double xi, power, tol;
  int max_iter, precision, flags;
  uint64_t user_tag;
  void* stream; /* hipStream_t */
} jacpcg_request;

/* Result of a request. status: the request's worst per-instance status (OK,
 * NOT_CONVERGED, E_BREAKDOWN), E_CANCELLED, E_HIP, or NOT_READY while in flight.
 * Times are microseconds of the session clock (jacpcg_session_clock_us):
 * submission, admission (launch of its batch) and completion as observed by
 * the session. */
typedef struct {
  int status;
  int32_t max_iters;
  double t_submit_us, t_admit_us, t_done_us;
  uint64_t user_tag;
} jacpcg_result;

/* Queue a request; returns a ticket. The session's scheduler admits requests
 * in FIFO order while its HBM budget (H + W + workspace of the admitted
 * requests) and in-flight batch slots allow, batches admitted requests of the
 * same shape and settings into one launch, and runs batches of different slots
 * concurrently. There is one slot per hardware queue of the process
 * (GPU_MAX_HW_QUEUES, 4 by default, at most 8), each with its own stream. A
 * request's result does not depend on what it is batched with.
 * Errors: E_INVALID_ARG (sizes, NULL buffers, xi < 0, power <= 0, tol < 0,
 * max_iter < 0, unknown flags), E_UNSUPPORTED (refinement requested),
 * E_BUDGET (the request alone needs more than the session budget), E_HIP (the
 * event on the request's stream could not be recorded). */
int jacpcg_submit(jacpcg_session* s, const jacpcg_request* r, uint64_t* ticket);

/* Non-blocking: NOT_READY while the request is queued or running; OK once final
 * (the result is then in *out and the ticket is released). E_INVALID_ARG for an
 * unknown or already collected ticket. */
int jacpcg_poll(jacpcg_session* s, uint64_t ticket, jacpcg_result* out);

/* Block until the request is final (timeout_ms < 0: no limit). OK with the
 * result in *out (ticket released), or E_TIMEOUT (ticket kept). */
int jacpcg_wait(jacpcg_session* s, uint64_t ticket, int timeout_ms, jacpcg_result* out);

/* Cancel: a queued request is removed and completes with E_CANCELLED; a
 * running one still finishes on the device (W may be written) and reports
 * E_CANCELLED. A completed request is unaffected. */
int jacpcg_cancel(jacpcg_session* s, uint64_t ticket);

/* Microseconds since the session was created (steady clock); the clock of the
 * request timestamps. */
double jacpcg_session_clock_us(jacpcg_session* s);

#ifdef __cplusplus
}
#endif

#endif /* JACPCG_H */
