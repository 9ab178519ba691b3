// C ABI of libjacpcg: argument validation, sessions and workspaces, and the
// composition of the Gram, PCG and precoder kernels into the whole path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jacpcg.h"
#include "common.hpp"
#include "session.hpp"

using namespace jacpcg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define JP_CHECK(cond, ...)                               \
  do {                                                    \
    if (!(cond)) return fail(JACPCG_E_INVALID_ARG, __VA_ARGS__); \
  } while (0)

#define JP_HIP(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail(JACPCG_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int worse(int a, int b) {
  auto sev = [](int s) { return s == kStatusBreakdown ? 2 : (s == kStatusNotConverged ? 1 : 0); };
  return sev(b) > sev(a) ? b : a;
}

// ---- shared argument checks ------------------------------------------------
int check_gram_args(int batch, int M, int K, const void* H, int64_t ldh, int64_t stride_h, double xi,
                    const void* A, int64_t lda, int64_t stride_a) {
  JP_CHECK(batch >= 0, "batch must be >= 0 (got %d)", batch);
  JP_CHECK(M >= 1, "M must be >= 1 (got %d)", M);
  JP_CHECK(K >= 1 && K <= kMaxK, "K must be in [1, %d] (got %d)", kMaxK, K);
  JP_CHECK(std::isfinite(xi) && xi >= 0.0, "xi must be finite and >= 0 (got %g)", xi);
  JP_CHECK(ldh >= M, "ldh must be >= M (got %lld < %d)", (long long)ldh, M);
  if (batch > 1) JP_CHECK(stride_h >= ldh * K, "stride_h must be >= ldh * K");
  if (batch > 0) JP_CHECK(H != nullptr, "H is NULL");
  if (A || lda) {
    JP_CHECK(lda >= K, "lda must be >= K (got %lld < %d)", (long long)lda, K);
    if (batch > 1) JP_CHECK(stride_a >= lda * K, "stride_a must be >= lda * K");
  }
  return JACPCG_OK;
}

int check_solve_args(int batch, int K, int nrhs, const void* A, int64_t lda, int64_t stride_a, const void* B,
                     int64_t ldb, int64_t stride_b, const void* X, int64_t ldx, int64_t stride_x, double tol,
                     int max_iter, int flags) {
  JP_CHECK(batch >= 0, "batch must be >= 0 (got %d)", batch);
  JP_CHECK(K >= 1 && K <= kMaxK, "K must be in [1, %d] (got %d)", kMaxK, K);
  JP_CHECK(nrhs >= 1 && nrhs <= kMaxNrhs, "nrhs must be in [1, %d] (got %d)", kMaxNrhs, nrhs);
  JP_CHECK(B != nullptr || nrhs == K, "B == NULL (identity) requires nrhs == K (got nrhs %d, K %d)", nrhs, K);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK(flags == JACPCG_PRECOND_JACOBI || flags == JACPCG_PRECOND_NONE, "unknown flags 0x%x", flags);
  JP_CHECK(lda >= K, "lda must be >= K");
  JP_CHECK(ldx >= K, "ldx must be >= K");
  if (B) JP_CHECK(ldb >= K, "ldb must be >= K");
  if (batch > 1) {
    JP_CHECK(stride_a >= lda * K, "stride_a must be >= lda * K");
    JP_CHECK(stride_x >= ldx * nrhs, "stride_x must be >= ldx * nrhs");
    if (B) JP_CHECK(stride_b >= ldb * nrhs, "stride_b must be >= ldb * nrhs");
  }
  if (batch > 0) {
    JP_CHECK(A != nullptr, "A is NULL");
    JP_CHECK(X != nullptr, "X is NULL");
  }
  return JACPCG_OK;
}

int check_session(jacpcg_session* s) {
  JP_CHECK(s != nullptr, "session is NULL");
  if (s->poisoned) return fail(JACPCG_E_HIP, "session poisoned by an earlier HIP error; recreate it");
  return JACPCG_OK;
}

int hip_fail(jacpcg_session* s, hipError_t e, const char* what) {
  if (s) s->poisoned = true;
  return fail(JACPCG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void fill_stats(jacpcg_stats* st, int batch, int K, const int32_t* iters, const float* relres,
                const int32_t* status, const float* beta) {
  std::memset(st, 0, sizeof *st);
  st->beta_pow_min = batch ? 1e300 : 0.0;
  st->beta_pow_max = 0.0;
  for (int b = 0; b < batch; ++b) {
    st->worst_status = worse(st->worst_status, status[b]);
    for (int j = 0; j < K; ++j) {
      st->max_iters = std::max(st->max_iters, iters[(size_t)b * K + j]);
      st->max_rel_residual = std::max(st->max_rel_residual, (double)relres[(size_t)b * K + j]);
    }
    if (beta) {
      st->beta_pow_min = std::min(st->beta_pow_min, (double)beta[b]);
      st->beta_pow_max = std::max(st->beta_pow_max, (double)beta[b]);
    }
  }
}

}  // namespace

// ============================================================================
extern "C" {

int jacpcg_version(void) { return 10000; }

const char* jacpcg_last_error(const jacpcg_session*) { return g_last_error.c_str(); }

const char* jacpcg_status_string(int status) {
  switch (status) {
    case JACPCG_OK: return "ok";
    case JACPCG_NOT_CONVERGED: return "not converged within max_iter";
    case JACPCG_NOT_READY: return "not ready";
    case JACPCG_E_INVALID_ARG: return "invalid argument";
    case JACPCG_E_UNSUPPORTED: return "unsupported";
    case JACPCG_E_NO_DEVICE: return "no such HIP device";
    case JACPCG_E_OUT_OF_MEMORY: return "out of device memory or over the session budget";
    case JACPCG_E_BREAKDOWN: return "PCG breakdown (p^H A p < 0 or non-finite)";
    case JACPCG_E_HIP: return "HIP runtime error";
    case JACPCG_E_BUDGET: return "request can never fit the HBM budget";
    case JACPCG_E_CANCELLED: return "cancelled";
    case JACPCG_E_TIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

int jacpcg_session_create(int device, size_t hbm_budget_bytes, const char* tune_cache_path, jacpcg_session** out) {
  JP_CHECK(out != nullptr, "out is NULL");
  *out = nullptr;
  JP_CHECK(device >= 0, "device must be >= 0 (got %d)", device);
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(JACPCG_E_NO_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  if (device >= n) return fail(JACPCG_E_NO_DEVICE, "device %d out of range (%d devices)", device, n);
  JP_HIP(hipSetDevice(device));
  auto* s = new jacpcg_session();
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (tune_cache_path) s->tune_path = tune_cache_path;
  s->tuner.load(s->tune_path);
  // Device address of the fixed scratch array of rzf_precoder_noalloc; a
  // failure is reported by that entry point, not here.
  (void)noalloc_setup(device);
  *out = s;
  return JACPCG_OK;
}

void jacpcg_session_destroy(jacpcg_session* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  s->shutdown();
  delete s;
}

int jacpcg_session_set_profiling(jacpcg_session* s, int enable) {
  int rc = check_session(s);
  if (rc) return rc;
  s->profiling = enable != 0;
  return JACPCG_OK;
}

int jacpcg_session_phase_times(jacpcg_session* s, double* ms_out, int64_t* launches_out, int reset) {
  int rc = check_session(s);
  if (rc) return rc;
  JP_CHECK(ms_out != nullptr, "ms_out is NULL");
  hipError_t e = s->collect_events();
  if (e != hipSuccess) return hip_fail(s, e, "collecting phase events");
  for (int i = 0; i < JACPCG_NUM_PHASES; ++i) {
    ms_out[i] = s->phase_ms[i];
    if (launches_out) launches_out[i] = s->phase_count[i];
    if (reset) {
      s->phase_ms[i] = 0.0;
      s->phase_count[i] = 0;
    }
  }
  return JACPCG_OK;
}

int jacpcg_gram(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H, int64_t ldh,
                int64_t stride_h, float xi, int precision, jacpcg_c64* A, int64_t lda, int64_t stride_a,
                float* diag) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, A, lda, stride_a);
  if (rc) return rc;
  if (batch > 0) JP_CHECK(A != nullptr, "A is NULL");
  if (precision < 0 || precision > 2) return fail(JACPCG_E_UNSUPPORTED, "unknown Gram precision %d", precision);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) return JACPCG_OK;
  JP_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  GramLaunch g{};
  g.H = (const float2*)H;
  g.ldh = ldh;
  g.stride_h = stride_h;
  g.batch = batch;
  g.M = M;
  g.K = K;
  g.xi = xi;
  g.A = (float2*)A;
  g.lda = lda;
  g.stride_a = stride_a;
  g.diag = diag;
  g.gdiag = nullptr;
  g.precision = precision;
  g.m_split = s->tuner.gram_waves(M, K, precision);
  hipError_t e = s->timed(st, JACPCG_PHASE_GRAM, [&] { return launch_gram(g, st); });
  if (e == hipErrorNotSupported) return fail(JACPCG_E_UNSUPPORTED, "Gram precision %d not available", precision);
  if (e != hipSuccess) return hip_fail(s, e, "gram launch");
  return JACPCG_OK;
}

int jacpcg_solve(jacpcg_session* s, void* stream, int batch, int K, int nrhs, const jacpcg_c64* A, int64_t lda,
                 int64_t stride_a, const jacpcg_c64* B, int64_t ldb, int64_t stride_b, jacpcg_c64* X, int64_t ldx,
                 int64_t stride_x, double tol, int max_iter, int flags, int32_t* iters, float* relres,
                 int32_t* status) {
  int rc = check_solve_args(batch, K, nrhs, A, lda, stride_a, B, ldb, stride_b, X, ldx, stride_x, tol, max_iter,
                            flags);
  if (rc) return rc;
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) return JACPCG_OK;
  JP_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  const int ncb = (nrhs + 31) / 32;
  Workspace ws;
  const size_t o_wg = ws.take<int32_t>((size_t)batch * ncb);
  rc = s->reserve(ws);
  if (rc) return rc;
  PcgLaunch p{};
  p.A = (const float2*)A;
  p.lda = lda;
  p.stride_a = stride_a;
  p.B = (const float2*)B;
  p.ldb = ldb;
  p.stride_b = stride_b;
  p.X = (float2*)X;
  p.ldx = ldx;
  p.stride_x = stride_x;
  p.batch = batch;
  p.K = K;
  p.nrhs = nrhs;
  p.tol = (float)tol;
  p.max_iter = max_iter;
  p.precond_none = flags == JACPCG_PRECOND_NONE;
  p.iters = iters;
  p.relres = relres;
  p.wg_status = status ? s->at<int32_t>(o_wg) : nullptr;
  return s->ordered(st, [&] {
    hipError_t e = s->timed(st, JACPCG_PHASE_SOLVE, [&] { return launch_pcg(p, st, nullptr); });
    if (e != hipSuccess) return hip_fail(s, e, "pcg launch");
    if (status) {
      e = launch_status_reduce(p.wg_status, ncb, batch, status, st);
      if (e != hipSuccess) return hip_fail(s, e, "status reduce launch");
    }
    return (int)JACPCG_OK;
  });
}

int rzf_precoder(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H, int64_t ldh,
                 int64_t stride_h, double xi, double power, double tol, int max_iter, int precision, int flags,
                 double refine_tol, jacpcg_c64* W, int64_t ldw, int64_t stride_w, jacpcg_c64* X_out,
                 jacpcg_c128* X64_out, jacpcg_stats* stats) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(std::isfinite(refine_tol) && refine_tol >= 0.0, "refine_tol must be finite and >= 0");
  JP_CHECK(ldw >= M, "ldw must be >= M (got %lld < %d)", (long long)ldw, M);
  if (batch > 1) JP_CHECK(stride_w >= ldw * K, "stride_w must be >= ldw * K");
  if (batch > 0) JP_CHECK(W != nullptr, "W is NULL");
  const int gram_prec = precision & 0xff;
  const bool refine = (precision & JACPCG_REFINE_FP64) != 0;
  if (gram_prec > 3 || (gram_prec == JACPCG_GRAM_FP64_ROUNDED && !refine) ||
      (precision & ~(0xff | JACPCG_REFINE_FP64)))
    return fail(JACPCG_E_UNSUPPORTED, "unknown precision 0x%x", precision);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return JACPCG_OK;
  }
  JP_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  return s->ordered(st, [&] {
    return s->run_rzf(st, batch, M, K, (const float2*)H, ldh, stride_h, K, nullptr, 0, 0, xi, power, tol, max_iter,
                      gram_prec, refine, (flags & JACPCG_PRECOND_NONE) != 0, (flags & JACPCG_EPILOGUE_FP32) == 0,
                      refine_tol, (float2*)W, ldw, stride_w, (float2*)X_out, (double2*)X64_out, stats);
  });
}

int rzf_precoder_noalloc(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H,
                         int64_t ldh, int64_t stride_h, double xi, double power, double tol, int max_iter,
                         int precision, int flags, jacpcg_c64* W, int64_t ldw, int64_t stride_w, int32_t* status) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(ldw >= M, "ldw must be >= M (got %lld < %d)", (long long)ldw, M);
  if (batch > 1) JP_CHECK(stride_w >= ldw * K, "stride_w must be >= ldw * K");
  if (batch > 0) JP_CHECK(W != nullptr, "W is NULL");
  if (precision & JACPCG_REFINE_FP64) return fail(JACPCG_E_UNSUPPORTED, "no refinement without allocation");
  if (precision < 0 || precision > 2) return fail(JACPCG_E_UNSUPPORTED, "unknown precision 0x%x", precision);
  const size_t need = noalloc_need(batch, K), cap = noalloc_scratch_bytes();
  JP_CHECK(need <= cap, "batch of %d instances at K = %d needs %zu bytes of scratch, more than its fixed %zu",
           batch, K, need, cap);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) return JACPCG_OK;
  JP_HIP(hipSetDevice(s->device));
  return run_rzf_noalloc(s, (hipStream_t)stream, batch, M, K, (const float2*)H, ldh, stride_h, xi, power, tol,
                         max_iter, precision, (flags & JACPCG_PRECOND_NONE) != 0,
                         (flags & JACPCG_EPILOGUE_FP32) == 0, (float2*)W, ldw, stride_w, status);
}

int rzf_precoder_vr(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H, int64_t ldh,
                    int64_t stride_h, const int32_t* user_span, double xi, double power, double tol, int max_iter,
                    int precision, int flags, double refine_tol, jacpcg_c64* W, int64_t ldw, int64_t stride_w,
                    jacpcg_c64* X_out, jacpcg_stats* stats) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(std::isfinite(refine_tol) && refine_tol >= 0.0, "refine_tol must be finite and >= 0");
  JP_CHECK(ldw >= M, "ldw must be >= M (got %lld < %d)", (long long)ldw, M);
  if (batch > 1) JP_CHECK(stride_w >= ldw * K, "stride_w must be >= ldw * K");
  if (batch > 0) JP_CHECK(W != nullptr, "W is NULL");
  const int gram_prec = precision & 0xff;
  const bool refine = (precision & JACPCG_REFINE_FP64) != 0;
  if (gram_prec > 3 || (gram_prec == JACPCG_GRAM_FP64_ROUNDED && !refine) ||
      (precision & ~(0xff | JACPCG_REFINE_FP64)))
    return fail(JACPCG_E_UNSUPPORTED, "unknown precision 0x%x", precision);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return JACPCG_OK;
  }
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->run_rzf((hipStream_t)stream, batch, M, K, (const float2*)H, ldh, stride_h, K, nullptr, 0, 0, xi, power,
                      tol, max_iter, gram_prec, refine, (flags & JACPCG_PRECOND_NONE) != 0,
                      (flags & JACPCG_EPILOGUE_FP32) == 0, refine_tol, (float2*)W, ldw, stride_w, (float2*)X_out,
                      nullptr, stats, true, user_span);
  });
}

int rzf_transmit(jacpcg_session* s, void* stream, int batch, int M, int K, int nsym, const jacpcg_c64* H,
                 int64_t ldh, int64_t stride_h, const jacpcg_c64* S, int64_t lds, int64_t stride_s, double xi,
                 double power, double tol, int max_iter, int precision, int flags, jacpcg_c64* x, int64_t ldx,
                 int64_t stride_x, jacpcg_c64* w_out, jacpcg_stats* stats) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(nsym >= 1, "nsym must be >= 1 (got %d)", nsym);
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(lds >= K, "lds must be >= K (got %lld < %d)", (long long)lds, K);
  if (batch > 1) JP_CHECK(stride_s >= lds * nsym, "stride_s must be >= lds * nsym");
  JP_CHECK(ldx >= M, "ldx must be >= M (got %lld < %d)", (long long)ldx, M);
  if (batch > 1) JP_CHECK(stride_x >= ldx * nsym, "stride_x must be >= ldx * nsym");
  if (batch > 0) {
    JP_CHECK(S != nullptr, "S is NULL");
    JP_CHECK(x != nullptr, "x is NULL");
  }
  if ((precision & ~0xff) != 0)
    return fail(JACPCG_E_UNSUPPORTED, "rzf_transmit takes an FP32 or split-BF16 Gram, no refinement (0x%x)",
                precision);
  if ((precision & 0xff) > 2) return fail(JACPCG_E_UNSUPPORTED, "unknown precision 0x%x", precision);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return JACPCG_OK;
  }
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->run_rzf((hipStream_t)stream, batch, M, K, (const float2*)H, ldh, stride_h, nsym, (const float2*)S, lds,
                      stride_s, xi, power, tol, max_iter, precision & 0xff, false, (flags & JACPCG_PRECOND_NONE) != 0,
                      (flags & JACPCG_EPILOGUE_FP32) == 0, 0.0, (float2*)x, ldx, stride_x, (float2*)w_out, nullptr,
                      stats);
  });
}

int rzf_precoder_plain(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H, int64_t ldh,
                       int64_t stride_h, double xi, double power, double tol, int max_iter, int flags,
                       jacpcg_c64* W, int64_t ldw, int64_t stride_w, jacpcg_c64* X_out, jacpcg_stats* stats) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(ldw >= M, "ldw must be >= M (got %lld < %d)", (long long)ldw, M);
  if (batch > 1) JP_CHECK(stride_w >= ldw * K, "stride_w must be >= ldw * K");
  if (batch > 0) JP_CHECK(W != nullptr, "W is NULL");
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return JACPCG_OK;
  }
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->run_rzf_plain((hipStream_t)stream, batch, M, K, (const float2*)H, ldh, stride_h, xi, power, tol, max_iter,
                            (flags & JACPCG_PRECOND_NONE) != 0, (flags & JACPCG_EPILOGUE_FP32) == 0, (float2*)W, ldw,
                            stride_w, (float2*)X_out, stats);
  });
}

int rzf_block_precoder(jacpcg_session* s, void* stream, int batch, int M1, int Mc, int M2, int K1, int K2,
                       const jacpcg_c64* H, int64_t ldh, int64_t stride_h, double xi, double power, double tol,
                       int max_iter, int precision, int flags, double refine_tol, jacpcg_c64* G, int64_t ldg,
                       int64_t stride_g, jacpcg_stats* stats) {
  JP_CHECK(M1 >= 0 && Mc >= 0 && M2 >= 0, "subarray sizes must be >= 0 (got %d, %d, %d)", M1, Mc, M2);
  JP_CHECK(K1 >= 0 && K2 >= 0, "group sizes must be >= 0 (got %d, %d)", K1, K2);
  const int M = M1 + Mc + M2, K = K1 + K2;
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, xi, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(power) && power > 0.0, "power must be finite and > 0 (got %g)", power);
  JP_CHECK(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0 (got %g)", tol);
  JP_CHECK(max_iter >= 0, "max_iter must be >= 0 (got %d)", max_iter);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  JP_CHECK(std::isfinite(refine_tol) && refine_tol >= 0.0, "refine_tol must be finite and >= 0");
  JP_CHECK(ldg >= M, "ldg must be >= M1 + Mc + M2 (got %lld < %d)", (long long)ldg, M);
  if (batch > 1) JP_CHECK(stride_g >= ldg * K, "stride_g must be >= ldg * (K1 + K2)");
  if (batch > 0) JP_CHECK(G != nullptr, "G is NULL");
  const int gram_prec = precision & 0xff;
  const bool refine = (precision & JACPCG_REFINE_FP64) != 0;
  if (gram_prec > 3 || (gram_prec == JACPCG_GRAM_FP64_ROUNDED && !refine) ||
      (precision & ~(0xff | JACPCG_REFINE_FP64)))
    return fail(JACPCG_E_UNSUPPORTED, "unknown precision 0x%x", precision);
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return JACPCG_OK;
  }
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->run_block((hipStream_t)stream, batch, M1, Mc, M2, K1, K2, (const float2*)H, ldh, stride_h, xi, power, tol,
                        max_iter, gram_prec, refine, (flags & JACPCG_PRECOND_NONE) != 0,
                        (flags & JACPCG_EPILOGUE_FP32) == 0, refine_tol, (float2*)G, ldg, stride_g, stats);
  });
}

int rzf_sinr(jacpcg_session* s, void* stream, int batch, int M, int K, const jacpcg_c64* H, int64_t ldh,
             int64_t stride_h, const jacpcg_c64* W, int64_t ldw, int64_t stride_w, double sigma2, float* sinr,
             float* se) {
  int rc = check_gram_args(batch, M, K, H, ldh, stride_h, 0.0, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(std::isfinite(sigma2) && sigma2 >= 0.0, "sigma2 must be finite and >= 0 (got %g)", sigma2);
  JP_CHECK(ldw >= M, "ldw must be >= M (got %lld < %d)", (long long)ldw, M);
  if (batch > 1) JP_CHECK(stride_w >= ldw * K, "stride_w must be >= ldw * K");
  if (batch > 0) {
    JP_CHECK(W != nullptr, "W is NULL");
    JP_CHECK(sinr != nullptr || se != nullptr, "sinr and se are both NULL");
  }
  rc = check_session(s);
  if (rc) return rc;
  if (batch == 0) return JACPCG_OK;
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->run_sinr((hipStream_t)stream, batch, M, K, (const float2*)H, ldh, stride_h, (const float2*)W, ldw,
                       stride_w, sigma2, sinr, se);
  });
}

int jacpcg_session_set_graphs(jacpcg_session* s, int enable) {
  int rc = check_session(s);
  if (rc) return rc;
  s->use_graphs = enable != 0;
  if (!s->use_graphs) s->graph_clear();
  return JACPCG_OK;
}

int jacpcg_autotune(jacpcg_session* s, void* stream, int batch, int M, int K, int precision, int flags) {
  int rc = check_gram_args(batch, M, K, (const void*)1, M, (int64_t)M * K, 1.0, nullptr, 0, 0);
  if (rc) return rc;
  JP_CHECK(batch >= 1, "batch must be >= 1");
  if (precision < 0 || precision > 2) return fail(JACPCG_E_UNSUPPORTED, "unknown Gram precision %d", precision);
  JP_CHECK((flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) == 0, "unknown flags 0x%x", flags);
  rc = check_session(s);
  if (rc) return rc;
  JP_HIP(hipSetDevice(s->device));
  return s->ordered((hipStream_t)stream, [&] {
    return s->autotune((hipStream_t)stream, batch, M, K, precision, flags);
  });
}

double jacpcg_session_clock_us(jacpcg_session* s) {
  if (!s) return 0.0;
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - s->t0).count();
}

int jacpcg_tune_set(jacpcg_session* s, const char* knob, int M, int K, int variant, int value) {
  JP_CHECK(knob != nullptr, "knob is NULL");
  const int k = Tuner::knob_of(knob);
  JP_CHECK(k >= 0, "unknown knob '%s'", knob);
  JP_CHECK(Tuner::valid(k, value), "value %d is not a choice of knob '%s'", value, knob);
  int rc = check_session(s);
  if (rc) return rc;
  s->tuner.set(k, M, K, variant, value);
  s->graph_clear();  // captured graphs hold the previous choices
  return JACPCG_OK;
}

int jacpcg_tune_get(jacpcg_session* s, const char* knob, int M, int K, int variant, int* value) {
  JP_CHECK(knob != nullptr && value != nullptr, "knob or value is NULL");
  const int k = Tuner::knob_of(knob);
  JP_CHECK(k >= 0, "unknown knob '%s'", knob);
  int rc = check_session(s);
  if (rc) return rc;
  *value = s->tuner.get(k, M, K, variant);
  return JACPCG_OK;
}

int jacpcg_submit(jacpcg_session* s, const jacpcg_request* r, uint64_t* ticket) {
  JP_CHECK(r != nullptr, "request is NULL");
  JP_CHECK(ticket != nullptr, "ticket is NULL");
  int rc = check_session(s);
  if (rc) return rc;
  if (!s->sched) s->sched.reset(new Scheduler(s));
  return s->sched->submit(*r, ticket);
}

int jacpcg_poll(jacpcg_session* s, uint64_t ticket, jacpcg_result* out) {
  JP_CHECK(out != nullptr, "result is NULL");
  int rc = check_session(s);
  if (rc) return rc;
  if (!s->sched) return fail(JACPCG_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  return s->sched->poll(ticket, out);
}

int jacpcg_wait(jacpcg_session* s, uint64_t ticket, int timeout_ms, jacpcg_result* out) {
  JP_CHECK(out != nullptr, "result is NULL");
  int rc = check_session(s);
  if (rc) return rc;
  if (!s->sched) return fail(JACPCG_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  return s->sched->wait(ticket, timeout_ms, out);
}

int jacpcg_cancel(jacpcg_session* s, uint64_t ticket) {
  int rc = check_session(s);
  if (rc) return rc;
  if (!s->sched) return fail(JACPCG_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  return s->sched->cancel(ticket);
}

}  // extern "C"

// ============================================================================
// Session methods that need the fail() helpers.
namespace jacpcg {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

void fill_stats_host(jacpcg_stats* st, int batch, int K, const int32_t* iters, const float* relres,
                     const int32_t* status, const float* beta) {
  fill_stats(st, batch, K, iters, relres, status, beta);
}

}  // namespace jacpcg
