// Session runtime: workspace arena, timing events and the composed paths
// (batched persistent path and the plain one-instance-at-a-time path).
#include "session.hpp"

#include <algorithm>
#include <cstring>

using namespace jacpcg;

namespace {

constexpr int kMaxRefineSteps = 16;

int hip_error(jacpcg_session* s, hipError_t e, const char* what) {
  s->poisoned = true;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_error(JACPCG_E_HIP, m.c_str());
}

#define S_HIP(expr)                                       \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_error(this, e_, #expr); \
  } while (0)

}  // namespace

int jacpcg_session::reserve(const Workspace& ws) {
  if (ws.bytes <= arena_bytes) return JACPCG_OK;
  if (budget && ws.bytes > budget) return set_error(JACPCG_E_OUT_OF_MEMORY, "workspace exceeds the session budget");
  // Work already enqueued may still use the old arena; captured graphs refer to it.
  S_HIP(hipDeviceSynchronize());
  graph_clear();
  if (arena) S_HIP(hipFree(arena));
  arena = nullptr;
  arena_bytes = 0;
  const size_t want = std::max(ws.bytes, (size_t)1 << 20);
  hipError_t e = hipMalloc((void**)&arena, want);
  if (e != hipSuccess) {
    arena = nullptr;
    (void)hipGetLastError();
    return set_error(JACPCG_E_OUT_OF_MEMORY, "hipMalloc of the workspace failed");
  }
  arena_bytes = want;
  return JACPCG_OK;
}

void* jacpcg_session::host_scratch(size_t bytes) {
  if (bytes <= pinned_bytes) return pinned;
  if (pinned) (void)hipHostFree(pinned);
  pinned = nullptr;
  pinned_bytes = 0;
  const size_t want = std::max(bytes, (size_t)1 << 16);
  if (hipHostMalloc(&pinned, want, hipHostMallocDefault) != hipSuccess) {
    pinned = nullptr;
    return nullptr;
  }
  pinned_bytes = want;
  return pinned;
}

hipEvent_t jacpcg_session::get_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

hipError_t jacpcg_session::collect_events() {
  for (auto& p : pending) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return e;
    phase_ms[p.phase] += ms;
    phase_count[p.phase] += 1;
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
  return hipSuccess;
}

uint64_t jacpcg_session::graph_key(std::initializer_list<uint64_t> fields) {
  uint64_t h = 1469598103934665603ULL;
  for (uint64_t v : fields) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    h *= 1099511628211ULL;
  }
  return h;
}

uint64_t jacpcg_session::bits_of(double d) {
  uint64_t u;
  std::memcpy(&u, &d, sizeof u);
  return u;
}

hipGraphExec_t jacpcg_session::graph_lookup(uint64_t key) {
  for (size_t i = 0; i < graphs.size(); ++i)
    if (graphs[i].key == key) {
      CachedGraph g = graphs[i];
      graphs.erase(graphs.begin() + i);
      graphs.push_back(g);
      return g.exec;
    }
  return nullptr;
}

void jacpcg_session::graph_insert(uint64_t key, hipGraphExec_t exec) {
  constexpr size_t kMaxGraphs = 32;
  if (graphs.size() >= kMaxGraphs) {
    (void)hipDeviceSynchronize();  // the evicted graph may still be executing
    (void)hipGraphExecDestroy(graphs.front().exec);
    graphs.erase(graphs.begin());
  }
  graphs.push_back({key, exec});
}

void jacpcg_session::graph_clear() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

hipStream_t jacpcg_session::capture_stream() {
  if (!cap_stream && hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) cap_stream = nullptr;
  return cap_stream;
}

int jacpcg_session::ordered_fail(hipError_t e) {
  (void)hipGetLastError();
  return set_error(JACPCG_E_HIP, hipGetErrorString(e));
}

void jacpcg_session::shutdown() {
  if (sched) sched->stop();
  sched.reset();
  (void)hipDeviceSynchronize();
  if (order_ev) (void)hipEventDestroy(order_ev);
  order_ev = nullptr;
  order_valid = false;
  graph_clear();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending.clear();
  for (auto e : event_pool) (void)hipEventDestroy(e);
  event_pool.clear();
  if (arena) (void)hipFree(arena);
  arena = nullptr;
  if (pinned) (void)hipHostFree(pinned);
  pinned = nullptr;
  if (!tune_path.empty()) tuner.save(tune_path);
}

// ---------------------------------------------------------------------------
// Batched path: Gram -> persistent PCG (+ ||H X||^2 pass) -> precoder.
// ---------------------------------------------------------------------------
int jacpcg_session::run_rzf(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh, int64_t stride_h,
                            int nrhs, const float2* B, int64_t ldb, int64_t stride_b, double xi, double power,
                            double tol, int max_iter, int gram_prec, bool refine, bool precond_none,
                            bool split_epilogue, double refine_tol, float2* W, int64_t ldw, int64_t stride_w,
                            float2* X_out, double2* X64_out, jacpcg_stats* stats, bool vr_sparse,
                            const int32_t* user_span) {
  // nrhs right-hand-side columns (B = NULL: the identity, nrhs = K).
  const int ncb = (nrhs + 31) / 32;
  const size_t KK = (size_t)K * K;
  const size_t KN = (size_t)K * nrhs;
  Workspace ws;
  const size_t oA = ws.take<float2>(batch * KK);
  const size_t oG = ws.take<float>((size_t)batch * K);
  const size_t oX = X_out ? 0 : ws.take<float2>(batch * KN);
  const size_t oF = ws.take<float>((size_t)batch * ncb);
  const size_t oWG = ws.take<int32_t>((size_t)batch * ncb);
  const size_t oS = ws.take<int32_t>(batch);
  const size_t oI = ws.take<int32_t>((size_t)batch * nrhs);
  const size_t oR = ws.take<float>((size_t)batch * nrhs);
  const size_t oB = ws.take<float>(batch);
  // refinement buffers
  const int n16 = residual_workgroups_per_instance(K);
  const size_t oA64 = refine ? ws.take<double2>(batch * KK) : 0;
  const size_t oX64 = refine ? ws.take<double2>(batch * KK) : 0;
  const size_t oR32 = refine ? ws.take<float2>(batch * KK) : 0;
  const size_t oE32 = refine ? ws.take<float2>(batch * KK) : 0;
  const size_t oSc = refine ? ws.take<double>(batch * (size_t)K) : 0;
  const size_t oRn = refine ? ws.take<double>((size_t)batch * n16) : 0;
  const size_t oQd = refine ? ws.take<double>((size_t)batch * n16) : 0;
  const size_t oWG2 = refine ? ws.take<int32_t>((size_t)batch * ncb) : 0;
  // visibility-region spans per 32-user block (sparse Gram tiles and solver)
  const int nt = (K + 31) / 32;
  const bool use_spans = vr_sparse && nt > 2;
  const size_t oTS = use_spans ? ws.take<int2>((size_t)batch * nt) : 0;
  if (int rc = reserve(ws)) return rc;
  const int2* tspan = use_spans ? at<int2>(oTS) : nullptr;
  float2* A = at<float2>(oA);
  float* gdiag = at<float>(oG);
  float2* X = X_out ? X_out : at<float2>(oX);
  float* fpart = at<float>(oF);
  int32_t* wgs = at<int32_t>(oWG);
  int32_t* status = at<int32_t>(oS);
  int32_t* iters = at<int32_t>(oI);
  float* relres = at<float>(oR);
  float* beta = at<float>(oB);

  // Gram -> persistent PCG -> status; on stream q, phases timed when `timed_run`.
  auto enqueue_solve = [&](hipStream_t q, bool timed_run) -> hipError_t {
    auto run = [&](int phase, auto&& launch) -> hipError_t {
      return timed_run ? timed(q, phase, launch) : launch();
    };
    if (use_spans) {
      SpanLaunch sl{};
      sl.H = H;
      sl.ldh = ldh;
      sl.stride_h = stride_h;
      sl.user_span_in = user_span;
      sl.batch = batch;
      sl.M = M;
      sl.K = K;
      sl.tile_span = const_cast<int2*>(tspan);
      hipError_t es = launch_spans(sl, q);
      if (es != hipSuccess) return es;
    }
    hipError_t e = hipSuccess;
    if (refine) {
      // The refinement needs the FP64 Gram anyway: the FP32 solves take it
      // rounded once to FP32 (the Gram precision bits do not apply).
      Gram64Launch g64{H, ldh, stride_h, batch, M, K, xi, at<double2>(oA64)};
      e = run(JACPCG_PHASE_GRAM64, [&] { return launch_gram64(g64, q); });
      if (e != hipSuccess) return e;
      e = launch_narrow_gram(at<double2>(oA64), K, batch, xi, A, K, (int64_t)KK, gdiag, q);
      if (e != hipSuccess) return e;
    } else {
      GramLaunch g{};
      g.H = H;
      g.ldh = ldh;
      g.stride_h = stride_h;
      g.batch = batch;
      g.M = M;
      g.K = K;
      g.xi = (float)xi;
      g.A = A;
      g.lda = K;
      g.stride_a = (int64_t)KK;
      g.diag = nullptr;
      g.gdiag = gdiag;
      g.precision = gram_prec;
      g.m_split = tuner.gram_waves(M, K, gram_prec);
      g.tile_span = tspan;
      e = run(JACPCG_PHASE_GRAM, [&] { return launch_gram(g, q); });
      if (e != hipSuccess) return e;
    }

    PcgLaunch p{};
    p.A = A;
    p.lda = K;
    p.stride_a = (int64_t)KK;
    p.B = B;
    p.ldb = ldb;
    p.stride_b = stride_b;
    p.X = X;
    p.ldx = K;
    p.stride_x = (int64_t)KN;
    p.batch = batch;
    p.K = K;
    p.nrhs = nrhs;
    p.tol = (float)tol;
    p.max_iter = max_iter;
    p.precond_none = precond_none;
    p.iters = iters;
    p.relres = relres;
    p.wg_status = wgs;
    p.gdiag = gdiag;
    p.fpart = fpart;
    p.tile_span = tspan;
    e = run(JACPCG_PHASE_SOLVE, [&] { return launch_pcg(p, q, nullptr); });
    if (e != hipSuccess) return e;
    return hipSuccess;  // the per-instance status is reduced by the precoder kernel
  };
  // W = beta_pow H X (and the FP64 copy of X) on stream q.
  auto enqueue_precoder = [&](hipStream_t q, bool timed_run, const double* quad64, int nq) -> hipError_t {
    PrecoderLaunch E{};
    E.H = H;
    E.ldh = ldh;
    E.stride_h = stride_h;
    E.X = X;
    E.ldx = K;
    E.stride_x = (int64_t)KN;
    E.W = W;
    E.ldw = ldw;
    E.stride_w = stride_w;
    E.batch = batch;
    E.M = M;
    E.K = K;
    E.nrhs = nrhs;
    E.fpart = fpart;
    E.ncb = ncb;
    E.power = (float)power;
    E.beta_out = beta;
    E.wg_status = wgs;
    E.status = status;
    E.split = split_epilogue ? 3 : 0;
    E.nj = tuner.precoder_nj(M, K, E.split);
    E.fpart64 = quad64;  // refined path: ||H X64||^2 from the last FP64 residual
    E.ncb64 = nq;
    E.tile_span = tspan;
    hipError_t e = timed_run ? timed(q, JACPCG_PHASE_EPILOGUE, [&] { return launch_precoder(E, q); })
                             : launch_precoder(E, q);
    if (e != hipSuccess) return e;
    if (X64_out && !refine) e = launch_widen(X, K, (int64_t)KN, batch, K, nrhs, X64_out, q);
    return e;
  };

  // Repeated calls with identical arguments replay one captured HIP graph
  // (captured on a side stream, launched on the caller's stream).
  if (!refine && !stats && use_graphs && !profiling) {
    const uint64_t key = graph_key({(uint64_t)batch, (uint64_t)M, (uint64_t)K, (uint64_t)nrhs,
                                    (uint64_t)(uintptr_t)B, (uint64_t)ldb, (uint64_t)stride_b, (uint64_t)(uintptr_t)H,
                                    (uint64_t)ldh, (uint64_t)stride_h, bits_of(xi), bits_of(power), bits_of(tol),
                                    (uint64_t)max_iter, (uint64_t)gram_prec, (uint64_t)precond_none,
                                    (uint64_t)split_epilogue, (uint64_t)(uintptr_t)W, (uint64_t)ldw,
                                    (uint64_t)stride_w, (uint64_t)(uintptr_t)X_out, (uint64_t)(uintptr_t)X64_out,
                                    (uint64_t)(uintptr_t)arena, (uint64_t)vr_sparse, (uint64_t)(uintptr_t)user_span});
    hipGraphExec_t ex = graph_lookup(key);
    if (!ex) {
      hipStream_t cs = capture_stream();
      hipError_t e = cs ? hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) : hipErrorInvalidValue;
      if (e == hipSuccess) {
        hipError_t e1 = enqueue_solve(cs, false);
        if (e1 == hipSuccess) e1 = enqueue_precoder(cs, false, nullptr, 0);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (e1 == hipErrorNotSupported) {
          if (graph) (void)hipGraphDestroy(graph);
          return set_error(JACPCG_E_UNSUPPORTED, "Gram precision not available");
        }
        if (e == hipSuccess && e1 == hipSuccess && graph) {
          if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (ex) graph_insert(key, ex);
      }
      (void)hipGetLastError();
    }
    if (ex) {
      hipError_t e = hipGraphLaunch(ex, st);
      if (e != hipSuccess) return hip_error(this, e, "graph launch");
      return JACPCG_OK;
    }
    // capture not possible: fall through to the eager launches
  }

  {
    hipError_t e = enqueue_solve(st, true);
    if (e == hipErrorNotSupported) return set_error(JACPCG_E_UNSUPPORTED, "Gram precision not available");
    if (e != hipSuccess) return hip_error(this, e, "gram/pcg launch");
  }

  // ---- FP64-residual iterative refinement (B = I) --------------------------
  int refine_steps = 0;
  double refine_res = 0.0;
  double2* X64 = refine ? at<double2>(oX64) : nullptr;
  double* quad = refine ? at<double>(oQd) : nullptr;
  if (refine) {
    double2* A64 = at<double2>(oA64);
    float2* R32 = at<float2>(oR32);
    float2* E32 = at<float2>(oE32);
    double* scale = at<double>(oSc);
    double* rn2 = at<double>(oRn);
    // A64 was formed before the first solve.
    AccumulateLaunch acc{X64, X, nullptr, batch, K, K, 1, nullptr};
    hipError_t e = launch_accumulate(acc, st);  // X64 = X (exact widening)
    if (e != hipSuccess) return hip_error(this, e, "accumulate launch");
    double* h_rn = (double*)host_scratch((size_t)batch * n16 * sizeof(double));
    if (!h_rn) return set_error(JACPCG_E_OUT_OF_MEMORY, "pinned host staging allocation failed");
    for (int step = 0;; ++step) {
      ResidualLaunch rl{A64, X64, nullptr, 0, 0, batch, K, K, xi, R32, scale, rn2, quad};
      e = timed(st, JACPCG_PHASE_RESIDUAL, [&] { return launch_residual(rl, st); });
      if (e != hipSuccess) return hip_error(this, e, "residual launch");
      S_HIP(hipMemcpyAsync(h_rn, rn2, (size_t)batch * n16 * sizeof(double), hipMemcpyDeviceToHost, st));
      S_HIP(hipStreamSynchronize(st));
      refine_res = 0.0;
      for (int b = 0; b < batch; ++b) {
        double f = 0.0;
        for (int c = 0; c < n16; ++c) f += h_rn[(size_t)b * n16 + c];
        refine_res = std::max(refine_res, std::sqrt(f / K));  // ||R||_F / ||I||_F
      }
      if (refine_res <= refine_tol || step >= kMaxRefineSteps) break;
      // correction: A E = R / ||r_j|| column by column, in FP32
      PcgLaunch pc{};
      pc.A = A;
      pc.lda = K;
      pc.stride_a = (int64_t)KK;
      pc.B = R32;
      pc.ldb = K;
      pc.stride_b = (int64_t)KK;
      pc.X = E32;
      pc.ldx = K;
      pc.stride_x = (int64_t)KK;
      pc.batch = batch;
      pc.K = K;
      pc.nrhs = K;
      pc.tol = (float)tol;
      pc.max_iter = max_iter;
      pc.precond_none = precond_none;
      pc.wg_status = at<int32_t>(oWG2);
      pc.tile_span = tspan;
      e = timed(st, JACPCG_PHASE_SOLVE, [&] { return launch_pcg(pc, st, nullptr); });
      if (e != hipSuccess) return hip_error(this, e, "correction pcg launch");
      AccumulateLaunch ac{X64, E32, scale, batch, K, K, 0, X};
      e = launch_accumulate(ac, st);
      if (e != hipSuccess) return hip_error(this, e, "accumulate launch");
      ++refine_steps;
    }
  }

  {
    hipError_t e = enqueue_precoder(st, true, quad, n16);
    if (e != hipSuccess) return hip_error(this, e, "precoder launch");
    if (X64_out && refine) {
      e = hipMemcpyAsync(X64_out, X64, batch * KK * sizeof(double2), hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_error(this, e, "X64 output");
    }
  }

  jacpcg_stats local_stats;
  if (!stats && refine) stats = &local_stats;  // the refined path synchronises anyway
  if (!stats) return JACPCG_OK;
  const size_t hb = (size_t)batch * nrhs * 8 + (size_t)batch * 8;
  char* h = (char*)host_scratch(hb);
  if (!h) return set_error(JACPCG_E_OUT_OF_MEMORY, "pinned host staging allocation failed");
  int32_t* h_it = (int32_t*)h;
  float* h_rr = (float*)(h_it + (size_t)batch * nrhs);
  int32_t* h_st = (int32_t*)(h_rr + (size_t)batch * nrhs);
  float* h_b = (float*)(h_st + batch);
  S_HIP(hipMemcpyAsync(h_it, iters, (size_t)batch * nrhs * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_rr, relres, (size_t)batch * nrhs * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_st, status, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_b, beta, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipStreamSynchronize(st));
  fill_stats_host(stats, batch, nrhs, h_it, h_rr, h_st, h_b);
  stats->refine_steps = refine_steps;
  stats->max_refine_residual = refine_res;
  if (refine && refine_res > refine_tol && stats->worst_status == JACPCG_OK) stats->worst_status = JACPCG_NOT_CONVERGED;
  return stats->worst_status;
}

// ---------------------------------------------------------------------------
// Subarray-block RZF: three independent batched precoders on strided views.
// ---------------------------------------------------------------------------
int jacpcg_session::run_block(hipStream_t st, int batch, int M1, int Mc, int M2, int K1, int K2, const float2* H,
                              int64_t ldh, int64_t stride_h, double xi, double power, double tol, int max_iter,
                              int gram_prec, bool refine, bool precond_none, bool split_epilogue, double refine_tol,
                              float2* G, int64_t ldg, int64_t stride_g, jacpcg_stats* stats) {
  const int M = M1 + Mc + M2, K = K1 + K2;
  // The blocks outside the groups' subarrays are zero (eq. 6).
  S_HIP(launch_zero_block(G, ldg, stride_g, batch, 0, M1, K1, K2, st));
  S_HIP(launch_zero_block(G, ldg, stride_g, batch, M1 + Mc, M2, 0, K1, st));
  struct Block {
    int row0, rows, col0, cols;
  };
  const Block blocks[3] = {{0, M1, 0, K1}, {M1, Mc, 0, K}, {M1 + Mc, M2, K1, K2}};
  jacpcg_stats acc{};
  bool first = true;
  int worst = JACPCG_OK;
  for (const Block& bl : blocks) {
    if (bl.rows == 0 || bl.cols == 0) continue;
    jacpcg_stats part{};
    const int rc = run_rzf(st, batch, bl.rows, bl.cols, H + bl.row0 + (int64_t)bl.col0 * ldh, ldh, stride_h,
                           bl.cols, nullptr, 0, 0, xi, power, tol, max_iter, gram_prec, refine, precond_none,
                           split_epilogue, refine_tol, G + bl.row0 + (int64_t)bl.col0 * ldg, ldg, stride_g, nullptr,
                           nullptr, stats ? &part : nullptr);
    if (rc < 0) return rc;
    if (!stats) continue;
    if (first) {
      acc = part;
      first = false;
    } else {
      acc.max_rel_residual = std::max(acc.max_rel_residual, part.max_rel_residual);
      acc.max_refine_residual = std::max(acc.max_refine_residual, part.max_refine_residual);
      acc.max_iters = std::max(acc.max_iters, part.max_iters);
      acc.refine_steps = std::max(acc.refine_steps, part.refine_steps);
      acc.beta_pow_min = std::min(acc.beta_pow_min, part.beta_pow_min);
      acc.beta_pow_max = std::max(acc.beta_pow_max, part.beta_pow_max);
    }
    if (part.worst_status < 0 || (worst >= 0 && part.worst_status > worst)) worst = part.worst_status;
  }
  (void)M;
  if (!stats) return JACPCG_OK;
  acc.worst_status = worst;
  *stats = acc;
  return worst;
}

// ---------------------------------------------------------------------------
// Precoder evaluation: C = H^H W, per-user SINR and sum rate.
// ---------------------------------------------------------------------------
int jacpcg_session::run_sinr(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh,
                             int64_t stride_h, const float2* W, int64_t ldw, int64_t stride_w, double sigma2,
                             float* sinr, float* se) {
  Workspace ws;
  const size_t oC = ws.take<float2>((size_t)batch * K * K);
  const size_t oS = sinr ? 0 : ws.take<float>((size_t)batch * K);
  if (int rc = reserve(ws)) return rc;
  EvalLaunch e{};
  e.H = H;
  e.ldh = ldh;
  e.stride_h = stride_h;
  e.W = W;
  e.ldw = ldw;
  e.stride_w = stride_w;
  e.batch = batch;
  e.M = M;
  e.K = K;
  e.sigma2 = (float)sigma2;
  e.C = at<float2>(oC);
  e.sinr = sinr ? sinr : at<float>(oS);
  e.se = se;
  S_HIP(launch_eval(e, st));
  return JACPCG_OK;
}

// ---------------------------------------------------------------------------
// Plain path: one instance at a time, one launch per PCG iteration.
// ---------------------------------------------------------------------------
int jacpcg_session::run_rzf_plain(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh,
                                  int64_t stride_h, double xi, double power, double tol, int max_iter,
                                  bool precond_none, bool split_epilogue, float2* W, int64_t ldw, int64_t stride_w,
                                  float2* X_out,
                                  jacpcg_stats* stats) {
  const int ncb = (K + 31) / 32;
  const size_t KK = (size_t)K * K;
  Workspace ws;
  const size_t oA = ws.take<float2>(KK);
  const size_t oG = ws.take<float>(K);
  const size_t oX = X_out ? 0 : ws.take<float2>(batch * KK);
  const size_t oF = ws.take<float>(ncb);
  const size_t oWG = ws.take<int32_t>(ncb);
  const size_t oS = ws.take<int32_t>(batch);
  const size_t oI = ws.take<int32_t>((size_t)batch * K);
  const size_t oR = ws.take<float>((size_t)batch * K);
  const size_t oB = ws.take<float>(batch);
  const size_t oSV = ws.take<float>(pcg_state_floats_per_wg(K) * ncb);
  const size_t oSC = ws.take<float>((size_t)8 * 32 * ncb);
  const size_t oSD = ws.take<int32_t>(ncb);
  if (int rc = reserve(ws)) return rc;
  float2* A = at<float2>(oA);
  float* gdiag = at<float>(oG);
  float2* X = X_out ? X_out : at<float2>(oX);
  float* fpart = at<float>(oF);
  int32_t* wgs = at<int32_t>(oWG);
  int32_t* status = at<int32_t>(oS);
  int32_t* iters = at<int32_t>(oI);
  float* relres = at<float>(oR);
  float* beta = at<float>(oB);
  PcgState state{at<float>(oSV), at<float>(oSC), at<int32_t>(oSD)};
  int32_t* h_done = (int32_t*)host_scratch(std::max<size_t>((size_t)ncb * 4, (size_t)batch * K * 8 + batch * 8));
  if (!h_done) return set_error(JACPCG_E_OUT_OF_MEMORY, "pinned host staging allocation failed");

  for (int b = 0; b < batch; ++b) {
    const float2* Hb = H + (int64_t)b * stride_h;
    GramLaunch g{};
    g.H = Hb;
    g.ldh = ldh;
    g.stride_h = 0;
    g.batch = 1;
    g.M = M;
    g.K = K;
    g.xi = (float)xi;
    g.A = A;
    g.lda = K;
    g.stride_a = (int64_t)KK;
    g.gdiag = gdiag;
    g.precision = 0;
    g.m_split = tuner.gram_waves(M, K, 0);
    hipError_t e = timed(st, JACPCG_PHASE_GRAM, [&] { return launch_gram(g, st); });
    if (e != hipSuccess) return hip_error(this, e, "gram launch");

    PcgLaunch p{};
    p.A = A;
    p.lda = K;
    p.stride_a = (int64_t)KK;
    p.X = X + (int64_t)b * KK;
    p.ldx = K;
    p.stride_x = (int64_t)KK;
    p.batch = 1;
    p.K = K;
    p.nrhs = K;
    p.tol = (float)tol;
    p.max_iter = max_iter;
    p.precond_none = precond_none;
    p.iters = iters + (int64_t)b * K;
    p.relres = relres + (int64_t)b * K;
    p.wg_status = wgs;
    p.gdiag = gdiag;
    p.fpart = fpart;
    p.st = state;
    p.chunk = 1;
    const int launches = std::max(1, max_iter);
    for (int t = 0; t < launches; ++t) {
      p.first = (t == 0);
      e = timed(st, JACPCG_PHASE_SOLVE, [&] { return launch_pcg(p, st, nullptr); });
      if (e != hipSuccess) return hip_error(this, e, "pcg launch");
      if (tol > 0.0 && t + 1 < launches) {
        // Host-driven convergence test after every iteration.
        S_HIP(hipMemcpyAsync(h_done, state.done, (size_t)ncb * 4, hipMemcpyDeviceToHost, st));
        S_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int c = 0; c < ncb; ++c) all = all && h_done[c] != 0;
        if (all) break;
      }
    }
    e = launch_status_reduce(wgs, ncb, 1, status + b, st);
    if (e != hipSuccess) return hip_error(this, e, "status reduce launch");

    PrecoderLaunch E{};
    E.H = Hb;
    E.ldh = ldh;
    E.stride_h = 0;
    E.X = X + (int64_t)b * KK;
    E.ldx = K;
    E.stride_x = (int64_t)KK;
    E.W = W + (int64_t)b * stride_w;
    E.ldw = ldw;
    E.stride_w = 0;
    E.batch = 1;
    E.M = M;
    E.K = K;
    E.nrhs = K;
    E.fpart = fpart;
    E.ncb = ncb;
    E.power = (float)power;
    E.beta_out = beta + b;
    E.split = split_epilogue ? 3 : 0;
    E.nj = tuner.precoder_nj(M, K, E.split);
    e = timed(st, JACPCG_PHASE_EPILOGUE, [&] { return launch_precoder(E, st); });
    if (e != hipSuccess) return hip_error(this, e, "precoder launch");
  }

  if (!stats) return JACPCG_OK;
  char* h = (char*)h_done;
  int32_t* h_it = (int32_t*)h;
  float* h_rr = (float*)(h_it + (size_t)batch * K);
  int32_t* h_st = (int32_t*)(h_rr + (size_t)batch * K);
  float* h_b = (float*)(h_st + batch);
  S_HIP(hipMemcpyAsync(h_it, iters, (size_t)batch * K * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_rr, relres, (size_t)batch * K * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_st, status, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_b, beta, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipStreamSynchronize(st));
  fill_stats_host(stats, batch, K, h_it, h_rr, h_st, h_b);
  return stats->worst_status;
}

// ---------------------------------------------------------------------------
// Autotuning: time the launch variants of one shape on synthetic data and keep
// the fastest (Gram waves per workgroup; precoder column tiles per wave).
// ---------------------------------------------------------------------------
int jacpcg_session::autotune(hipStream_t st, int batch, int M, int K, int precision, int flags) {
  const size_t KK = (size_t)K * K;
  const int ncb = (K + 31) / 32;
  Workspace ws;
  const size_t oH = ws.take<float2>((size_t)batch * M * K);
  const size_t oW = ws.take<float2>((size_t)batch * M * K);
  const size_t oA = ws.take<float2>(batch * KK);
  const size_t oG = ws.take<float>((size_t)batch * K);
  const size_t oX = ws.take<float2>(batch * KK);
  const size_t oF = ws.take<float>((size_t)batch * ncb);
  if (int rc = reserve(ws)) return rc;
  float2* H = at<float2>(oH);
  float2* W = at<float2>(oW);
  float2* A = at<float2>(oA);
  float* gdiag = at<float>(oG);
  float2* X = at<float2>(oX);
  float* fpart = at<float>(oF);
  S_HIP(launch_fill_synthetic(H, (size_t)batch * M * K, 12345u, st));
  hipEvent_t e0 = get_event(), e1 = get_event();
  auto time_it = [&](auto&& launch) -> float {
    (void)launch();  // warm-up (code object load, caches)
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; ++r) (void)launch();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 1e30f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
    return ms;
  };
  GramLaunch g{};
  g.H = H;
  g.ldh = M;
  g.stride_h = (int64_t)M * K;
  g.batch = batch;
  g.M = M;
  g.K = K;
  g.xi = 1.0f;
  g.A = A;
  g.lda = K;
  g.stride_a = (int64_t)KK;
  g.gdiag = gdiag;
  g.precision = precision;
  int best_w = 0;
  float best_t = 1e30f;
  for (int w : {2, 4, 8}) {
    if (precision != 0 && w > 4) continue;  // split kernels take at most 4 waves
    g.m_split = w;
    const float t = time_it([&] { return launch_gram(g, st); });
    if (t < best_t) {
      best_t = t;
      best_w = w;
    }
  }
  tuner.set_gram_waves(M, K, precision, best_w);
  g.m_split = best_w;
  S_HIP(launch_gram(g, st));
  PcgLaunch p{};
  p.A = A;
  p.lda = K;
  p.stride_a = (int64_t)KK;
  p.X = X;
  p.ldx = K;
  p.stride_x = (int64_t)KK;
  p.batch = batch;
  p.K = K;
  p.nrhs = K;
  p.max_iter = 4;
  p.gdiag = gdiag;
  p.fpart = fpart;
  S_HIP(launch_pcg(p, st, nullptr));
  PrecoderLaunch E{};
  E.H = H;
  E.ldh = M;
  E.stride_h = (int64_t)M * K;
  E.X = X;
  E.ldx = K;
  E.stride_x = (int64_t)KK;
  E.W = W;
  E.ldw = M;
  E.stride_w = (int64_t)M * K;
  E.batch = batch;
  E.M = M;
  E.K = K;
  E.nrhs = K;
  E.fpart = fpart;
  E.ncb = ncb;
  E.power = 1.0f;
  E.split = (flags & JACPCG_EPILOGUE_FP32) ? 0 : 3;
  int best_nj = 0;
  best_t = 1e30f;
  if (K <= 128 && K > 32) {
    for (int nj : {1, 2}) {
      E.nj = nj;
      const float t = time_it([&] { return launch_precoder(E, st); });
      if (t < best_t) {
        best_t = t;
        best_nj = nj;
      }
    }
    tuner.set_precoder_nj(M, K, E.split, best_nj);
  }
  event_pool.push_back(e0);
  event_pool.push_back(e1);
  graph_clear();  // captured graphs hold the previous choices
  S_HIP(hipStreamSynchronize(st));
  return JACPCG_OK;
}
