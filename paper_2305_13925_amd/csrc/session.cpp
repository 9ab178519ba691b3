// Session runtime: workspace arena, timing events and the composed paths
// (batched persistent path and the plain one-instance-at-a-time path).
#include "session.hpp"

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstring>
#include <limits>

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
  // Work already enqueued may still use the old arena; captured graphs refer
  // to it. Every call of the session records order_ev at its end, and a call
  // on another stream first waits for the previous call's event, so the last
  // call's event completing means every earlier call's work is done: only
  // that is waited for, not the whole device (the scheduler's slots and
  // other streams keep running).
  if (order_valid) S_HIP(hipEventSynchronize(order_ev));
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
    // The evicted graph may still be executing: its launches belong to
    // earlier calls, all done once the last call's end event completes.
    if (order_valid) (void)hipEventSynchronize(order_ev);
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
  // nrhs right-hand-side columns (B = NULL: the identity, nrhs = K; the
  // refined path always has B = I).
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
  const int n16 = refine_workgroups_per_instance(K);
  const size_t oA64 = refine ? ws.take<double2>(batch * KK) : 0;
  const size_t oX64 = (refine && !X64_out) ? ws.take<double2>(batch * KK) : 0;
  const size_t oR32 = refine ? ws.take<float2>(batch * KK) : 0;
  const size_t oE32 = refine ? ws.take<float2>(batch * KK) : 0;
  const size_t oSc = refine ? ws.take<double>(batch * (size_t)K) : 0;
  const size_t oRn = refine ? ws.take<double>((size_t)batch * n16) : 0;
  const size_t oQd = refine ? ws.take<double>((size_t)batch * n16) : 0;
  const size_t oSt = refine ? ws.take<int32_t>((size_t)batch * n16) : 0;
  const size_t oWG2 = refine ? ws.take<int32_t>((size_t)batch * ncb) : 0;
  // visibility-region spans per 32-user block (sparse Gram tiles and solver)
  const int nt = (K + 31) / 32;
  const bool use_spans = vr_sparse && nt > 2;
  const size_t oTS = use_spans ? ws.take<int2>((size_t)batch * nt) : 0;
  // FP64 and FP32 Grams in antenna chunks: their partial 64 x 64 blocks, one
  // buffer for both (launched one after the other on the same stream)
  const int g64_chunks = refine ? gram64_antenna_chunks(K, batch, use_spans) : 1;
  const bool fp32_class_gram = !(refine && gram_prec == JACPCG_GRAM_FP64_ROUNDED);
  const int g32_chunks = fp32_class_gram ? gram_antenna_chunks(K, batch, gram_prec, use_spans) : 1;
  const int g_nb = (K + 63) / 64;
  const size_t part_blocks = (size_t)batch * (g_nb * (g_nb + 1) / 2) * 64 * 64;
  const size_t part_d2 = std::max(g64_chunks > 1 ? part_blocks * g64_chunks : 0,
                                  g32_chunks > 1 ? (part_blocks * g32_chunks + 1) / 2 : 0);
  const size_t oPart = part_d2 ? ws.take<double2>(part_d2) : 0;
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
  double2* A64 = refine ? at<double2>(oA64) : nullptr;
  double2* X64 = refine ? (X64_out ? X64_out : at<double2>(oX64)) : nullptr;
  double* scale = refine ? at<double>(oSc) : nullptr;
  double* quad = refine ? at<double>(oQd) : nullptr;
  int32_t* rsteps = refine ? at<int32_t>(oSt) : nullptr;

  // The whole path on stream q, phases timed when `timed_run`:
  //   Gram (and the FP64 Gram) -> persistent PCG -> [refinement steps] -> precoder.
  // The refinement runs on the device: kMaxRefineSteps correction solves are
  // enqueued, and each column stops taking corrections once its FP64 residual
  // meets refine_tol (later launches find nothing left to do for it).
  auto enqueue_all = [&](hipStream_t q, bool timed_run) -> hipError_t {
    static const char* const kPhaseName[JACPCG_NUM_PHASES] = {"gram", "solve", "epilogue", "gram64",
                                                             "refine step"};
    auto run = [&](int phase, auto&& launch) -> hipError_t {
      const PhaseRange range(kPhaseName[phase]);
      return timed_run ? timed(q, phase, launch) : launch();
    };
    hipError_t e = hipSuccess;
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
      e = launch_spans(sl, q);
      if (e != hipSuccess) return e;
    }
    if (refine) {
      Gram64Launch g64{H, ldh, stride_h, batch, M, K, xi, A64, tspan, g64_chunks,
                       g64_chunks > 1 ? at<double2>(oPart) : nullptr};
      e = run(JACPCG_PHASE_GRAM64, [&] { return launch_gram64(g64, q); });
      if (e != hipSuccess) return e;
    }
    if (refine && gram_prec == JACPCG_GRAM_FP64_ROUNDED) {
      // the FP32 solves take the FP64 Gram rounded once to FP32
      e = launch_narrow_gram(A64, K, batch, xi, A, K, (int64_t)KK, gdiag, q);
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
      g.msplit = g32_chunks;
      g.partial = g32_chunks > 1 ? reinterpret_cast<float2*>(at<double2>(oPart)) : nullptr;
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
    p.gdiag = refine ? nullptr : gdiag;  // refined path: the power factor comes from FP64 X
    p.fpart = fpart;
    p.tile_span = tspan;
    p.a_source = tuner.pcg_a_source(K);
    e = run(JACPCG_PHASE_SOLVE, [&] { return launch_pcg(p, q, nullptr); });
    if (e != hipSuccess) return e;

    if (refine) {
      RefineStepLaunch rs{};
      rs.A64 = A64;
      rs.X64 = X64;
      rs.X32 = X;
      rs.E32 = at<float2>(oE32);
      rs.batch = batch;
      rs.K = K;
      rs.nrhs = K;
      rs.xi = xi;
      rs.tol = refine_tol;
      rs.R32 = at<float2>(oR32);
      rs.scale = scale;
      rs.rnorm2 = at<double>(oRn);
      rs.quad = quad;
      rs.steps = rsteps;
      rs.tile_span = tspan;
      PcgLaunch pc{};
      pc.A = A;
      pc.lda = K;
      pc.stride_a = (int64_t)KK;
      pc.B = rs.R32;
      pc.ldb = K;
      pc.stride_b = (int64_t)KK;
      pc.X = at<float2>(oE32);
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
      pc.col_gate = scale;
      pc.gate_tol = refine_tol;
      pc.a_source = p.a_source;
      for (int step = 0;; ++step) {
        rs.step = step;
        e = run(JACPCG_PHASE_RESIDUAL, [&] { return launch_refine_step(rs, q); });
        if (e != hipSuccess) return e;
        if (step == kMaxRefineSteps) break;
        e = run(JACPCG_PHASE_SOLVE, [&] { return launch_pcg(pc, q, nullptr); });
        if (e != hipSuccess) return e;
      }
    }

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
    E.mtiles = tuner.precoder_mtiles(M, K, E.split);
    E.fpart64 = refine ? quad : nullptr;  // ||H X64||^2 from the last FP64 residual
    E.ncb64 = n16;
    E.ref_scale = scale;
    E.ref_tol = refine_tol;
    E.tile_span = tspan;
    e = run(JACPCG_PHASE_EPILOGUE, [&] { return launch_precoder(E, q); });
    if (e != hipSuccess) return e;
    if (X64_out && !refine) e = launch_widen(X, K, (int64_t)KN, batch, K, nrhs, X64_out, q);
    return e;
  };

  // Repeated calls with identical arguments replay one captured HIP graph
  // (captured on a side stream, launched on the caller's stream).
  const PhaseRange call_range(refine ? "rzf_precoder (refined)" : "rzf_precoder");
  bool launched = false;
  if (use_graphs && !profiling) {
    const uint64_t key = graph_key({(uint64_t)batch, (uint64_t)M, (uint64_t)K, (uint64_t)nrhs,
                                    (uint64_t)(uintptr_t)B, (uint64_t)ldb, (uint64_t)stride_b, (uint64_t)(uintptr_t)H,
                                    (uint64_t)ldh, (uint64_t)stride_h, bits_of(xi), bits_of(power), bits_of(tol),
                                    (uint64_t)max_iter, (uint64_t)gram_prec, (uint64_t)precond_none,
                                    (uint64_t)split_epilogue, (uint64_t)(uintptr_t)W, (uint64_t)ldw,
                                    (uint64_t)stride_w, (uint64_t)(uintptr_t)X_out, (uint64_t)(uintptr_t)X64_out,
                                    (uint64_t)(uintptr_t)arena, (uint64_t)vr_sparse, (uint64_t)(uintptr_t)user_span,
                                    (uint64_t)refine, bits_of(refine ? refine_tol : 0.0)});
    hipGraphExec_t ex = graph_lookup(key);
    if (!ex) {
      hipStream_t cs = capture_stream();
      hipError_t e = cs ? hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) : hipErrorInvalidValue;
      if (e == hipSuccess) {
        const hipError_t e1 = enqueue_all(cs, false);
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
      launched = true;
    }
    // capture not possible: fall through to the eager launches
  }
  if (!launched) {
    hipError_t e = enqueue_all(st, true);
    if (e == hipErrorNotSupported) return set_error(JACPCG_E_UNSUPPORTED, "Gram precision not available");
    if (e != hipSuccess) return hip_error(this, e, "precoder path launch");
  }

  if (!stats) return JACPCG_OK;
  const size_t hb = (size_t)batch * nrhs * 8 + (size_t)batch * 8 +
                    (refine ? (size_t)batch * K * sizeof(double) + (size_t)batch * n16 * 4 : 0);
  char* h = (char*)host_scratch(hb);
  if (!h) return set_error(JACPCG_E_OUT_OF_MEMORY, "pinned host staging allocation failed");
  int32_t* h_it = (int32_t*)h;
  float* h_rr = (float*)(h_it + (size_t)batch * nrhs);
  int32_t* h_st = (int32_t*)(h_rr + (size_t)batch * nrhs);
  float* h_b = (float*)(h_st + batch);
  double* h_sc = (double*)(h_b + batch);  // 8-byte aligned: 8 (batch * nrhs + batch) bytes precede it
  int32_t* h_steps = (int32_t*)(h_sc + (refine ? (size_t)batch * K : 0));
  S_HIP(hipMemcpyAsync(h_it, iters, (size_t)batch * nrhs * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_rr, relres, (size_t)batch * nrhs * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_st, status, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  S_HIP(hipMemcpyAsync(h_b, beta, (size_t)batch * 4, hipMemcpyDeviceToHost, st));
  if (refine) {
    S_HIP(hipMemcpyAsync(h_sc, scale, (size_t)batch * K * sizeof(double), hipMemcpyDeviceToHost, st));
    S_HIP(hipMemcpyAsync(h_steps, rsteps, (size_t)batch * n16 * 4, hipMemcpyDeviceToHost, st));
  }
  S_HIP(hipStreamSynchronize(st));
  fill_stats_host(stats, batch, nrhs, h_it, h_rr, h_st, h_b);
  if (refine) {
    double worst = 0.0;
    for (size_t i = 0; i < (size_t)batch * K; ++i)
      worst = std::isfinite(h_sc[i]) ? std::max(worst, h_sc[i]) : std::numeric_limits<double>::infinity();
    int steps_max = 0;
    for (size_t i = 0; i < (size_t)batch * n16; ++i) steps_max = std::max(steps_max, (int)h_steps[i]);
    stats->refine_steps = steps_max;
    stats->max_refine_residual = worst;
  }
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
  // The Gram in as many antenna chunks as the batched call takes for this
  // batch, so that both paths give the same A (partial blocks of one instance).
  const int g32_chunks = gram_antenna_chunks(K, batch, 0, false);
  const int g_nb = (K + 63) / 64;
  const size_t oPart =
      g32_chunks > 1 ? ws.take<float2>((size_t)(g_nb * (g_nb + 1) / 2) * g32_chunks * 64 * 64) : 0;
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
    g.msplit = g32_chunks;
    g.partial = g32_chunks > 1 ? at<float2>(oPart) : nullptr;
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
  // Times a set of launch choices: each launched once first (code object
  // load, caches; a choice the kernel rejects counts as infinitely slow), then
  // five rounds that launch every choice once in turn, keeping each choice's
  // fastest launch. Round-robin puts any drift of the GPU's speed over the
  // tuning time (the first tens of milliseconds after allocation run slower)
  // on all choices alike; the fastest launch is the one other work on the GPU
  // disturbed least.
  auto time_all = [&](const std::vector<std::function<hipError_t()>>& fns) {
    std::vector<float> best(fns.size(), 1e30f);
    std::vector<bool> ok(fns.size(), false);
    for (size_t i = 0; i < fns.size(); ++i) {
      ok[i] = fns[i]() == hipSuccess;
      if (!ok[i]) (void)hipGetLastError();
    }
    for (int r = 0; r < 5; ++r)
      for (size_t i = 0; i < fns.size(); ++i) {
        if (!ok[i]) continue;
        (void)hipEventRecord(e0, st);
        (void)fns[i]();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 1e30f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best[i]) best[i] = ms;
      }
    return best;
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
  // Each knob in turn: time every valid value on the synthetic batch and keep
  // the fastest (the earlier knobs already at their chosen values).
  auto pick = [&](int knob, int Mk, int Kk, int variant, std::initializer_list<int> values, auto&& launch_with) {
    const std::vector<int> vals(values);
    std::vector<std::function<hipError_t()>> fns;
    for (int v : vals) fns.push_back([&launch_with, v] { return launch_with(v); });
    const std::vector<float> t = time_all(fns);
    int best = 0;
    float best_t = 1e30f;
    for (size_t i = 0; i < vals.size(); ++i)
      if (t[i] < best_t) {
        best_t = t[i];
        best = vals[i];
      }
    tuner.set(knob, Mk, Kk, variant, best);
    return best;
  };
  g.m_split = pick(kGramWaves, M, K, precision, {2, 4, 8}, [&](int w) {
    if (precision != 0 && w > 4) return hipErrorInvalidValue;  // split kernels take at most 4 waves
    g.m_split = w;
    return launch_gram(g, st);
  });
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
  p.max_iter = 8;
  p.gdiag = gdiag;
  p.fpart = fpart;
  {  // where the solver keeps A (registers or streamed from L2) and, above
     // K = 64, FP32 or split-BF16 products
    auto solve_with = [&](int v) {
      p.a_source = v;
      return launch_pcg(p, st, nullptr);
    };
    if (K <= 64)
      p.a_source = pick(kPcgASource, 0, K, 0, {1, 2}, solve_with);
    else
      p.a_source = pick(kPcgASource, 0, K, 0, {2, 3}, solve_with);
  }
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
  // Column tiles per wave and (split-BF16) antenna blocks per workgroup
  // interact, so they are searched together.
  const bool tune_nj = K <= 128 && K > 32, tune_mt = E.split == 3;
  if (tune_nj || tune_mt) {
    std::vector<std::pair<int, int>> cand;  // (column tiles, antenna blocks)
    for (int nj : {1, 2}) {
      if (!tune_nj && nj > 1) break;
      for (int mt : {1, 2, 4}) {
        if (!tune_mt && mt > 1) break;
        cand.emplace_back(tune_nj ? nj : 0, tune_mt ? mt : 0);
      }
    }
    std::vector<std::function<hipError_t()>> fns;
    for (const auto& c : cand)
      fns.push_back([&E, &st, c] {
        PrecoderLaunch e = E;
        e.nj = c.first;
        e.mtiles = c.second;
        return launch_precoder(e, st);
      });
    const std::vector<float> t = time_all(fns);
    int best_nj = 0, best_mt = 0;
    float best_t = 1e30f;
    for (size_t i = 0; i < cand.size(); ++i)
      if (t[i] < best_t) {
        best_t = t[i];
        best_nj = cand[i].first;
        best_mt = cand[i].second;
      }
    if (tune_nj) tuner.set(kPrecoderNj, M, K, E.split, best_nj);
    if (tune_mt) tuner.set(kPrecoderMtiles, M, K, E.split, best_mt);
  }
  event_pool.push_back(e0);
  event_pool.push_back(e1);
  graph_clear();  // captured graphs hold the previous choices
  S_HIP(hipStreamSynchronize(st));
  return JACPCG_OK;
}
