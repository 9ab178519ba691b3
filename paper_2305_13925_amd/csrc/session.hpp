// Session state of libjacpcg: device, workspace arena, pinned staging memory,
// per-phase kernel timing and the autotuned launch choices.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <initializer_list>
#include <memory>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/jacpcg.h"
#include "common.hpp"
#include "sched.hpp"
#include "tuner.hpp"

namespace jacpcg {

// A roctx range around the host-side enqueue of one call or phase: named
// ranges in a rocprofv3 --marker-trace, and a no-op without a profiler.
struct PhaseRange {
  explicit PhaseRange(const char* name) { roctxRangePushA(name); }
  ~PhaseRange() { roctxRangePop(); }
  PhaseRange(const PhaseRange&) = delete;
  PhaseRange& operator=(const PhaseRange&) = delete;
};

// Two-phase workspace plan: offsets are taken first, the arena is sized once,
// then offsets become device pointers.
struct Workspace {
  size_t bytes = 0;
  template <class T>
  size_t take(size_t n) {
    const size_t off = (bytes + 255) & ~size_t(255);
    bytes = off + n * sizeof(T);
    return off;
  }
};

int set_error(int code, const char* msg);

// Fixed device workspace of rzf_precoder_noalloc (noalloc.hip).
hipError_t noalloc_setup(int device);
size_t noalloc_scratch_bytes();
size_t noalloc_need(int batch, int K);
void fill_stats_host(jacpcg_stats* st, int batch, int K, const int32_t* iters, const float* relres,
                     const int32_t* status, const float* beta);

}  // namespace jacpcg

struct jacpcg_session {
  int device = 0;
  size_t budget = 0;
  std::string tune_path;
  jacpcg::Tuner tuner;
  bool poisoned = false;
  bool profiling = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::unique_ptr<jacpcg::Scheduler> sched;  // created on the first request

  char* arena = nullptr;
  size_t arena_bytes = 0;

  // The calls of a session share its workspace. A call on another stream than
  // the previous call first waits for that call's work (an event recorded at
  // the end of every call), so the streams a caller alternates between never
  // use the workspace at the same time.
  hipEvent_t order_ev = nullptr;
  hipStream_t order_stream = nullptr;
  bool order_valid = false;
  template <class F>
  int ordered(hipStream_t st, F&& call) {
    if (order_valid && st != order_stream) {
      const hipError_t e = hipStreamWaitEvent(st, order_ev, 0);
      if (e != hipSuccess) return ordered_fail(e);
    }
    const int rc = call();
    if (!order_ev && hipEventCreateWithFlags(&order_ev, hipEventDisableTiming) != hipSuccess) {
      order_ev = nullptr;
      (void)hipGetLastError();
      return rc;
    }
    if (hipEventRecord(order_ev, st) == hipSuccess) {
      order_stream = st;
      order_valid = true;
    } else {
      (void)hipGetLastError();
    }
    return rc;
  }
  int ordered_fail(hipError_t e);
  void* pinned = nullptr;
  size_t pinned_bytes = 0;

  struct PendingEvent {
    hipEvent_t a, b;
    int phase;
  };
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> event_pool;
  double phase_ms[JACPCG_NUM_PHASES] = {};
  int64_t phase_count[JACPCG_NUM_PHASES] = {};

  // HIP graph cache of rzf_precoder launch sequences (keyed by every argument
  // and the workspace address; cleared when the workspace moves).
  bool use_graphs = true;
  struct CachedGraph {
    uint64_t key;
    hipGraphExec_t exec;
  };
  std::vector<CachedGraph> graphs;  // most recent last
  hipStream_t cap_stream = nullptr;
  static uint64_t graph_key(std::initializer_list<uint64_t> fields);
  static uint64_t bits_of(double d);
  hipGraphExec_t graph_lookup(uint64_t key);
  void graph_insert(uint64_t key, hipGraphExec_t exec);
  void graph_clear();
  hipStream_t capture_stream();
  int autotune(hipStream_t st, int batch, int M, int K, int precision, int flags);

  // Grow the arena to hold `ws` (synchronises the device when it has to grow).
  int reserve(const jacpcg::Workspace& ws);
  template <class T>
  T* at(size_t off) {
    return reinterpret_cast<T*>(arena + off);
  }
  // Pinned host staging buffer of at least `bytes`.
  void* host_scratch(size_t bytes);

  hipEvent_t get_event();
  template <class F>
  hipError_t timed(hipStream_t st, int phase, F&& launch) {
    if (!profiling) return launch();
    hipEvent_t a = get_event(), b = get_event();
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    pending.push_back({a, b, phase});
    return e;
  }
  hipError_t collect_events();
  void shutdown();

  int run_rzf(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh, int64_t stride_h, int nrhs,
              const float2* B, int64_t ldb, int64_t stride_b, double xi, double power, double tol, int max_iter,
              int gram_prec, bool refine, bool precond_none, bool split_epilogue, double refine_tol, float2* W,
              int64_t ldw, int64_t stride_w, float2* X_out, double2* X64_out, jacpcg_stats* stats,
              bool vr_sparse = false, const int32_t* user_span = nullptr);
  int run_block(hipStream_t st, int batch, int M1, int Mc, int M2, int K1, int K2, const float2* H, int64_t ldh,
                int64_t stride_h, double xi, double power, double tol, int max_iter, int gram_prec, bool refine,
                bool precond_none, bool split_epilogue, double refine_tol, float2* G, int64_t ldg, int64_t stride_g,
                jacpcg_stats* stats);
  int run_sinr(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh, int64_t stride_h,
               const float2* W, int64_t ldw, int64_t stride_w, double sigma2, float* sinr, float* se);
  int run_rzf_plain(hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh, int64_t stride_h,
                    double xi, double power, double tol, int max_iter, bool precond_none, bool split_epilogue,
                    float2* W, int64_t ldw,
                    int64_t stride_w, float2* X_out, jacpcg_stats* stats);
};

namespace jacpcg {
int run_rzf_noalloc(jacpcg_session* s, hipStream_t st, int batch, int M, int K, const float2* H, int64_t ldh,
                    int64_t stride_h, double xi, double power, double tol, int max_iter, int gram_prec,
                    bool precond_none, bool split_epilogue, float2* W, int64_t ldw, int64_t stride_w,
                    int32_t* status);
}  // namespace jacpcg
