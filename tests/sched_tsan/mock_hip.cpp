// Host implementation of the HIP stand-in (see hip/hip_runtime.h) and of the
// kernel launchers the scheduler calls. Every stream owns a worker thread that
// runs its queued operations in order; an event records the generation of its
// last recording and completes when its stream reaches it. The launchers
// enqueue work that writes the outputs the scheduler reads back (statuses,
// iteration counts) and touches every instance's W, so the sanitizer sees
// the same producer / consumer pattern as on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>

#include "../../paper_2305_13925_amd/csrc/common.hpp"

struct MockStream {
  std::mutex m;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool stop = false, busy = false;
  std::thread th;
  MockStream() {
    th = std::thread([this] {
      std::unique_lock<std::mutex> lk(m);
      while (true) {
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) break;
        auto f = std::move(q.front());
        q.pop_front();
        busy = true;
        lk.unlock();
        f();
        lk.lock();
        busy = false;
        cv.notify_all();
      }
    });
  }
  void push(std::function<void()> f) {
    std::lock_guard<std::mutex> lk(m);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(m);
    cv.wait(lk, [&] { return q.empty() && !busy; });
  }
  ~MockStream() {
    {
      std::lock_guard<std::mutex> lk(m);
      stop = true;
      cv.notify_all();
    }
    th.join();
  }
};

// An event's state is shared with the stream tasks that complete or wait on
// it, so destroying an event whose last record is still pending is safe, as
// HIP allows (the resources go when the record completes).
struct EventState {
  std::mutex m;
  std::condition_variable cv;
  uint64_t recorded = 0, completed = 0;
};
struct MockEvent {
  std::shared_ptr<EventState> st = std::make_shared<EventState>();
};

namespace {
MockStream* null_stream() {
  static MockStream s;
  return &s;
}
MockStream* S(hipStream_t s) { return s ? s : null_stream(); }
// A little time per launch, so batches overlap with later submissions.
void work() { std::this_thread::sleep_for(std::chrono::microseconds(50 + std::rand() % 200)); }
}  // namespace

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new MockStream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  S(s)->drain();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::shared_ptr<EventState> st = e->st;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(st->m);
    gen = ++st->recorded;
  }
  S(s)->push([st, gen] {
    std::lock_guard<std::mutex> lk(st->m);
    if (st->completed < gen) st->completed = gen;
    st->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::shared_ptr<EventState> st = e->st;
  std::unique_lock<std::mutex> lk(st->m);
  const uint64_t gen = st->recorded;
  st->cv.wait(lk, [&] { return st->completed >= gen; });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(e->st->m);
  return e->st->completed >= e->st->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  std::shared_ptr<EventState> st = e->st;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(st->m);
    gen = st->recorded;
  }
  S(s)->push([st, gen] {
    std::unique_lock<std::mutex> lk(st->m);
    st->cv.wait(lk, [&] { return st->completed >= gen; });
  });
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  S(s)->push([=] { std::memcpy(dst, src, n); });
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }

namespace jacpcg {

int set_error(int code, const char*) { return code; }

hipError_t launch_gram(const GramLaunch& g, hipStream_t s) {
  const GramLaunch c = g;
  S(s)->push([c] {
    work();
    for (int b = 0; b < c.batch; ++b) {
      const float2* h = c.H_ptrs ? c.H_ptrs[b] : c.H + (int64_t)b * c.stride_h;
      c.A[(int64_t)b * c.stride_a] = h[0];  // reads the request's channel
    }
  });
  return hipSuccess;
}

hipError_t launch_pcg(const PcgLaunch& p, hipStream_t s, int*) {
  const PcgLaunch c = p;
  S(s)->push([c] {
    work();
    const int ncb = (c.nrhs + 31) / 32;
    for (int b = 0; b < c.batch; ++b) {
      for (int j = 0; j < c.nrhs; ++j)
        if (c.iters) c.iters[(int64_t)b * c.nrhs + j] = 1 + (b + j) % 5;
      for (int q = 0; q < ncb; ++q)
        if (c.wg_status) c.wg_status[b * ncb + q] = kStatusOk;
    }
  });
  return hipSuccess;
}

hipError_t launch_precoder(const PrecoderLaunch& e, hipStream_t s) {
  const PrecoderLaunch c = e;
  S(s)->push([c] {
    work();
    for (int b = 0; b < c.batch; ++b) {
      if (c.status) c.status[b] = kStatusOk;
      float2* w = c.W_ptrs ? c.W_ptrs[b] : c.W + (int64_t)b * c.stride_w;
      w[0] = make_float2(1.f, (float)b);  // writes the request's precoder
    }
  });
  return hipSuccess;
}

}  // namespace jacpcg
