// Request scheduler of a session: continuous batching of precoder requests.
//
// Requests (n_sub subcarrier instances of one (M, K) shape each) are admitted
// in FIFO order while the session's HBM budget and the in-flight slots allow.
// Admitted requests with the same shape and solve settings form one batch,
// launched on its slot's stream as Gram -> persistent PCG -> precoder with
// per-instance channel and precoder pointers (no gather copies). Batches on
// different slots run concurrently on the device, and requests that arrive
// while others are in flight are admitted as soon as a slot and budget free up.
// Every instance's arithmetic is independent of the other instances in its
// batch and kernel choices depend only on the shape, so a request's result is
// bitwise the same alone and in any mix.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/jacpcg.h"
#include "sched_policy.hpp"

struct jacpcg_session;

namespace jacpcg {

class Scheduler {
 public:
  explicit Scheduler(jacpcg_session* s);
  ~Scheduler();
  int submit(const jacpcg_request& r, uint64_t* ticket);
  int poll(uint64_t ticket, jacpcg_result* out);
  int wait(uint64_t ticket, int timeout_ms, jacpcg_result* out);
  int cancel(uint64_t ticket);
  void stop();

 private:
  enum State { kQueued, kRunning, kDone };
  struct Req {
    jacpcg_request r;
    size_t bytes = 0;
    BatchKey key;
    int state = kQueued;
    int status = JACPCG_NOT_READY;
    int max_iters = 0;
    bool cancelled = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    hipEvent_t ready = nullptr;  // recorded on the request's stream at submission
  };
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* host = nullptr;  // pinned staging
    size_t host_bytes = 0;
    bool busy = false;   // reserved by the scheduler thread
    bool armed = false;  // launched and its completion event recorded: its completion thread may finish it
    std::vector<uint64_t> members;
    std::vector<int> inst_begin;  // first instance of each member in the batch
    int instances = 0;
    int K = 0;
    size_t bytes = 0;
    int32_t* h_status = nullptr;
    int32_t* h_iters = nullptr;
  };

  void start();
  void scheduler_loop();
  void completion_loop(size_t slot);
  int launch(Slot& slot, const std::vector<uint64_t>& members, const std::vector<jacpcg_request>& rq,
             const std::vector<hipEvent_t>& ready);
  hipEvent_t take_event();             // from the pool, or a new one (lock held)
  void give_event(hipEvent_t e);       // back to the pool (lock held)
  std::vector<hipEvent_t> ev_pool_;
  void finish(Slot& slot);
  double now_us() const;

  jacpcg_session* s_;
  std::mutex mu_;
  std::condition_variable cv_sched_, cv_done_, cv_comp_;
  std::deque<uint64_t> queue_;
  std::unordered_map<uint64_t, Req> reqs_;
  std::vector<Slot> slots_;
  uint64_t next_ticket_ = 1;
  size_t used_ = 0;
  bool running_ = false, stop_ = false;
  int inflight_ = 0;
  std::thread sched_thread_;
  std::vector<std::thread> slot_threads_;  // one completion thread per slot
};

}  // namespace jacpcg
