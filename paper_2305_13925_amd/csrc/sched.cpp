// Request scheduler: admission, batching, launch and completion of precoder
// requests (see sched.hpp).
#include "sched.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <unordered_set>

#include "common.hpp"
#include "session.hpp"

namespace jacpcg {

namespace {

// One slot per hardware queue of the process (GPU_MAX_HW_QUEUES, HIP's
// default 4; at most 8 slots): one more stream would share an in-order
// hardware queue with the first, so a small batch could wait behind a large
// one's kernels instead of running beside them.
int slot_count() {
  int n = 4;
  if (const char* v = std::getenv("GPU_MAX_HW_QUEUES")) {
    const int q = std::atoi(v);
    if (q > 0) n = q;
  }
  return std::min(8, std::max(1, n));
}

uint64_t bits(double d) {
  uint64_t u;
  std::memcpy(&u, &d, sizeof u);
  return u;
}

}  // namespace

Scheduler::Scheduler(jacpcg_session* s) : s_(s) {}

Scheduler::~Scheduler() { stop(); }

double Scheduler::now_us() const {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - s_->t0).count();
}

void Scheduler::start() {
  if (running_) return;
  slots_.resize(slot_count());
  for (auto& sl : slots_) {
    (void)hipSetDevice(s_->device);
    (void)hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    // A blocking-sync event: its waiter sleeps until the batch completes.
    (void)hipEventCreateWithFlags(&sl.done, hipEventDisableTiming | hipEventBlockingSync);
  }
  running_ = true;
  sched_thread_ = std::thread([this] { scheduler_loop(); });
  for (size_t i = 0; i < slots_.size(); ++i) slot_threads_.emplace_back([this, i] { completion_loop(i); });
}

void Scheduler::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (!running_) return;
    stop_ = true;
  }
  cv_sched_.notify_all();
  cv_comp_.notify_all();
  cv_done_.notify_all();
  if (sched_thread_.joinable()) sched_thread_.join();
  for (auto& t : slot_threads_)
    if (t.joinable()) t.join();
  slot_threads_.clear();
  (void)hipSetDevice(s_->device);
  for (auto& kv : reqs_)
    if (kv.second.ready) give_event(kv.second.ready);
  for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
  ev_pool_.clear();
  for (auto& sl : slots_) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ws) (void)hipFree(sl.ws);
    if (sl.host) (void)hipHostFree(sl.host);
    sl = Slot{};
  }
  running_ = false;
}

hipEvent_t Scheduler::take_event() {
  if (!ev_pool_.empty()) {
    hipEvent_t e = ev_pool_.back();
    ev_pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipSetDevice(s_->device);
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void Scheduler::give_event(hipEvent_t e) {
  if (e) ev_pool_.push_back(e);
}

int Scheduler::submit(const jacpcg_request& r, uint64_t* ticket) {
  if (!ticket) return set_error(JACPCG_E_INVALID_ARG, "ticket is NULL");
  if (r.M < 1 || r.K < 1 || r.K > kMaxK || r.n_sub < 1)
    return set_error(JACPCG_E_INVALID_ARG, "request needs M >= 1, 1 <= K <= 256, n_sub >= 1");
  if (!r.H || !r.W) return set_error(JACPCG_E_INVALID_ARG, "request H or W is NULL");
  if (!std::isfinite(r.xi) || r.xi < 0.0) return set_error(JACPCG_E_INVALID_ARG, "request xi must be >= 0");
  if (!std::isfinite(r.power) || r.power <= 0.0) return set_error(JACPCG_E_INVALID_ARG, "request power must be > 0");
  if (!std::isfinite(r.tol) || r.tol < 0.0 || r.max_iter < 0)
    return set_error(JACPCG_E_INVALID_ARG, "request tol and max_iter must be >= 0");
  if (r.precision < 0 || r.precision > 2)
    return set_error(JACPCG_E_UNSUPPORTED, "request precision must be a Gram precision (no refinement)");
  if ((r.flags & ~(JACPCG_PRECOND_NONE | JACPCG_EPILOGUE_FP32)) != 0)
    return set_error(JACPCG_E_INVALID_ARG, "unknown request flags");
  const size_t bytes = request_bytes(r.M, r.K, r.n_sub);
  if (s_->budget && bytes > s_->budget)
    return set_error(JACPCG_E_BUDGET, "request needs more device memory than the session budget");
  std::lock_guard<std::mutex> lk(mu_);
  if (stop_) return set_error(JACPCG_E_INVALID_ARG, "session is shutting down");
  start();
  Req q;
  q.r = r;
  q.bytes = bytes;
  q.key.M = r.M;
  q.key.K = r.K;
  q.key.precision = r.precision;
  q.key.flags = r.flags;
  q.key.max_iter = r.max_iter;
  q.key.tol_bits = bits(r.tol);
  q.key.xi_bits = bits(r.xi);
  q.key.power_bits = bits(r.power);
  // The request's device work will wait for what is queued on its stream now
  // (the production of H).
  q.ready = take_event();
  if (!q.ready) return set_error(JACPCG_E_HIP, "creating the request's ready event failed");
  (void)hipSetDevice(s_->device);
  const hipError_t er = hipEventRecord(q.ready, (hipStream_t)r.stream);
  if (er != hipSuccess) {
    (void)hipGetLastError();
    give_event(q.ready);
    return set_error(JACPCG_E_HIP, hipGetErrorString(er));
  }
  q.t_submit = now_us();
  const uint64_t t = next_ticket_++;
  reqs_.emplace(t, q);
  queue_.push_back(t);
  *ticket = t;
  cv_sched_.notify_one();
  return JACPCG_OK;
}

static void fill(jacpcg_result* out, int status, int iters, double ts, double ta, double td, uint64_t tag) {
  out->status = status;
  out->max_iters = iters;
  out->t_submit_us = ts;
  out->t_admit_us = ta;
  out->t_done_us = td;
  out->user_tag = tag;
}

int Scheduler::poll(uint64_t ticket, jacpcg_result* out) {
  if (!out) return set_error(JACPCG_E_INVALID_ARG, "result is NULL");
  std::lock_guard<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return set_error(JACPCG_E_INVALID_ARG, "unknown ticket (never issued or already collected)");
  const Req& q = it->second;
  if (q.state != kDone) {
    fill(out, JACPCG_NOT_READY, 0, q.t_submit, q.t_admit, 0.0, q.r.user_tag);
    return JACPCG_NOT_READY;
  }
  fill(out, q.status, q.max_iters, q.t_submit, q.t_admit, q.t_done, q.r.user_tag);
  reqs_.erase(it);
  return JACPCG_OK;
}

int Scheduler::wait(uint64_t ticket, int timeout_ms, jacpcg_result* out) {
  if (!out) return set_error(JACPCG_E_INVALID_ARG, "result is NULL");
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return set_error(JACPCG_E_INVALID_ARG, "unknown ticket (never issued or already collected)");
  auto ready = [&] {
    auto i = reqs_.find(ticket);
    return i == reqs_.end() || i->second.state == kDone;
  };
  if (timeout_ms < 0)
    cv_done_.wait(lk, ready);
  else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    const Req& q = reqs_.at(ticket);
    fill(out, JACPCG_NOT_READY, 0, q.t_submit, q.t_admit, 0.0, q.r.user_tag);
    return set_error(JACPCG_E_TIMEOUT, "request still in flight");
  }
  it = reqs_.find(ticket);
  if (it == reqs_.end()) return set_error(JACPCG_E_INVALID_ARG, "ticket collected by another caller");
  const Req& q = it->second;
  fill(out, q.status, q.max_iters, q.t_submit, q.t_admit, q.t_done, q.r.user_tag);
  reqs_.erase(it);
  return JACPCG_OK;
}

int Scheduler::cancel(uint64_t ticket) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return set_error(JACPCG_E_INVALID_ARG, "unknown ticket (never issued or already collected)");
  Req& q = it->second;
  if (q.state == kQueued) {
    queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
    give_event(q.ready);
    q.ready = nullptr;
    q.state = kDone;
    q.status = JACPCG_E_CANCELLED;
    q.t_done = now_us();
    cv_done_.notify_all();
  } else if (q.state == kRunning) {
    q.cancelled = true;  // the batch runs to completion; the result reports the cancellation
  }
  return JACPCG_OK;
}

void Scheduler::scheduler_loop() {
  (void)hipSetDevice(s_->device);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    cv_sched_.wait(lk, [&] {
      if (stop_) return true;
      if (queue_.empty()) return false;
      for (auto& sl : slots_)
        if (!sl.busy) return true;
      return false;
    });
    if (stop_) break;
    std::vector<PendingReq> pend;
    for (uint64_t t : queue_) {
      const Req& q = reqs_.at(t);
      pend.push_back({t, q.bytes, q.key});
    }
    const size_t n = admit_prefix(pend, used_, s_->budget);
    if (n == 0) {
      cv_sched_.wait(lk);  // budget exhausted: a completion frees it
      continue;
    }
    pend.resize(n);
    bool launched = false;
    for (const auto& grp : group_by_key(pend)) {
      Slot* free_slot = nullptr;
      for (auto& sl : slots_)
        if (!sl.busy) {
          free_slot = &sl;
          break;
        }
      if (!free_slot) break;
      std::vector<uint64_t> members;
      size_t bytes = 0;
      const double ta = now_us();
      for (size_t i : grp) {
        // The lock was released around the previous group's launch: a request
        // of this group may have been cancelled (and even collected) since
        // the admission list was made. Only requests still queued are admitted.
        const uint64_t t = pend[i].ticket;
        auto it = reqs_.find(t);
        if (it == reqs_.end() || it->second.state != kQueued) continue;
        const auto qi = std::find(queue_.begin(), queue_.end(), t);
        if (qi == queue_.end()) continue;
        queue_.erase(qi);
        members.push_back(t);
        Req& q = it->second;
        q.state = kRunning;
        q.t_admit = ta;
        bytes += q.bytes;
      }
      if (members.empty()) continue;
      used_ += bytes;
      free_slot->busy = true;  // reserved; the completion thread ignores it until armed
      free_slot->bytes = bytes;
      std::vector<jacpcg_request> rq;  // copies: the map may rehash while unlocked
      std::vector<hipEvent_t> ready;
      for (uint64_t t : members) {
        Req& q = reqs_.at(t);
        rq.push_back(q.r);
        ready.push_back(q.ready);
        q.ready = nullptr;
      }
      lk.unlock();
      const int rc = launch(*free_slot, members, rq, ready);
      lk.lock();
      // The slot's stream waits on the events' state at launch; later
      // submissions may record them again.
      for (hipEvent_t e : ready) give_event(e);
      if (rc != JACPCG_OK) {
        for (uint64_t t : members) {
          Req& q = reqs_.at(t);
          q.state = kDone;
          q.status = rc;
          q.t_done = now_us();
        }
        used_ -= bytes;
        free_slot->busy = false;
        cv_done_.notify_all();
      } else {
        free_slot->armed = true;
        ++inflight_;
        launched = true;
      }
    }
    if (launched) cv_comp_.notify_all();
  }
}

int Scheduler::launch(Slot& sl, const std::vector<uint64_t>& members, const std::vector<jacpcg_request>& rq,
                      const std::vector<hipEvent_t>& ready) {
  const PhaseRange range("serve batch");
  (void)hipSetDevice(s_->device);
  const jacpcg_request& r0 = rq[0];
  const int M = r0.M, K = r0.K;
  int G = 0;
  sl.members = members;
  sl.inst_begin.clear();
  for (const auto& r : rq) {
    sl.inst_begin.push_back(G);
    G += r.n_sub;
  }
  sl.instances = G;
  sl.K = K;
  const BatchLayout lay(G, K);
  if (lay.total > sl.ws_bytes) {
    const size_t want = std::max(lay.total, sl.ws_bytes * 2);  // grow geometrically
    if (sl.ws) (void)hipFree(sl.ws);  // the slot is idle: its previous batch completed
    sl.ws = nullptr;
    sl.ws_bytes = 0;
    if (hipMalloc((void**)&sl.ws, want) != hipSuccess) {
      (void)hipGetLastError();
      return JACPCG_E_OUT_OF_MEMORY;
    }
    sl.ws_bytes = want;
  }
  const size_t host_need = (size_t)2 * G * sizeof(void*) + (size_t)G * 4 + (size_t)G * K * 4;
  if (host_need > sl.host_bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.host_bytes = 0;
    if (hipHostMalloc((void**)&sl.host, host_need * 2, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return JACPCG_E_OUT_OF_MEMORY;
    }
    sl.host_bytes = host_need * 2;
  }
  const float2** hp = (const float2**)sl.host;
  float2** wp = (float2**)(sl.host + (size_t)G * sizeof(void*));
  sl.h_status = (int32_t*)(sl.host + (size_t)2 * G * sizeof(void*));
  sl.h_iters = sl.h_status + G;
  bool vec_ok = (M % 2) == 0;
  for (size_t i = 0; i < rq.size(); ++i) {
    const jacpcg_request& r = rq[i];
    for (int s = 0; s < r.n_sub; ++s) {
      hp[sl.inst_begin[i] + s] = (const float2*)r.H + (size_t)s * M * K;
      wp[sl.inst_begin[i] + s] = (float2*)r.W + (size_t)s * M * K;
    }
    vec_ok = vec_ok && ((uintptr_t)r.H % 16 == 0) && ((uintptr_t)r.W % 16 == 0);
  }
  char* ws = sl.ws;
  const float2* const* d_hp = (const float2* const*)(ws + lay.hp);
  float2* const* d_wp = (float2* const*)(ws + lay.wp);
  float2* A = (float2*)(ws + lay.a);
  float* gdiag = (float*)(ws + lay.gd);
  float2* X = (float2*)(ws + lay.x);
  float* fpart = (float*)(ws + lay.fp);
  int32_t* wgs = (int32_t*)(ws + lay.wg);
  int32_t* status = (int32_t*)(ws + lay.st);
  int32_t* iters = (int32_t*)(ws + lay.it);
  float* relres = (float*)(ws + lay.rr);
  const int ncb = (K + 31) / 32;
  const size_t KK = (size_t)K * K;
  hipStream_t st = sl.stream;
  // Every member's H is complete (its producer stream's work at submission).
  hipError_t e = hipSuccess;
  for (hipEvent_t ev : ready)
    if (e == hipSuccess && ev) e = hipStreamWaitEvent(st, ev, 0);
  // The two pointer arrays are adjacent on the host but 256-byte aligned apart
  // on the device: one copy each.
  if (e == hipSuccess) e = hipMemcpyAsync((void*)d_hp, hp, (size_t)G * sizeof(void*), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync((void*)d_wp, wp, (size_t)G * sizeof(void*), hipMemcpyHostToDevice, st);

  GramLaunch g{};
  g.H_ptrs = d_hp;
  g.ldh = M;
  g.batch = G;
  g.M = M;
  g.K = K;
  g.xi = (float)r0.xi;
  g.A = A;
  g.lda = K;
  g.stride_a = (int64_t)KK;
  g.gdiag = gdiag;
  g.precision = r0.precision;
  g.m_split = s_->tuner.gram_waves(M, K, r0.precision);
  g.no_vec = vec_ok ? 0 : 1;
  // Antenna chunks of the FP32 Gram (the launch uses them for the FP32 block
  // kernel only): four times the workgroups, which fills the GPU for a few
  // subcarriers (the layout holds their partial blocks).
  g.msplit = gram_chunks_for(K, G);
  g.partial = g.msplit > 1 ? (float2*)(ws + lay.part) : nullptr;
  if (e == hipSuccess) e = launch_gram(g, st);

  PcgLaunch p{};
  p.A = A;
  p.lda = K;
  p.stride_a = (int64_t)KK;
  p.X = X;
  p.ldx = K;
  p.stride_x = (int64_t)KK;
  p.batch = G;
  p.K = K;
  p.nrhs = K;
  p.tol = (float)r0.tol;
  p.max_iter = r0.max_iter;
  p.precond_none = (r0.flags & JACPCG_PRECOND_NONE) != 0;
  p.iters = iters;
  p.relres = relres;
  p.wg_status = wgs;
  p.gdiag = gdiag;
  p.fpart = fpart;
  p.a_source = s_->tuner.pcg_a_source(K);
  if (e == hipSuccess) e = launch_pcg(p, st, nullptr);

  PrecoderLaunch E{};
  E.H_ptrs = d_hp;
  E.W_ptrs = d_wp;
  E.ldh = M;
  E.ldw = M;
  E.X = X;
  E.ldx = K;
  E.stride_x = (int64_t)KK;
  E.batch = G;
  E.M = M;
  E.K = K;
  E.nrhs = K;
  E.fpart = fpart;
  E.ncb = ncb;
  E.wg_status = wgs;  // the precoder reduces them into the per-instance status
  E.status = status;
  E.power = (float)r0.power;
  E.split = (r0.flags & JACPCG_EPILOGUE_FP32) ? 0 : 3;
  E.nj = s_->tuner.precoder_nj(M, K, E.split);
  E.mtiles = s_->tuner.precoder_mtiles(M, K, E.split);
  E.no_vec = vec_ok ? 0 : 1;
  if (e == hipSuccess) e = launch_precoder(E, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.h_status, status, (size_t)G * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.h_iters, iters, (size_t)G * K * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(sl.done, st);
  if (e != hipSuccess) {
    set_error(JACPCG_E_HIP, hipGetErrorString(e));
    return JACPCG_E_HIP;
  }
  return JACPCG_OK;
}

void Scheduler::finish(Slot& sl) {
  // called with the lock held, after the slot's event completed
  const double td = now_us();
  for (size_t i = 0; i < sl.members.size(); ++i) {
    Req& q = reqs_.at(sl.members[i]);
    int status = JACPCG_OK, it = 0;
    for (int s = 0; s < q.r.n_sub; ++s) {
      const int b = sl.inst_begin[i] + s;
      const int v = sl.h_status[b];
      if (v == kStatusBreakdown) status = JACPCG_E_BREAKDOWN;
      else if (v == kStatusNotConverged && status == JACPCG_OK) status = JACPCG_NOT_CONVERGED;
      for (int j = 0; j < sl.K; ++j) it = std::max(it, (int)sl.h_iters[(size_t)b * sl.K + j]);
    }
    q.state = kDone;
    q.status = q.cancelled ? JACPCG_E_CANCELLED : status;
    q.max_iters = it;
    q.t_done = td;
  }
  used_ -= sl.bytes;
  sl.busy = false;
  sl.armed = false;
  --inflight_;
}

// One completion thread per slot: it sleeps until its slot is armed, then in
// hipEventSynchronize on the slot's blocking-sync event, and publishes the
// batch's results as soon as the event completes (no polling).
void Scheduler::completion_loop(size_t i) {
  (void)hipSetDevice(s_->device);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    cv_comp_.wait(lk, [&] { return stop_ || slots_[i].armed; });
    Slot& sl = slots_[i];
    if (!sl.armed) break;  // stopping, nothing in flight on this slot
    const hipEvent_t ev = sl.done;
    lk.unlock();
    const hipError_t q = hipEventSynchronize(ev);
    lk.lock();
    if (q != hipSuccess) {
      (void)hipGetLastError();
      for (uint64_t t : sl.members) {
        Req& r = reqs_.at(t);
        r.state = kDone;
        r.status = JACPCG_E_HIP;
        r.t_done = now_us();
      }
      used_ -= sl.bytes;
      sl.busy = false;
      sl.armed = false;
      --inflight_;
    } else {
      finish(sl);
    }
    cv_done_.notify_all();
    cv_sched_.notify_one();
  }
}

}  // namespace jacpcg
