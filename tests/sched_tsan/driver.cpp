// Concurrency check of the request scheduler on the CPU: client threads
// submit, poll, wait for and cancel requests while the scheduler thread admits
// and launches batches and the per-slot completion threads publish results.
// Built with -fsanitize=thread against the host stand-in of the HIP runtime.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_2305_13925_amd/csrc/session.hpp"

using namespace jacpcg;

int main() {
  jacpcg_session s;
  s.device = 0;
  s.budget = (size_t)8 << 20;  // small: admission has to wait for completions
  s.sched.reset(new Scheduler(&s));
  constexpr int kClients = 6, kPerClient = 60;
  std::atomic<int> ok{0}, cancelled{0}, bad{0};
  std::vector<std::thread> clients;
  for (int c = 0; c < kClients; ++c) {
    clients.emplace_back([&, c] {
      std::srand(1000 + c);
      for (int i = 0; i < kPerClient; ++i) {
        jacpcg_request r{};
        r.M = 64 << (std::rand() % 3);
        r.K = 8 << (std::rand() % 3);
        r.n_sub = 1 + std::rand() % 4;
        r.xi = (c % 2) ? 1.6 : 3.2;  // two keys per shape
        r.power = 1.0;
        r.tol = 1e-6;
        r.max_iter = 16;
        const size_t n = (size_t)r.n_sub * r.M * r.K;
        std::vector<float2> H(n, make_float2(0.5f, 0.25f)), W(n, make_float2(0.f, 0.f));
        r.H = reinterpret_cast<const jacpcg_c64*>(H.data());
        r.W = reinterpret_cast<jacpcg_c64*>(W.data());
        uint64_t t = 0;
        if (s.sched->submit(r, &t) != JACPCG_OK) {
          ++bad;
          continue;
        }
        jacpcg_result res{};
        const int mode = std::rand() % 3;
        if (mode == 1) (void)s.sched->cancel(t);
        if (mode == 2) {
          while (s.sched->poll(t, &res) == JACPCG_NOT_READY) std::this_thread::yield();
        } else if (s.sched->wait(t, -1, &res) != JACPCG_OK) {
          ++bad;
          continue;
        }
        if (res.status == JACPCG_OK) {
          bool written = true;  // every instance's precoder was written before the result was final
          for (int b = 0; b < r.n_sub; ++b) written = written && W[(size_t)b * r.M * r.K].x == 1.f;
          written ? ++ok : ++bad;
        } else if (res.status == JACPCG_E_CANCELLED) {
          ++cancelled;
        } else {
          ++bad;
        }
      }
    });
  }
  for (auto& t : clients) t.join();
  s.sched->stop();
  s.sched.reset();
  std::printf("requests ok %d cancelled %d bad %d\n", ok.load(), cancelled.load(), bad.load());
  return (bad.load() == 0 && ok.load() + cancelled.load() == kClients * kPerClient) ? 0 : 1;
}
