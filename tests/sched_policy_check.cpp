// Host-only checks of the request scheduler's admission policy.
#include <cassert>
#include <cstdio>

#include "../paper_2305_13925_amd/csrc/sched_policy.hpp"

using namespace jacpcg;

static BatchKey key(int M, int K, int max_iter = 16, uint64_t tol_bits = 1) {
  BatchKey k;
  k.M = M;
  k.K = K;
  k.max_iter = max_iter;
  k.tol_bits = tol_bits;
  return k;
}

int main() {
  const BatchKey k7 = key(1024, 64), k8 = key(2048, 64), k9 = key(1024, 128);
  // FIFO prefix under a budget; the first request that does not fit blocks the rest
  std::vector<PendingReq> q = {{1, 100, k7}, {2, 300, k8}, {3, 50, k7}, {4, 10, k9}};
  assert(admit_prefix(q, 0, 0) == 4);        // no budget: everything
  assert(admit_prefix(q, 0, 1000) == 4);
  assert(admit_prefix(q, 0, 399) == 1);      // 100 fits, 100+300 does not, 3 and 4 wait (FIFO)
  assert(admit_prefix(q, 600, 1000) == 2);   // 600 in use: 100 and 300 fit exactly, 50 does not
  assert(admit_prefix(q, 950, 1000) == 0);
  assert(admit_prefix({}, 0, 10) == 0);
  // grouping: keys in first-arrival order, arrival order inside a group
  auto g = group_by_key(q);
  assert(g.size() == 3);
  assert(g[0].size() == 2 && g[0][0] == 0 && g[0][1] == 2);
  assert(g[1].size() == 1 && g[1][0] == 1);
  assert(g[2].size() == 1 && g[2][0] == 3);
  // keys that differ in one field never share a batch; these pairs collided
  // under a 64-bit hash of the fields (M 42/43 at K 59; max_iter 468/502)
  std::vector<PendingReq> c = {{1, 1, key(42, 59)}, {2, 1, key(43, 59)},
                               {3, 1, key(4096, 8, 468)}, {4, 1, key(4096, 8, 502)},
                               {5, 1, key(42, 59)}, {6, 1, key(4096, 8, 468, 2)}};
  BatchKey kf = key(42, 59);
  kf.flags = 1;
  BatchKey kp = key(42, 59);
  kp.precision = 1;
  BatchKey kx = key(42, 59);
  kx.xi_bits = 5;
  BatchKey kw = key(42, 59);
  kw.power_bits = 5;
  c.push_back({7, 1, kf});
  c.push_back({8, 1, kp});
  c.push_back({9, 1, kx});
  c.push_back({10, 1, kw});
  g = group_by_key(c);
  assert(g.size() == 9);
  assert(g[0].size() == 2 && g[0][0] == 0 && g[0][1] == 4);  // the one exact repeat batches together
  for (size_t i = 1; i < g.size(); ++i) assert(g[i].size() == 1);
  // footprint: H + W plus the batch workspace, monotone in every size
  const size_t b1 = request_bytes(1024, 64, 1), b2 = request_bytes(1024, 64, 2);
  assert(b1 >= (size_t)2 * 1024 * 64 * 8 + (size_t)2 * 64 * 64 * 8);
  assert(b2 > b1 && request_bytes(2048, 64, 1) > b1 && request_bytes(1024, 128, 1) > b1);
  BatchLayout L(3, 40);
  assert(L.hp == 0 && L.wp >= 3 * sizeof(void*) && L.total % 256 == 0 && L.rr < L.total);
  std::printf("sched policy ok\n");
  return 0;
}
