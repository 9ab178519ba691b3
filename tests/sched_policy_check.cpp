// Host-only checks of the request scheduler's admission policy.
#include <cassert>
#include <cstdio>

#include "../paper_2305_13925_amd/csrc/sched_policy.hpp"

using namespace jacpcg;

int main() {
  // FIFO prefix under a budget; the first request that does not fit blocks the rest
  std::vector<PendingReq> q = {{1, 100, 7}, {2, 300, 8}, {3, 50, 7}, {4, 10, 9}};
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
  // footprint: H + W plus the batch workspace, monotone in every size
  const size_t b1 = request_bytes(1024, 64, 1), b2 = request_bytes(1024, 64, 2);
  assert(b1 >= (size_t)2 * 1024 * 64 * 8 + (size_t)2 * 64 * 64 * 8);
  assert(b2 > b1 && request_bytes(2048, 64, 1) > b1 && request_bytes(1024, 128, 1) > b1);
  BatchLayout L(3, 40);
  assert(L.hp == 0 && L.wp >= 3 * sizeof(void*) && L.total % 256 == 0 && L.rr < L.total);
  std::printf("sched policy ok\n");
  return 0;
}
