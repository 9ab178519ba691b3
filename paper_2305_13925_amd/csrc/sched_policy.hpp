// Host-side policy of the request scheduler: request footprint, FIFO admission
// under the HBM budget and grouping into batches. Plain C++ (no HIP), so it is
// unit-tested on the host.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace jacpcg {

// What requests must share to run as one batch: the shape and every solve
// setting, compared field by field (floating-point settings by their bits, so
// two requests batch together only when the kernels would see identical
// arguments).
struct BatchKey {
  int M = 0, K = 0, precision = 0, flags = 0, max_iter = 0;
  uint64_t tol_bits = 0, xi_bits = 0, power_bits = 0;
  bool operator==(const BatchKey& o) const {
    return M == o.M && K == o.K && precision == o.precision && flags == o.flags && max_iter == o.max_iter &&
           tol_bits == o.tol_bits && xi_bits == o.xi_bits && power_bits == o.power_bits;
  }
  bool operator!=(const BatchKey& o) const { return !(*this == o); }
};

struct PendingReq {
  uint64_t ticket;
  size_t bytes;
  BatchKey key;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device workspace of one batch of G instances with K users, in launch order:
// instance pointer arrays, A, diag(H^H H), X, per-workgroup partials and
// statuses, per-column iterations and residuals, and above K = 128 the
// partial 64 x 64 blocks of an FP32 Gram summed over kGramChunks antenna
// chunks.
// Four chunks above K = 128, and above K = 64 when the batch has fewer than
// 512 blocks of A (two per compute unit): the chunks then fill idle compute
// units. (With every block resident at once, as 256 instances of K = 128 are,
// chunks only add the partial sums.)
constexpr int kGramChunks = 4;
inline int gram_chunks_for(int K, int batch) {
  const int nb = (K + 63) / 64;
  const long items = (long)batch * (nb * (nb + 1) / 2);
  return (K > 128 || (K > 64 && items < 512)) ? kGramChunks : 1;
}
struct BatchLayout {
  size_t hp, wp, a, gd, x, fp, wg, st, it, rr, part, total;
  BatchLayout(int G, int K) {
    const int ncb = (K + 31) / 32;
    size_t o = 0;
    auto take = [&](size_t bytes) {
      const size_t off = o;
      o = align256(o + bytes);
      return off;
    };
    hp = take((size_t)G * sizeof(void*));
    wp = take((size_t)G * sizeof(void*));
    a = take((size_t)G * K * K * 8);
    gd = take((size_t)G * K * 4);
    x = take((size_t)G * K * K * 8);
    fp = take((size_t)G * ncb * 4);
    wg = take((size_t)G * ncb * 4);
    st = take((size_t)G * 4);
    it = take((size_t)G * K * 4);
    rr = take((size_t)G * K * 4);
    const int nb = (K + 63) / 64, chunks = gram_chunks_for(K, G);
    part = chunks > 1 ? take((size_t)G * (nb * (nb + 1) / 2) * chunks * 64 * 64 * 8) : 0;
    total = o;
  }
};

// Device bytes a request holds while admitted: H in, W out and its workspace.
inline size_t request_bytes(int M, int K, int n_sub) {
  const size_t io = (size_t)2 * n_sub * M * K * 8;
  return io + BatchLayout(n_sub, K).total;
}

// FIFO admission under a budget (0 = unlimited): the longest prefix of `queue`
// whose bytes fit next to `used`. Strict FIFO: a request that does not fit
// blocks the ones behind it, so large requests cannot starve.
inline size_t admit_prefix(const std::vector<PendingReq>& queue, size_t used, size_t budget) {
  size_t n = 0;
  for (const auto& q : queue) {
    if (budget && used + q.bytes > budget) break;
    used += q.bytes;
    ++n;
  }
  return n;
}

// Admitted requests grouped by key (shape and solve settings, every field
// equal); groups ordered by their first request, requests in arrival order
// inside a group.
inline std::vector<std::vector<size_t>> group_by_key(const std::vector<PendingReq>& admitted) {
  std::vector<std::vector<size_t>> groups;
  std::vector<BatchKey> keys;
  for (size_t i = 0; i < admitted.size(); ++i) {
    size_t g = 0;
    while (g < keys.size() && keys[g] != admitted[i].key) ++g;
    if (g == keys.size()) {
      keys.push_back(admitted[i].key);
      groups.emplace_back();
    }
    groups[g].push_back(i);
  }
  return groups;
}

}  // namespace jacpcg
