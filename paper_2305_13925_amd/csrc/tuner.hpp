// Launch choices of the kernels, keyed by problem shape, with a JSON cache.
// Choices depend only on the shape (never on the batch), so a request's result
// does not depend on what it is batched with. Internally locked: the request
// scheduler's thread reads choices while the caller may autotune.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace jacpcg {

class Tuner {
 public:
  // Waves per Gram workgroup that split the antenna range.
  int gram_waves(int M, int K, int precision) const;
  void set_gram_waves(int M, int K, int precision, int waves);
  // Column tiles per wave of the precoder (0 = the kernel's default rule).
  int precoder_nj(int M, int K, int split) const;
  void set_precoder_nj(int M, int K, int split, int nj);
  bool load(const std::string& path);
  bool save(const std::string& path) const;
  size_t entries() const {
    std::lock_guard<std::mutex> lk(mu_);
    return gram_waves_.size() + precoder_nj_.size();
  }

 private:
  mutable std::mutex mu_;
  std::map<std::tuple<int, int, int>, int> gram_waves_;
  std::map<std::tuple<int, int, int>, int> precoder_nj_;
};

}  // namespace jacpcg
