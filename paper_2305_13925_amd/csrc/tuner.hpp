// Launch choices of the kernels, keyed by problem shape, with a JSON cache.
#pragma once

#include <map>
#include <string>
#include <tuple>

namespace jacpcg {

class Tuner {
 public:
  // Waves per Gram workgroup that split the antenna range.
  int gram_waves(int M, int K, int precision) const;
  void set_gram_waves(int M, int K, int precision, int waves);
  bool load(const std::string& path);
  bool save(const std::string& path) const;

 private:
  std::map<std::tuple<int, int, int>, int> gram_waves_;
};

}  // namespace jacpcg
