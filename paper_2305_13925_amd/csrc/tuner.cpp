// Autotuned launch choices with a flat JSON cache:
//   {"gram_waves": [[M, K, precision, waves], ...]}
#include "tuner.hpp"

#include <cstdio>
#include <fstream>
#include <sstream>
#include <vector>

namespace jacpcg {

int Tuner::gram_waves(int M, int K, int precision) const {
  auto it = gram_waves_.find(std::make_tuple(M, K, precision));
  if (it != gram_waves_.end()) return it->second;
  (void)K;
  (void)precision;
  // Default: enough waves to split long antenna ranges, at least 2 MFMA
  // chains per SIMD for short ones.
  return M >= 2048 ? 8 : 4;
}

void Tuner::set_gram_waves(int M, int K, int precision, int waves) {
  gram_waves_[std::make_tuple(M, K, precision)] = waves;
}

bool Tuner::load(const std::string& path) {
  if (path.empty()) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  const size_t key = s.find("\"gram_waves\"");
  if (key == std::string::npos) return false;
  size_t pos = s.find('[', key);
  if (pos == std::string::npos) return false;
  ++pos;
  while (true) {
    const size_t open = s.find('[', pos);
    const size_t close_outer = s.find(']', pos);
    if (open == std::string::npos || (close_outer != std::string::npos && close_outer < open)) break;
    int v[4];
    if (std::sscanf(s.c_str() + open, "[%d , %d , %d , %d ]", &v[0], &v[1], &v[2], &v[3]) == 4 && v[3] > 0 &&
        v[3] <= 8)
      gram_waves_[std::make_tuple(v[0], v[1], v[2])] = v[3];
    const size_t close = s.find(']', open);
    if (close == std::string::npos) break;
    pos = close + 1;
  }
  return true;
}

bool Tuner::save(const std::string& path) const {
  if (path.empty()) return false;
  std::ofstream f(path);
  if (!f) return false;
  f << "{\"gram_waves\": [";
  bool first = true;
  for (auto& kv : gram_waves_) {
    f << (first ? "" : ", ") << "[" << std::get<0>(kv.first) << ", " << std::get<1>(kv.first) << ", "
      << std::get<2>(kv.first) << ", " << kv.second << "]";
    first = false;
  }
  f << "]}\n";
  return true;
}

}  // namespace jacpcg
