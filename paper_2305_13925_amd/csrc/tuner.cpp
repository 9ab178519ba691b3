// Autotuned launch choices with a flat JSON cache:
//   {"gram_waves": [[M, K, precision, waves], ...], "precoder_nj": [[M, K, split, nj], ...]}
#include "tuner.hpp"

#include <cstdio>
#include <fstream>
#include <sstream>

namespace jacpcg {

int Tuner::gram_waves(int M, int K, int precision) const {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = gram_waves_.find(std::make_tuple(M, K, precision));
  if (it != gram_waves_.end()) return it->second;
  (void)K;
  (void)precision;
  // Default: enough waves to split long antenna ranges.
  return M >= 2048 ? 8 : 4;
}

void Tuner::set_gram_waves(int M, int K, int precision, int waves) {
  std::lock_guard<std::mutex> lk(mu_);
  gram_waves_[std::make_tuple(M, K, precision)] = waves;
}

int Tuner::precoder_nj(int M, int K, int split) const {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = precoder_nj_.find(std::make_tuple(M, K, split));
  return it != precoder_nj_.end() ? it->second : 0;
}

void Tuner::set_precoder_nj(int M, int K, int split, int nj) {
  std::lock_guard<std::mutex> lk(mu_);
  precoder_nj_[std::make_tuple(M, K, split)] = nj;
}

namespace {

// Parse the list of 4-integer entries that follows "key" in a flat JSON text.
template <class F>
void parse_list(const std::string& s, const char* key, F&& put) {
  const size_t k = s.find(key);
  if (k == std::string::npos) return;
  size_t pos = s.find('[', k);
  if (pos == std::string::npos) return;
  ++pos;
  while (true) {
    const size_t open = s.find('[', pos);
    const size_t close_outer = s.find(']', pos);
    if (open == std::string::npos || (close_outer != std::string::npos && close_outer < open)) break;
    int v[4];
    if (std::sscanf(s.c_str() + open, "[%d , %d , %d , %d ]", &v[0], &v[1], &v[2], &v[3]) == 4) put(v);
    const size_t close = s.find(']', open);
    if (close == std::string::npos) break;
    pos = close + 1;
  }
}

}  // namespace

bool Tuner::load(const std::string& path) {
  if (path.empty()) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  std::lock_guard<std::mutex> lk(mu_);
  parse_list(s, "\"gram_waves\"", [&](const int* v) {
    if (v[3] >= 1 && v[3] <= 8) gram_waves_[std::make_tuple(v[0], v[1], v[2])] = v[3];
  });
  parse_list(s, "\"precoder_nj\"", [&](const int* v) {
    if (v[3] >= 0 && v[3] <= 2) precoder_nj_[std::make_tuple(v[0], v[1], v[2])] = v[3];
  });
  return true;
}

bool Tuner::save(const std::string& path) const {
  if (path.empty()) return false;
  std::ofstream f(path);
  if (!f) return false;
  std::lock_guard<std::mutex> lk(mu_);
  auto dump = [&](const char* key, const std::map<std::tuple<int, int, int>, int>& m) {
    f << "\"" << key << "\": [";
    bool first = true;
    for (auto& kv : m) {
      f << (first ? "" : ", ") << "[" << std::get<0>(kv.first) << ", " << std::get<1>(kv.first) << ", "
        << std::get<2>(kv.first) << ", " << kv.second << "]";
      first = false;
    }
    f << "]";
  };
  f << "{";
  dump("gram_waves", gram_waves_);
  f << ", ";
  dump("precoder_nj", precoder_nj_);
  f << "}\n";
  return true;
}

}  // namespace jacpcg
