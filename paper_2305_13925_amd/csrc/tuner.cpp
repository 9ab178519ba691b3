// Autotuned launch choices with a flat JSON cache, one list per knob:
//   {"gram_waves": [[M, K, variant, value], ...], "precoder_nj": [...], ...}
#include "tuner.hpp"

#include <cstdio>
#include <fstream>
#include <sstream>

namespace jacpcg {

namespace {
const char* const kNames[kNumKnobs] = {"gram_waves", "precoder_nj", "precoder_mtiles", "pcg_a_source"};
}  // namespace

const char* Tuner::name(int knob) { return (knob >= 0 && knob < kNumKnobs) ? kNames[knob] : ""; }

int Tuner::knob_of(const std::string& n) {
  for (int k = 0; k < kNumKnobs; ++k)
    if (n == kNames[k]) return k;
  return -1;
}

bool Tuner::valid(int knob, int v) {
  if (v == 0) return true;
  switch (knob) {
    case kGramWaves: return v == 2 || v == 4 || v == 8;
    case kPrecoderNj: return v == 1 || v == 2;
    case kPrecoderMtiles: return v == 1 || v == 2 || v == 4;
    case kPcgASource: return v >= 1 && v <= 3;
    default: return false;
  }
}

int Tuner::get(int knob, int M, int K, int variant) const {
  if (knob < 0 || knob >= kNumKnobs) return 0;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = m_[knob].find(std::make_tuple(M, K, variant));
  return it != m_[knob].end() ? it->second : 0;
}

void Tuner::set(int knob, int M, int K, int variant, int value) {
  if (knob < 0 || knob >= kNumKnobs) return;
  std::lock_guard<std::mutex> lk(mu_);
  if (value == 0)
    m_[knob].erase(std::make_tuple(M, K, variant));
  else
    m_[knob][std::make_tuple(M, K, variant)] = value;
}

int Tuner::gram_waves(int M, int K, int precision) const {
  const int v = get(kGramWaves, M, K, precision);
  if (v) return v;
  // Default: enough waves to split long antenna ranges.
  return M >= 2048 ? 8 : 4;
}

size_t Tuner::entries() const {
  std::lock_guard<std::mutex> lk(mu_);
  size_t n = 0;
  for (const auto& m : m_) n += m.size();
  return n;
}

namespace {

// Parse the list of 4-integer entries that follows "key" in a flat JSON text.
template <class F>
void parse_list(const std::string& s, const std::string& key, F&& put) {
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
  for (int knob = 0; knob < kNumKnobs; ++knob) {
    parse_list(s, std::string("\"") + kNames[knob] + "\"", [&](const int* v) {
      if (v[3] != 0 && valid(knob, v[3])) m_[knob][std::make_tuple(v[0], v[1], v[2])] = v[3];
    });
  }
  return true;
}

bool Tuner::save(const std::string& path) const {
  if (path.empty()) return false;
  std::ofstream f(path);
  if (!f) return false;
  std::lock_guard<std::mutex> lk(mu_);
  f << "{";
  for (int knob = 0; knob < kNumKnobs; ++knob) {
    f << (knob ? ", " : "") << "\"" << kNames[knob] << "\": [";
    bool first = true;
    for (auto& kv : m_[knob]) {
      f << (first ? "" : ", ") << "[" << std::get<0>(kv.first) << ", " << std::get<1>(kv.first) << ", "
        << std::get<2>(kv.first) << ", " << kv.second << "]";
      first = false;
    }
    f << "]";
  }
  f << "}\n";
  return true;
}

}  // namespace jacpcg
