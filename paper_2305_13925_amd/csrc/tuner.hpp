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

// The tunable launch choices. Each is stored per (M, K, variant), where the
// variant is the Gram precision or the epilogue's split count; 0 means the
// kernel's default rule.
enum Knob {
  kGramWaves = 0,       // waves per Gram workgroup that split the antenna range (2, 4, 8)
  kPrecoderNj = 1,      // column tiles per precoder wave (1, 2)
  kPrecoderMtiles = 2,  // antenna blocks per split-BF16 precoder workgroup (1, 2, 4)
  kPcgASource = 3,      // where the solver keeps A: 1 registers (K <= 64), 2 streamed from L2
  kNumKnobs = 4
};

class Tuner {
 public:
  static const char* name(int knob);
  static int knob_of(const std::string& name);  // -1 when unknown
  // Valid values of a knob (0, the default rule, is always valid).
  static bool valid(int knob, int value);
  int get(int knob, int M, int K, int variant) const;  // 0 when not tuned
  void set(int knob, int M, int K, int variant, int value);

  // The Gram's waves with its default rule applied.
  int gram_waves(int M, int K, int precision) const;
  int precoder_nj(int M, int K, int split) const { return get(kPrecoderNj, M, K, split); }
  int precoder_mtiles(int M, int K, int split) const { return get(kPrecoderMtiles, M, K, split); }
  int pcg_a_source(int K) const { return get(kPcgASource, 0, K, 0); }
  bool load(const std::string& path);
  bool save(const std::string& path) const;
  size_t entries() const;

 private:
  mutable std::mutex mu_;
  std::map<std::tuple<int, int, int>, int> m_[kNumKnobs];
};

}  // namespace jacpcg
