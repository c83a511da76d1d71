// Sampled kernel timing: every `every`-th launch of a timed kernel class is
// bracketed by HIP events on the stream it is launched on.
#pragma once

#include "common.h"

namespace rcs {

enum KernelClass : int {
  kKcChainGemm = 0,   // sampler / amplitude shot GEMM
  kKcJacGram = 1,     // Jacobi partial Grams
  kKcJacRotate = 2,   // Jacobi inner solve + block rotation
  kKcTwoSite = 3,     // two-site contraction
  kKcRange = 4,       // randomized range-finder products (fp32)
  kKcCount = 5
};

// RAII probe: construct before the launch, destroy after it.
class Probe {
 public:
  Probe(int kclass, hipStream_t s, double flops, double bytes);
  ~Probe();
  Probe(const Probe&) = delete;
  Probe& operator=(const Probe&) = delete;

 private:
  int slot_ = -1;
  hipStream_t s_ = nullptr;
};

}  // namespace rcs
