// Sampled kernel timing: every `every`-th launch of a timed kernel class is
// timed by start/stop events attached to the launch itself
// (hipExtLaunchKernelGGL), on the stream it is launched on, so the interval
// is the kernel's execution and not the gaps around it.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"

namespace rcs {

enum KernelClass : int {
  kKcChainGemm = 0,   // sampler / amplitude shot GEMM (every launch timed)
  kKcJacGram = 1,     // Jacobi partial Grams
  kKcJacRotate = 2,   // Jacobi inner solve + block rotation
  kKcTwoSite = 3,     // two-site contraction
  kKcRange = 4,       // randomized range-finder products (fp32)
  kKcFactor = 5,      // the other fp64 factorisation kernels (Gram, Cholesky,
                      // triangular inverse, projections, Newton-Schulz, ranks);
                      // every launch is timed, the kernels differ in size
  kKcCount = 6
};

// Launch `kernel` (plain arguments) timed under kernel class kc.
#define RCS_PROBED_LAUNCH(kc, kernel, grid, block, shmem, stream, ...)                                   \
  do {                                                                                                  \
    ::rcs::Probe pr_(kc, stream, 0.0, 0.0);                                                             \
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, pr_.start(), pr_.stop(), 0, __VA_ARGS__); \
  } while (0)

// RAII probe: construct before the launch, pass start()/stop() to
// hipExtLaunchKernelGGL (null when this launch is not sampled), destroy
// after it.
class Probe {
 public:
  Probe(int kclass, hipStream_t s, double flops, double bytes);
  ~Probe();
  Probe(const Probe&) = delete;
  Probe& operator=(const Probe&) = delete;
  hipEvent_t start() const { return e0_; }
  hipEvent_t stop() const { return e1_; }

 private:
  void* entry_ = nullptr;   // its pending record (stable until this probe closes it)
  hipEvent_t e0_ = nullptr, e1_ = nullptr;
};

}  // namespace rcs
