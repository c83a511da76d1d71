// Shared internals of librcs: error reporting, Philox4x32-10, device helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rcs.h"

namespace rcs {

// ---------------------------------------------------------------- errors
// Every entry point catches rcs::Error and returns its status; the message
// is kept for rcs_last_error().
struct Error : std::runtime_error {
  rcs_status status;
  Error(rcs_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void set_last_error(const char* msg);

[[noreturn]] inline void fail(rcs_status s, const std::string& m) { throw Error(s, m); }

#define RCS_REQUIRE(cond, msg)                                                      \
  do {                                                                              \
    if (!(cond)) ::rcs::fail(RCS_ERR_INVALID_ARG, std::string(__func__) + ": " + (msg)); \
  } while (0)

#define HIP_OK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::rcs::fail(e_ == hipErrorOutOfMemory ? RCS_ERR_OUT_OF_MEMORY : RCS_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                \
    }                                                                                \
  } while (0)

// Checks a kernel launch (configuration errors surface here).
#define HIP_LAUNCH_OK() HIP_OK(hipGetLastError())

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the halves recombined with the other two words
// and the key; the key advances by two Weyl constants between rounds.
struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t w0 = 0x9E3779B9u, w1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)m0 * c.x;
    uint64_t p1 = (uint64_t)m1 * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += w0;
    k1 += w1;
  }
  return c;
}

// Counter streams (word w of the counter).
enum Stream : uint32_t {
  kStreamCircuit = 0,
  kStreamLayout = 1,
  kStreamShots = 2,
  kStreamTestBits = 3,
  kStreamSketch = 4,
  kStreamMlp = 5,
  kStreamBatch = 6
};

// Top 53 bits of the 64-bit word hi:lo as a double in [0, 1).
__host__ __device__ inline double u53(uint32_t lo, uint32_t hi) {
  uint64_t x = ((uint64_t)hi << 32) | lo;
  return (double)(x >> 11) * 0x1.0p-53;
}

// Uniform for shot `shot` at MPS site `site`: counter (shot lo, shot hi,
// site/2, stream 2); words (x, y) serve even sites and (z, w) odd sites.
__host__ __device__ inline double shot_uniform(uint64_t seed, uint64_t shot, int site) {
  U4 c{(uint32_t)shot, (uint32_t)(shot >> 32), (uint32_t)(site >> 1), kStreamShots};
  U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return (site & 1) ? u53(r.z, r.w) : u53(r.x, r.y);
}

// ------------------------------------------------------------ device misc
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// 1/sqrt(x) and 1/x for normal positive (resp. nonzero normal) x: hardware
// estimate plus two Newton steps (each doubles the correct bits; the
// estimate carries about 23), i.e. within a couple of ulps.
__device__ inline double rsqrt_fast(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-h * r, r, 0.5);
  return fma(r, e, r);
}
__device__ inline double rcp_fast(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Stream handle helper.
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace rcs
