// Device-resident MPS state and the internal launch interfaces.
#pragma once

#include <memory>
#include <vector>

#include "common.h"

namespace rcs {

// Device buffer owned by RAII (hipFree on destruction).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Grows (never shrinks) to at least `need` bytes; contents are not kept.
  void ensure(size_t need) {
    if (need <= bytes) return;
    release();
    HIP_OK(hipMalloc(&p, need));
    bytes = need;
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

struct SpectrumRecord {
  int32_t pos, cycle, m, kept, chi_l, chi_r;
  std::vector<double> values;  // descending
};

// Shape of one two-site update (always recorded; a few ints per update).
// path: 0 full fp64 SVD, 1 randomized split accepted, 2 randomized split
// rejected and redone with the full SVD.
struct UpdateRecord {
  int32_t pos, cycle, chi_l, chi_m, chi_r, kept, path;
};

// Decisions of one randomized split (learned / rsvd-at-cap modes).
struct RsvdRecord {
  int32_t update, pos, cycle, m, k_hat, l, k, accepted, early;
  double eps_pred, eps_rand, outside, total;
  float feat[66];
  float y[32];
  std::vector<double> values;  // projected spectrum (descending), logging builds only
};

}  // namespace rcs

// Site tensor k lives in site[k] with layout [s][a][b] (physical index
// outermost, then a row-major dims[k] x dims[k+1] matrix), complex128
// interleaved.  Capacity of site k is cap[k] * 2 * cap[k+1] complex values,
// cap[b] = min(2^b, 2^(n-b), chi) for bond b.
struct rcs_state_s {
  int n = 0;
  int chi = 0;
  std::vector<int> pi;      // position -> qubit
  std::vector<int> dims;    // n + 1 bond dimensions, dims[0] = dims[n] = 1
  std::vector<int> cap;     // n + 1 capacities
  std::vector<double2*> site;
  rcs::DevBuf slab;         // all site tensors
  rcs::DevBuf spare;        // one extra site-sized buffer (ping-pong)
  double2* spare_ptr = nullptr;
  int center = 0;
  bool canonical = false;
  hipStream_t stream = nullptr;
  int device = 0;
  // bookkeeping
  int n_trunc = 0, n_fallback = 0, n_rsvd_ok = 0, jacobi_sweeps_max = 0;
  int n_rsvd_early = 0;   // fall-backs decided before the projected SVD
  double log_fest = 0.0, sum_eps = 0.0;
  double build_seconds = 0.0, svd_seconds = 0.0;
  int n_moves = 0;
  int n_precond = 0, n_precond_fallback = 0;   // preconditioned splits, and those redone plainly
  int n_moves_cholqr = 0;                        // centre moves done by CholeskyQR
  int n_svd_f32 = 0, n_svd_f32_redone = 0;       // fp32 Jacobi splits, and those redone in fp64
  double nominal_svd_flops = 0.0, nominal_qr_flops = 0.0;
  std::vector<rcs::SpectrumRecord> spectra;
  std::vector<rcs::UpdateRecord> updates;
  std::vector<rcs::RsvdRecord> rsvd_log;
  // sampler workspace (grown on demand)
  rcs::DevBuf wbuf[2], part, sel, lastp, vnorm, idx1;
};

namespace rcs {

// Allocates site storage for bond caps; sets all sites to |0>.
void state_alloc(rcs_state_s& st, int n, int chi);
size_t site_capacity(const rcs_state_s& st, int k);

// Sampler / amplitude engine: runs the per-site shot GEMMs.
//   mode 0: sample (bits_dev written), mode 1: amplitudes for given bits.
// run_chain grows the state's own workspace; run_chain_with uses the given
// buffers (S0 shots per pass) and allocates nothing.
struct ChainBuffers {
  double2* w[2] = {nullptr, nullptr};
  double* part = nullptr;
  int8_t* sel = nullptr;     // chosen branch, written at even sites
  int8_t* sel2 = nullptr;    // chosen branch, written at odd sites
  double* vnorm = nullptr;   // per-shot ||v||^2 (split sites)
  int* idx1 = nullptr;       // shots that chose 1 at a split site
  int* n1 = nullptr;         // their count
  int64_t S0 = 0;
};
int state_max_bond(const rcs_state_s& st);
size_t chain_work_bytes(int64_t S, int maxd);
ChainBuffers chain_buffers_in(char* base, int64_t S, int maxd);
void run_chain(rcs_state_s& st, uint64_t first_shot, uint64_t n_shots, uint64_t seed, int mode,
               uint64_t* bits_dev, double* log2p_dev, const uint64_t* in_bits_dev,
               double* amps_dev);
void run_chain_with(rcs_state_s& st, const ChainBuffers& buf, uint64_t first_shot, uint64_t n_shots,
                    uint64_t seed, int mode, uint64_t* bits_dev, double* log2p_dev,
                    const uint64_t* in_bits_dev, double* amps_dev, bool probe = true);

// Same shots as run_chain (mode 0) with the workspace in the library's
// static per-device scratch array: no device allocation.
void run_chain_noalloc(rcs_state_s& st, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                       uint64_t* bits_dev, double* log2p_dev);
size_t noalloc_scratch_bytes();
int64_t noalloc_pass_shots(int maxd);

// Shots from several states: grouped launches captured in one HIP graph.
void run_chain_batch(rcs_state_s** states, int n, uint64_t n_shots, uint64_t seed, uint64_t* bits_dev,
                     double* log2p_dev, hipStream_t user_stream);

// out[i] = |z[i]|^2.
void abs2_to(const double2* z, uint64_t m, double* out, hipStream_t stream);

// Linear XEB from device probabilities (is_log2: values are log2 p).
void xeb_reduce(int n_qubits, const double* vals_dev, uint64_t m, bool is_log2, double* xeb,
                double* se, hipStream_t stream);

}  // namespace rcs
