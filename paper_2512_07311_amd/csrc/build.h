// Internal interface of the state builder.
#pragma once

#include <vector>

#include "circuit.h"
#include "state.h"

namespace rcs {

struct BuildOptions {
  int contraction = RCS_PREC_C128;
  int rank_mode = RCS_RANK_FULL_SVD;
  double fallback_tau = 1e-6;
  std::vector<float> mlp;
  int rsvd_p = 16, rsvd_q = 2;
  uint64_t rsvd_seed = 0;
  void* stream = nullptr;
  bool log_spectra = false;
  int max_ops = -1;
  bool canonicalize = true;
  bool svd_f32 = false;      // RCS_SVD_F32
};

struct BuildWork;
BuildWork* new_work();
void delete_work(BuildWork* w);

// Runs the schedule of circuit c on the freshly allocated state st.
void build_one(rcs_state_s& st, const rcs_circuit_s& c, int chi, double eps, const BuildOptions& o,
               BuildWork& ws);

// Learned-rank network pieces (fp32).
void spectrum_features(const double* s_dev, int k, int bond, int n_sites, int cycle, int n_cycles,
                       float* feat_dev, hipStream_t st);
void mlp_forward(const float* w, const float* x, int batch, float* out, float* act, hipStream_t s);

// Reduced-precision two-site products (complex64 or split-bf16 on MFMA).
void contract_two_site_lowp(const double2* A, const double2* B, double2* T, int dl, int dm, int dr,
                            int precision, hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

}  // namespace rcs
