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
};

struct BuildWork;
BuildWork* new_work();
void delete_work(BuildWork* w);

// Runs the schedule of circuit c on the freshly allocated state st.
void build_dispatch(rcs_state_s& st, const rcs_circuit_s& c, int chi, double eps,
                    const BuildOptions& o, BuildWork& ws);
void build_one(rcs_state_s& st, const rcs_circuit_s& c, int chi, double eps, const BuildOptions& o,
               BuildWork& ws);

}  // namespace rcs
