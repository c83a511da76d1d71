// Internal interface of the randomized range finder.
#pragma once

#include "state.h"

namespace rcs {

constexpr int kMaxKChunks = 16;   // row chunks of the Gram-Schmidt projections

struct RsvdWork {
  DevBuf bufQ, bufZ, bufC, bufCp, bufPp, bufG, bufR, bufGs;
  double2 *Q = nullptr, *Z = nullptr, *C = nullptr, *Cpart = nullptr, *Ppart = nullptr, *gpart = nullptr,
          *Rinv = nullptr, *gsum = nullptr;
  int ldq = 0, ldz = 0, ldc = 0;
};

void rsvd_work_ensure(RsvdWork& w, int len, int cnt, int l);
// Q (in w) <- orthonormal basis of the sketched range of M (len x cnt).
void range_finder(const double2* M, int ldx, int len, int cnt, int l, int q, uint64_t seed, uint64_t step,
                  RsvdWork& w, hipStream_t s);
// X = X0 = M^H Q  (cnt x l, col-major, leading dimension ldxo), fp64.
void project_to_basis(const double2* M, int ldx, int len, int cnt, int l, const RsvdWork& w, double2* X,
                      double2* X0, int ldxo, hipStream_t s);
// A_i[s1][a][j] = (Q conj(P)^T)[(s1, a)][j] for the k kept columns.
void basis_times_pc(const RsvdWork& w, int len, int l, const double2* P, int k, int dl, double2* Ai, hipStream_t s);

}  // namespace rcs
