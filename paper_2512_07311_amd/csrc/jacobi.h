// Internal interface of the fp64 one-sided block Jacobi SVD.
#pragma once

#include "common.h"

namespace rcs {

struct JacobiPlan {
  int len = 0, cnt = 0;   // matrix is len x cnt
  int ldx = 0;            // leading dimension (rows, padded to 64)
  int nbp = 0;            // number of 32-column blocks (even)
  int cnt_pad = 0;        // nbp * 32 columns allocated
  int n_pairs = 0;
  int n_chunks = 0, rows_per_chunk = 0;
};

JacobiPlan jacobi_plan(int len, int cnt);
size_t jacobi_work_bytes(const JacobiPlan& pl);
void jacobi_init_attributes();
// Orthogonalises the columns of x in place; returns the number of sweeps
// (the last one rotates nothing).  fro2 scales the absolute zero floor.
int jacobi_run(const JacobiPlan& pl, double2* x, void* work, int* rot_count_dev,
               int* rot_count_host, double fro2, hipStream_t stream, int max_sweeps);

}  // namespace rcs
