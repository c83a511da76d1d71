// Internal interface of the one-sided block Jacobi SVD (fp64 and fp32).
#pragma once

#include "common.h"

namespace rcs {

struct JacobiPlan {
  int jb = 16;            // columns per block (16 or 32)
  int inner = 1;          // inner sweeps per pair meeting
  int len = 0, cnt = 0;   // matrix is len x cnt
  int ldx = 0;            // leading dimension (rows, padded to 64)
  int nbp = 0;            // number of column blocks (even)
  int cnt_pad = 0;        // nbp * 32 columns allocated
  int n_pairs = 0;
  int n_chunks = 0, rows_per_chunk = 0;     // rotate pass row chunks
  int n_gchunks = 0, rows_per_gchunk = 0;   // Gram pass row chunks
};

// jb <= 0 picks the default block width for the shape.
JacobiPlan jacobi_plan(int len, int cnt, int jb = 0);
size_t jacobi_work_bytes(const JacobiPlan& pl);
// Orthogonalises the columns of x in place; returns the number of sweeps
// (the last one rotates nothing, or its largest entering cosine squared is
// below tol / 100, after which the next would rotate nothing: quadratic
// convergence).  fro2 = ||x||_F^2; columns below
// 8 u sqrt(len) ||x||_F count as numerically zero.
// tol > 0 replaces the default relative orthogonality tolerance 16 u sqrt(len).
// rot_count_dev and rot_count_host hold two ints (rotation count; whether a
// meeting of the sweep entered with a squared cosine above tol / 100).
int jacobi_run(const JacobiPlan& pl, double2* x, void* work, int* rot_count_dev,
               int* rot_count_host, double fro2, hipStream_t stream, int max_sweeps, double tol = 0.0);
// The same in fp32 (complex64 columns, u = 2^-24); work as sized by
// jacobi_work_bytes.
int jacobi_run_f32(const JacobiPlan& pl, float2* x, void* work, int* rot_count_dev,
                   int* rot_count_host, double fro2, hipStream_t stream, int max_sweeps, double tol = 0.0);

}  // namespace rcs
