// Internal interface of the triangular preconditioner (Gram, blocked
// Cholesky, Y = R^H) of the fp64 Jacobi SVD, and two small helpers of the
// preconditioned split.
#pragma once

#include "common.h"

namespace rcs {

// G (ldg x ldg, ldg a multiple of 64 and >= n) <- the Cholesky factor of
// X^H X (X: len x n, ld ldx) in its upper triangle (off-diagonal blocks) and
// Rd (ldg/64 blocks of 64 x 64, diagonal blocks); Y (ldy x ycols) <- R^H
// zero-padded.  *flag_dev is set to 1 (never cleared here) when a pivot is
// not positive, i.e. X is numerically rank deficient.
void chol_precondition(const double2* X, int ldx, int len, int n, double2* G, int ldg, double2* Rd, double2* Y,
                       int ldy, int ycols, int* flag_dev, hipStream_t s);
// CholeskyQR: R from the Cholesky factor of X^H X (X: len x n, ld ldx),
// R^{-1} in Ri (ldg x ldg, upper, by recursive doubling of its 64 x 64
// diagonal blocks; T is ldg x ldg scratch), Q = X R^{-1} (ld ldq).  Q is
// orthonormal up to about u cond(X)^2; *flag_dev is set on a non-positive
// pivot.
void cholqr(const double2* X, int ldx, int len, int n, double2* G, int ldg, double2* Rd, double2* Ri, double2* T,
            double2* Q, int ldq, int* flag_dev, hipStream_t s);
// *dev = max entry of |H - I|, H k x k row-major (one workgroup).
void max_dev_identity(const double2* H, int k, double* dev, hipStream_t s);
// P (k x len, row-major) = scale (X U)^H; X len x n (ld ldx), U n x k (ld ldu).
void project_rows(const double2* U, int ldu, const double2* X, int ldx, int len, int n, int k, double scale,
                  double2* P, hipStream_t s);
// out[:, j] = in[:, j] with row i moved to row order[i], for j < k.
void unpermute_rows(const double2* in, int ld, int n, int k, const int* order, double2* out, hipStream_t s);

}  // namespace rcs
