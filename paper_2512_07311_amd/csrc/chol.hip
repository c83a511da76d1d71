// Triangular preconditioner for the one-sided Jacobi SVD: the Gram matrix
// G = X^H X of the two-site matrix, its Cholesky factor G = R^H R (R upper
// triangular), and Y = R^H in the Jacobi layout.
//
// X = Q R for some orthonormal Q, so X and R share singular values and right
// singular vectors.  One-sided Jacobi on Y = R^H converges in far fewer
// sweeps than on X (Drmac & Veselic, "New fast and accurate Jacobi SVD
// algorithm", SIAM J. Matrix Anal. Appl. 29, 2008: the triangular factor is
// one QR-iteration step closer to diagonal), and it leaves Y J = U_Y S with
// U_Y the right singular vectors of X, so neither Q nor the accumulated
// rotations J are needed.  R comes from the Gram rather than a Householder
// QR, which costs relative accuracy below the Gram's rounding level
// (singular values under ~1e-6 of the largest); the caller accepts the
// result only where that level cannot change the truncation, and otherwise
// runs the Jacobi on X itself.
//
// The factorisation is blocked by 64 columns, right-looking:
//   panel kernel:  every workgroup factors the 64 x 64 diagonal block of G
//                  in LDS (redundantly); workgroup 0 stores R_jj in a
//                  separate array (the others are still reading G_jj), the
//                  others invert R_jj in place and solve their 64-column tile
//                  of the block row, R_jt = R_jj^{-H} G_jt;
//   update kernel: G_tu -= R_jt^H R_ju for the upper tiles of the trailing
//                  matrix, on the matrix cores.
// G is stored column-major with ld = round_up(n, 64); the padding carries an
// identity diagonal so that the padded matrix factors as blockdiag(R, I).
#include "chol.h"
#include "gemm_f64.h"
#include "prof.h"

namespace rcs {

constexpr int CB = 64;          // Cholesky block
constexpr int CHOL_THREADS = 256;

// G (ld ldg, column-major) = X^H X over the upper tiles (blockIdx.y <=
// blockIdx.x); entries outside n x n are the identity's.
__global__ __launch_bounds__(GT_THREADS) void k_gram_upper(const double2* X, int ldx, int len, int n,
                                                          double2* G, int ldg) {
  if (blockIdx.y > blockIdx.x) return;
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int kk) -> double2 {
    const double2 v = X[(int64_t)m * ldx + kk];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int kk, int c) -> double2 { return X[(int64_t)c * ldx + kk]; };
  LoadA<decltype(fa), true> la{fa, m0, n, len};
  LoadB<decltype(fb), false> lb{fb, n0, len, n};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, len, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r, col = n0 + c;
    double2 v = make_double2(re, im);
    if (m >= n || col >= n) v = make_double2(m == col ? 1.0 : 0.0, 0.0);
    G[(int64_t)col * ldg + m] = v;
  });
}

__device__ inline double2 cmul_c(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline double2 cmul_hc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Panel jb, 256 threads per workgroup: thread (q, c) = (t / 64, t % 64)
// works on column c of the 64 x 64 blocks in LDS and on the rows (or sum
// terms) congruent to q mod 4, so the four waves share each step's work:
//  * every workgroup factors the diagonal block G_jj = R^H R (right-looking:
//    at step k row k of R is formed once in a separate buffer, then each
//    thread updates its rows of its column's trailing part); a pivot that is
//    not positive and finite sets *flag;
//  * workgroup 0 stores R_jj (column-major in Rd) and, when Ri is given, the
//    diagonal block of R^{-1} (back substitution on every column at once);
//  * workgroup t >= 1 solves its tile of the block row, R_jt = R^{-H} G_jt,
//    by forward substitution on every column at once.
// The substitutions sum their terms in four interleaved partial sums,
// combined in a fixed order.
constexpr int PANEL_THREADS = 256;

// B[r][cc] = G[row0 + r][col0 + cc] (G column-major, ld ldg) for a 64 x 64
// block: each thread loads four columns' entries of one row, sixteen loads
// in flight before their LDS stores.
__device__ inline void load_block64(const double2* G, int ldg, int row0, int col0, double2 (*B)[CB + 1]) {
  const int r = threadIdx.x & (CB - 1), q = threadIdx.x >> 6;
  double2 v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = G[(int64_t)(col0 + q + 4 * u) * ldg + row0 + r];
#pragma unroll
  for (int u = 0; u < 16; ++u) B[r][q + 4 * u] = v[u];
}

__global__ __launch_bounds__(PANEL_THREADS) void k_chol_panel(double2* G, int ldg, int jb, int* flag, double2* Rd,
                                                              double2* Ri) {
  __shared__ double2 T[CB][CB + 1];
  __shared__ double2 A[CB][CB + 1];
  __shared__ double2 rowk[CB];
  __shared__ double2 part[4][CB];
  const int c = threadIdx.x & (CB - 1), q = threadIdx.x >> 6;
  const int j0 = jb * CB;
  load_block64(G, ldg, j0, j0, T);
  __syncthreads();
  for (int k = 0; k < CB; ++k) {
    double d = T[k][k].x;
    const bool bad = !(d > 0.0) || !(d < 1e300);
    if (bad) d = 1.0;
    if (bad && threadIdx.x == 0) atomicExch(flag, 1);
    const double r = sqrt(d), inv = 1.0 / r;
    if (q == 0 && c >= k) rowk[c] = c == k ? make_double2(r, 0.0) : make_double2(T[k][c].x * inv, T[k][c].y * inv);
    __syncthreads();
    if (q == 0 && c >= k) T[k][c] = rowk[c];
    if (c > k) {
      const double2 rc = rowk[c];
      for (int rr = k + 1 + q; rr <= c; rr += 4) {
        const double2 p = cmul_hc(rowk[rr], rc);
        T[rr][c] = make_double2(T[rr][c].x - p.x, T[rr][c].y - p.y);
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    double2* rd = Rd + (int64_t)jb * CB * CB;
    for (int cc = q; cc < CB; cc += 4) rd[cc * CB + c] = c <= cc ? T[c][cc] : make_double2(0.0, 0.0);
    if (Ri) {
      // column c of R^{-1}: x_c = 1 / R_cc; x_i = -(sum_{m=i+1}^{c} R_im x_m) / R_ii, i < c
      if (q == 0) A[c][c] = make_double2(1.0 / T[c][c].x, 0.0);
      __syncthreads();
      for (int i = CB - 2; i >= 0; --i) {
        double2 s2 = make_double2(0.0, 0.0);
        if (c > i)
          for (int m = i + 1 + q; m <= c; m += 4) {
            const double2 p = cmul_c(T[i][m], A[m][c]);
            s2.x += p.x;
            s2.y += p.y;
          }
        part[q][c] = s2;
        __syncthreads();
        if (q == 0 && c > i) {
          const double2 t0 = part[0][c], t1 = part[1][c], t2 = part[2][c], t3 = part[3][c];
          const double sx = (t0.x + t1.x) + (t2.x + t3.x), sy = (t0.y + t1.y) + (t2.y + t3.y);
          const double qq = -1.0 / T[i][i].x;
          A[i][c] = make_double2(qq * sx, qq * sy);
        }
        __syncthreads();
      }
      for (int cc = q; cc < CB; cc += 4)
        Ri[(int64_t)(j0 + cc) * ldg + j0 + c] = c <= cc ? A[c][cc] : make_double2(0.0, 0.0);
    }
    return;
  }
  const int t0 = j0 + blockIdx.x * CB;    // first column of this tile
  load_block64(G, ldg, j0, t0, A);
  __syncthreads();
  // R^H X = A, column c: X_i = (A_i - sum_{m<i} conj(R_mi) X_m) / R_ii
  for (int i = 0; i < CB; ++i) {
    double2 s2 = make_double2(0.0, 0.0);
    for (int m = q; m < i; m += 4) {
      const double2 p = cmul_hc(T[m][i], A[m][c]);
      s2.x += p.x;
      s2.y += p.y;
    }
    part[q][c] = s2;
    __syncthreads();
    if (q == 0) {
      const double2 t0p = part[0][c], t1 = part[1][c], t2 = part[2][c], t3 = part[3][c];
      const double sx = (t0p.x + t1.x) + (t2.x + t3.x), sy = (t0p.y + t1.y) + (t2.y + t3.y);
      const double qq = 1.0 / T[i][i].x;
      A[i][c] = make_double2(qq * (A[i][c].x - sx), qq * (A[i][c].y - sy));
    }
    __syncthreads();
  }
  for (int cc = q; cc < CB; cc += 4) G[(int64_t)(t0 + cc) * ldg + j0 + c] = A[c][cc];
}

// Trailing update after panel jb: tile (ti, tj), jb < ti <= tj < nb:
// G_{ti,tj} -= R_{jb,ti}^H R_{jb,tj}.  blockIdx.x enumerates the pairs.
__global__ __launch_bounds__(GT_THREADS) void k_chol_update(double2* G, int ldg, int nb, int jb) {
  __shared__ SmemC64 sm;
  const int T = nb - jb - 1;
  // pair index -> (ti, tj) with ti <= tj, row-major over the upper triangle
  int p = blockIdx.x, ti = 0;
  while (p >= T - ti) {
    p -= T - ti;
    ++ti;
  }
  const int tj = ti + p;
  const int r0 = (jb + 1 + ti) * CB, c0 = (jb + 1 + tj) * CB, k0 = jb * CB;
  auto fa = [&](int m, int kk) -> double2 {
    const double2 v = G[(int64_t)(r0 + m) * ldg + k0 + kk];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int kk, int n) -> double2 { return G[(int64_t)(c0 + n) * ldg + k0 + kk]; };
  LoadA<decltype(fa), true> la{fa, 0, CB, CB};
  LoadB<decltype(fb), false> lb{fb, 0, CB, CB};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, CB, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    double2* g = G + (int64_t)(c0 + c) * ldg + r0 + r;
    *g = make_double2(g->x - re, g->y - im);
  });
}

// Y (ldy x ncols, column-major) = R^H in the leading n x n block, zero
// elsewhere; R's diagonal blocks are in Rd (64 x 64 each, column-major), its
// off-diagonal blocks in the upper triangle of G.
__global__ void k_chol_to_y(const double2* G, int ldg, const double2* Rd, int n, double2* Y, int ldy, int ncols) {
  const int64_t tot = (int64_t)ldy * ncols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % ldy), j = (int)(e / ldy);
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n && i >= j) {
      // R[j][i], row j, column i
      const double2 r = (i / CB == j / CB) ? Rd[(int64_t)(j / CB) * CB * CB + (i % CB) * CB + (j % CB)]
                                           : G[(int64_t)i * ldg + j];
      v = make_double2(r.x, -r.y);
    }
    Y[e] = v;
  }
}

// Gram and blocked Cholesky (R's off-diagonal blocks in G, diagonal blocks
// in Rd, diagonal blocks of R^{-1} in Ri when Ri is not null).
static void gram_cholesky(const double2* X, int ldx, int len, int n, double2* G, int ldg, double2* Rd, double2* Ri,
                          int* flag_dev, hipStream_t s) {
  RCS_REQUIRE(ldg % CB == 0 && ldg >= n, "Gram leading dimension must be a multiple of 64");
  const int nb = ldg / CB;
  RCS_PROBED_LAUNCH(kKcFactor, k_gram_upper, dim3(nb, nb), dim3(GT_THREADS), 0, s, X, ldx, len, n, G, ldg);
  HIP_LAUNCH_OK();
  for (int jb = 0; jb < nb; ++jb) {
    RCS_PROBED_LAUNCH(kKcFactor, k_chol_panel, dim3(nb - jb), dim3(PANEL_THREADS), 0, s, G, ldg, jb, flag_dev, Rd, Ri);
    HIP_LAUNCH_OK();
    const int T = nb - jb - 1;
    if (T > 0) {
      RCS_PROBED_LAUNCH(kKcFactor, k_chol_update, dim3(T * (T + 1) / 2), dim3(GT_THREADS), 0, s, G, ldg, nb, jb);
      HIP_LAUNCH_OK();
    }
  }
}

void chol_precondition(const double2* X, int ldx, int len, int n, double2* G, int ldg, double2* Rd, double2* Y,
                       int ldy, int ycols, int* flag_dev, hipStream_t s) {
  gram_cholesky(X, ldx, len, n, G, ldg, Rd, nullptr, flag_dev, s);
  const int64_t tot = (int64_t)ldy * ycols;
  RCS_PROBED_LAUNCH(kKcFactor, k_chol_to_y, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 65535)), dim3(256), 0, s, G,
                     ldg, Rd, n, Y, ldy, ycols);
  HIP_LAUNCH_OK();
}

// Batched column-major complex GEMM on sub-blocks: for batch z,
// D_z = alpha A_z B_z with A_z = A + z sa (M x K, ld lda), B_z = B + z sb
// (K x N, ld ldb), D_z = D + z sd (M x N, ld ldd), overwritten.
__global__ __launch_bounds__(GT_THREADS) void k_cgemm_cm(const double2* A, int lda, int64_t sa, const double2* B,
                                                        int ldb, int64_t sb, double2* D, int ldd, int64_t sd, int M,
                                                        int N, int K, double alpha) {
  __shared__ SmemC64 sm;
  const int64_t z = blockIdx.z;
  const double2* a = A + z * sa;
  const double2* b = B + z * sb;
  double2* d = D + z * sd;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int k) -> double2 { return a[(int64_t)k * lda + m]; };
  auto fb = [&](int k, int n) -> double2 { return b[(int64_t)n * ldb + k]; };
  LoadA<decltype(fa), false> la{fa, m0, M, K};
  LoadB<decltype(fb), false> lb{fb, n0, K, N};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, K, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r, n = n0 + c;
    if (m < M && n < N) d[(int64_t)n * ldd + m] = make_double2(alpha * re, alpha * im);
  });
}

static void cgemm_cm(const double2* A, int lda, int64_t sa, const double2* B, int ldb, int64_t sb, double2* D,
                     int ldd, int64_t sd, int M, int N, int K, double alpha, int batch, hipStream_t s) {
  if (batch <= 0 || M <= 0 || N <= 0) return;
  RCS_PROBED_LAUNCH(kKcFactor, k_cgemm_cm, dim3(ceil_div(N, GT_N), ceil_div(M, GT_M), batch), dim3(GT_THREADS), 0, s, A, lda,
                     sa, B, ldb, sb, D, ldd, sd, M, N, K, alpha);
  HIP_LAUNCH_OK();
}

// R^{-1} (upper, ld ldg, lower part zero) from its 64 x 64 diagonal blocks
// (already in Ri) by recursive doubling: for blocks [A | C] of the leading
// diagonal, R^{-1}_{AC} = -R^{-1}_{AA} R_{AC} R^{-1}_{CC}, all pairs of a
// level at once (two GEMM launches per level; T is an ldg x ldg scratch).
static void triangular_inverse(const double2* G, int ldg, double2* Ri, double2* T, hipStream_t s) {
  for (int h = CB; h < ldg; h *= 2) {
    const int full = ldg / (2 * h);              // pairs with |C| = h
    const int tail0 = full * 2 * h;              // a last pair with |C| < h
    const int64_t stride = (int64_t)2 * h * ldg + 2 * h;
    // T_AC = R_AC R^{-1}_CC, then Ri_AC = -R^{-1}_AA T_AC
    cgemm_cm(G + (int64_t)h * ldg, ldg, stride, Ri + (int64_t)h * ldg + h, ldg, stride, T + (int64_t)h * ldg, ldg,
             stride, h, h, h, 1.0, full, s);
    cgemm_cm(Ri, ldg, stride, T + (int64_t)h * ldg, ldg, stride, Ri + (int64_t)h * ldg, ldg, stride, h, h, h, -1.0,
             full, s);
    const int hc = ldg - tail0 - h;
    if (hc > 0) {
      const int64_t a0 = (int64_t)tail0 * ldg + tail0, c0 = (int64_t)(tail0 + h) * ldg + (tail0 + h);
      const int64_t ac = (int64_t)(tail0 + h) * ldg + tail0;
      cgemm_cm(G + ac, ldg, 0, Ri + c0, ldg, 0, T + ac, ldg, 0, h, hc, hc, 1.0, 1, s);
      cgemm_cm(Ri + a0, ldg, 0, T + ac, ldg, 0, Ri + ac, ldg, 0, h, hc, h, -1.0, 1, s);
    }
  }
}

void cholqr(const double2* X, int ldx, int len, int n, double2* G, int ldg, double2* Rd, double2* Ri, double2* T,
            double2* Q, int ldq, int* flag_dev, hipStream_t s) {
  HIP_OK(hipMemsetAsync(Ri, 0, (size_t)ldg * ldg * sizeof(double2), s));
  gram_cholesky(X, ldx, len, n, G, ldg, Rd, Ri, flag_dev, s);
  triangular_inverse(G, ldg, Ri, T, s);
  cgemm_cm(X, ldx, 0, Ri, ldg, 0, Q, ldq, 0, len, n, n, 1.0, 1, s);
}

// *dev = max over entries of |H - I| (H k x k, row-major); *dev must be 0
// beforehand.  Non-negative doubles order like their bit patterns, so the
// workgroups combine with an integer atomic max.
__global__ void k_max_dev_identity(const double2* H, int k, double* dev) {
  __shared__ double red[256];
  double m = 0.0;
  const int64_t tot = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int r = (int)(e / k), c = (int)(e % k);
    const double2 h = H[e];
    const double re = h.x - (r == c ? 1.0 : 0.0);
    m = fmax(m, fmax(fabs(re), fabs(h.y)));
    if (!(h.x == h.x) || !(h.y == h.y)) m = 1e300;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h2 = 128; h2 > 0; h2 >>= 1) {
    if ((int)threadIdx.x < h2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h2]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(dev), (unsigned long long)__double_as_longlong(red[0]));
}

void max_dev_identity(const double2* H, int k, double* dev, hipStream_t s) {
  HIP_OK(hipMemsetAsync(dev, 0, sizeof(double), s));
  const int64_t tot = (int64_t)k * k;
  const int blocks = (int)std::min<int64_t>(1024, (tot + 255) / 256);
  RCS_PROBED_LAUNCH(kKcFactor, k_max_dev_identity, dim3(std::max(blocks, 1)), dim3(256), 0, s, H, k, dev);
  HIP_LAUNCH_OK();
}

// P (k x len, row-major) = scale * (X U)^H with X len x n (ld ldx) and U
// n x k (ld ldu): P[j][r] = scale * sum_i conj(U[i][j]) conj(X[r][i]).
__global__ __launch_bounds__(GT_THREADS) void k_project_rows(const double2* U, int ldu, const double2* X, int ldx,
                                                            int len, int n, int k, double scale, double2* P) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int j, int i) -> double2 {
    const double2 v = U[(int64_t)j * ldu + i];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int i, int r) -> double2 {
    const double2 v = X[(int64_t)i * ldx + r];
    return make_double2(v.x, -v.y);
  };
  LoadA<decltype(fa), true> la{fa, m0, k, n};
  LoadB<decltype(fb), true> lb{fb, n0, n, len};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, n, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int j = m0 + r, col = n0 + c;
    if (j < k && col < len) P[(int64_t)j * len + col] = make_double2(re * scale, im * scale);
  });
}

void project_rows(const double2* U, int ldu, const double2* X, int ldx, int len, int n, int k, double scale,
                  double2* P, hipStream_t s) {
  RCS_PROBED_LAUNCH(kKcFactor, k_project_rows, dim3(ceil_div(len, GT_N), ceil_div(k, GT_M)), dim3(GT_THREADS), 0, s, U, ldu,
                     X, ldx, len, n, k, scale, P);
  HIP_LAUNCH_OK();
}

// out[j*ld + order[i]] = in[j*ld + i] for i < n, j < k: rows back to the
// caller's column order.
__global__ void k_unpermute_rows(const double2* in, int ld, int n, int k, const int* order, double2* out) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[(int64_t)j * ld + order[i]] = in[(int64_t)j * ld + i];
}

void unpermute_rows(const double2* in, int ld, int n, int k, const int* order, double2* out, hipStream_t s) {
  RCS_PROBED_LAUNCH(kKcFactor, k_unpermute_rows, dim3(ceil_div(n, 256), k), dim3(256), 0, s, in, ld, n, k, order, out);
  HIP_LAUNCH_OK();
}

}  // namespace rcs
