// Randomized range finder for the learned-rank truncation.
//
// Halko, Martinsson, Tropp (SIAM Review 2011), randomized range finder with
// power iterations (their Algorithm 4.4): for the two-site matrix M (len x
// cnt) and a sketch width l,
//   Omega (cnt x l), entries {1, i, -1, -i}[x & 3] with x = word 0 of
//     Philox(seed; (row, col, step, 4))   (exact in every precision);
//   Y = M Omega;  Q = orth(Y);
//   q times:  Z = orth(M^H Q);  Q = orth(M Z).
// The products with M are the expensive part and run in fp32 on the matrix
// cores (v_mfma_f32_16x16x4f32); orth() keeps the basis in fp64: block
// classical Gram-Schmidt with two passes (BCGS2) over 64-column panels and
// two Cholesky-QR passes inside each panel (fp64 Gram, 64x64 Cholesky in LDS
// with a pivot guard that zeroes numerically dependent columns); the power
// iteration's intermediate bases take one pass of each.  The caller
// then takes the exact fp64 SVD of the projected matrix B = Q^H M (their
// Algorithm 5.1).
#include "build.h"
#include "gemm_f32.h"
#include "gemm_f64.h"
#include "prof.h"
#include "rsvd.h"

namespace rcs {

__global__ void k_sketch(double2* Z, int ldz, int cnt, int l, uint32_t k0, uint32_t k1, uint32_t step) {
  const int64_t tot = (int64_t)cnt * l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % cnt), c = (int)(e / cnt);
    const U4 x = philox4x32_10(U4{(uint32_t)r, (uint32_t)c, step, kStreamSketch}, k0, k1);
    const int ph = x.x & 3;
    const double2 v = ph == 0 ? make_double2(1.0, 0.0)
                              : ph == 1 ? make_double2(0.0, 1.0)
                                        : ph == 2 ? make_double2(-1.0, 0.0) : make_double2(0.0, -1.0);
    Z[(int64_t)c * ldz + r] = v;
  }
}

// Y (len x l) = M Z, fp32 MFMA.  M col-major (ldx), Z col-major (ldz).
__global__ __launch_bounds__(256) void k_mz32(const double2* M, int ldx, int len, int cnt, const double2* Z, int ldz,
                                             int l, double2* Y, int ldy) {
  __shared__ SmemF32C sm;
  const int m0 = blockIdx.y * FT_M, n0 = blockIdx.x * FT_N;
  auto fa = [&](int m, int k) -> double2 { return M[(int64_t)k * ldx + m]; };
  auto fb = [&](int k, int n) -> double2 { return Z[(int64_t)n * ldz + k]; };
  LoadA32<decltype(fa), false> la{fa, m0, len, cnt};
  LoadB32<decltype(fb), false> lb{fb, n0, cnt, l};
  AccF32C acc;
  acc_zero(acc);
  cgemm32_mainloop(la, lb, cnt, sm, acc);
  acc32_foreach(acc, [&](int r, int c, float re, float im) {
    const int m = m0 + r, n = n0 + c;
    if (m < len && n < l) Y[(int64_t)n * ldy + m] = make_double2(re, im);
  });
}

// Z (cnt x l) = M^H Q, fp32 MFMA.
__global__ __launch_bounds__(256) void k_mhq32(const double2* M, int ldx, int len, int cnt, const double2* Q, int ldq,
                                              int l, double2* Z, int ldz) {
  __shared__ SmemF32C sm;
  const int m0 = blockIdx.y * FT_M, n0 = blockIdx.x * FT_N;
  auto fa = [&](int m, int k) -> double2 {
    const double2 v = M[(int64_t)m * ldx + k];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int k, int n) -> double2 { return Q[(int64_t)n * ldq + k]; };
  LoadA32<decltype(fa), true> la{fa, m0, cnt, len};
  LoadB32<decltype(fb), false> lb{fb, n0, len, l};
  AccF32C acc;
  acc_zero(acc);
  cgemm32_mainloop(la, lb, len, sm, acc);
  acc32_foreach(acc, [&](int r, int c, float re, float im) {
    const int m = m0 + r, n = n0 + c;
    if (m < cnt && n < l) Z[(int64_t)n * ldz + m] = make_double2(re, im);
  });
}

// Partial C (j0 x pw, row-major ld 64) = Q[r0:r0+K, :j0]^H Y[r0:r0+K, j0:j0+pw]
// over the row chunk blockIdx.x (fp64); summed in fixed order by k_csum.
__global__ __launch_bounds__(GT_THREADS) void k_qhy(const double2* Q, int ldq, int len, int j0, int pw,
                                                   int rows_kc, int ldc, double2* Cpart) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, kc = blockIdx.x;
  const int r0 = kc * rows_kc;
  const int K = min(rows_kc, len - r0);
  auto fa = [&](int m, int k) -> double2 {
    const double2 v = Q[(int64_t)m * ldq + r0 + k];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int k, int n) -> double2 { return Q[(int64_t)(j0 + n) * ldq + r0 + k]; };
  LoadA<decltype(fa), true> la{fa, m0, j0, K};
  LoadB<decltype(fb), false> lb{fb, 0, K, pw};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, K, sm, acc);
  double2* C = Cpart + (int64_t)kc * ldc * 64;
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r;
    if (m < j0 && c < pw) C[(int64_t)m * 64 + c] = make_double2(re, im);
  });
}

// C[m][c] = sum over row chunks of the partials, in chunk order.
__global__ void k_csum(const double2* Cpart, int n_kc, int ldc, int j0, double2* C) {
  const int64_t tot = (int64_t)j0 * 64;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int kc = 0; kc < n_kc; ++kc) {
      const double2 v = Cpart[(int64_t)kc * ldc * 64 + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    C[e] = acc;
  }
}

// Partial P_kc (len x pw, col-major ld ldq) = Q[:, K-chunk kc] C[K-chunk kc, :]
// over the column chunk blockIdx.x of Q[:, :j0].
__global__ __launch_bounds__(GT_THREADS) void k_ysub(const double2* Q, int ldq, int len, int j0, int pw,
                                                    const double2* C, int cols_kc, double2* Ppart) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, kc = blockIdx.x;
  const int c0 = kc * cols_kc;
  const int K = min(cols_kc, j0 - c0);
  auto fa = [&](int m, int k) -> double2 { return Q[(int64_t)(c0 + k) * ldq + m]; };
  auto fb = [&](int k, int n) -> double2 { return C[(int64_t)(c0 + k) * 64 + n]; };
  LoadA<decltype(fa), false> la{fa, m0, len, K};
  LoadB<decltype(fb), true> lb{fb, 0, K, pw};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, K, sm, acc);
  double2* P = Ppart + (int64_t)kc * 64 * ldq;
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r;
    if (m < len && c < pw) P[(int64_t)c * ldq + m] = make_double2(re, im);
  });
}

// Y[:, j0:j0+pw] -= sum over column chunks of the partials, in chunk order.
__global__ void k_ysub_apply(double2* Y, int ldq, int len, int j0, int pw, const double2* Ppart, int n_kc) {
  const int64_t tot = (int64_t)pw * len;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / len), m = (int)(e % len);
    double2 acc = make_double2(0.0, 0.0);
    for (int kc = 0; kc < n_kc; ++kc) {
      const double2 v = Ppart[(int64_t)kc * 64 * ldq + (int64_t)c * ldq + m];
      acc.x += v.x;
      acc.y += v.y;
    }
    double2* y = Y + (int64_t)(j0 + c) * ldq + m;
    *y = make_double2(y->x - acc.x, y->y - acc.y);
  }
}

// G (64 x 64) = Yp^H Yp for the panel (partial over row chunks, summed in
// fixed chunk order by k_gsum).
__global__ __launch_bounds__(GT_THREADS) void k_panel_gram(const double2* Q, int ldq, int len, int j0, int pw,
                                                          int rows_per_chunk, double2* part) {
  __shared__ SmemC64 sm;
  const int chunk = blockIdx.x;
  const int r0 = chunk * rows_per_chunk;
  const int K = min(rows_per_chunk, len - r0);
  auto fa = [&](int m, int k) -> double2 {
    const double2 v = Q[(int64_t)(j0 + m) * ldq + r0 + k];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int k, int n) -> double2 { return Q[(int64_t)(j0 + n) * ldq + r0 + k]; };
  LoadA<decltype(fa), true> la{fa, 0, pw, K};
  LoadB<decltype(fb), false> lb{fb, 0, K, pw};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, K, sm, acc);
  double2* g = part + (int64_t)chunk * 64 * 64;
  acc_foreach(acc, [&](int r, int c, double re, double im) { g[r * 64 + c] = make_double2(re, im); });
}

// G = sum of the panel Gram's row-chunk partials (at most 16), one element
// per thread, added in chunk order; all loads of a thread issue together.
__global__ __launch_bounds__(256) void k_gsum(const double2* part, int n_chunks, double2* G) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  double2 t[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) t[u] = u < n_chunks ? part[(int64_t)u * 4096 + e] : make_double2(0.0, 0.0);
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    acc.x += t[u].x;
    acc.y += t[u].y;
  }
  G[e] = acc;
}

// Cholesky G = R^H R (R upper triangular) with pivot guard, then Rinv = R^-1.
// A pivot below guard * max(diag) marks the column dependent: its row of R
// is set to zero and its column of Rinv to zero, so the panel column becomes 0.
// Right-looking, one barrier per step: the trailing update of step k uses
// the unscaled row k and its pivot d (R_ij -= conj(R_ki) R_kj / d), and row k
// is scaled afterwards, while step k+1 touches only rows > k.  The inverse
// solves R Rinv = I bottom-up, one row per step, four lanes per column.
__global__ __launch_bounds__(256) void k_chol_inv(const double2* G, int pw, double guard, double2* Rinv) {
  __shared__ double2 R[64][65];
  __shared__ double2 Ri[64][65];
  __shared__ int dead[64];
  __shared__ double dmax;
  const int tid = threadIdx.x;
  {
    double2 g[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) g[u] = G[tid + 256 * u];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, i = e / 64, j = e % 64;
      R[i][j] = (i < pw && j < pw) ? g[u] : make_double2(i == j ? 1.0 : 0.0, 0.0);
      Ri[i][j] = make_double2(0.0, 0.0);
    }
  }
  if (tid < 64) dead[tid] = tid >= pw;
  __syncthreads();
  if (tid < 64) {   // max of the diagonal over wave 0
    double m = tid < pw ? R[tid][tid].x : 0.0;
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (tid == 0) dmax = m;
  }
  __syncthreads();
  const int ty = tid >> 4, tx = tid & 15;
  for (int k = 0; k < pw; ++k) {
    const double d = R[k][k].x;
    const bool dk = !(d > guard * dmax) || dead[k];
    if (!dk) {
      const double rd = rcp_fast(d);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int i = k + 1 + ty + 16 * ii;
        if (i < pw) {
          const double2 a = R[k][i];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int j = k + 1 + tx + 16 * jj;
            if (j < pw && j >= i) {
              const double2 b = R[k][j];
              const double re = (a.x * b.x + a.y * b.y) * rd, im = (a.x * b.y - a.y * b.x) * rd;
              R[i][j] = make_double2(R[i][j].x - re, R[i][j].y - im);
            }
          }
        }
      }
    }
    __syncthreads();
    const double rp = dk ? 0.0 : rsqrt_fast(d);
    if (tid > k && tid < pw) R[k][tid] = make_double2(R[k][tid].x * rp, R[k][tid].y * rp);
    if (tid == k) {
      R[k][k] = make_double2(dk ? 0.0 : d * rp, 0.0);
      dead[k] = dk ? 1 : 0;
    }
  }
  __syncthreads();
  // Rinv: row i = (e_i - sum_{j>i} R[i][j] Rinv[j][:]) / R[i][i], bottom-up
  const int c = tid >> 2, part4 = tid & 3;
  for (int i = pw - 1; i >= 0; --i) {
    double2 acc = make_double2(0.0, 0.0);
    if (c < pw && c >= i) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int j = i + 1 + part4 + 4 * q;
        if (j <= c) {
          const double2 a = R[i][j], b = Ri[j][c];
          acc.x += a.x * b.x - a.y * b.y;
          acc.y += a.x * b.y + a.y * b.x;
        }
      }
    }
    acc.x += __shfl_xor(acc.x, 1);
    acc.y += __shfl_xor(acc.y, 1);
    acc.x += __shfl_xor(acc.x, 2);
    acc.y += __shfl_xor(acc.y, 2);
    if (part4 == 0 && c < pw && c >= i) {
      if (dead[i] || dead[c]) {
        Ri[i][c] = make_double2(0.0, 0.0);
      } else {
        const double rd = rcp_fast(R[i][i].x);
        Ri[i][c] = make_double2(((i == c ? 1.0 : 0.0) - acc.x) * rd, -acc.y * rd);
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += 256) Rinv[e] = Ri[e / 64][e % 64];
}

// Y[:, j0:j0+pw] <- Y[:, j0:j0+pw] Rinv   (in place by row tiles)
__global__ __launch_bounds__(GT_THREADS) void k_panel_apply(double2* Q, int ldq, int len, int j0, int pw,
                                                           const double2* Rinv) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M;
  auto fa = [&](int m, int k) -> double2 { return Q[(int64_t)(j0 + k) * ldq + m]; };
  auto fb = [&](int k, int n) -> double2 { return Rinv[(int64_t)k * 64 + n]; };
  LoadA<decltype(fa), false> la{fa, m0, len, pw};
  LoadB<decltype(fb), true> lb{fb, 0, pw, pw};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, pw, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r;
    if (m < len && c < pw) Q[(int64_t)(j0 + c) * ldq + m] = make_double2(re, im);
  });
}

// Orthonormalise the l columns of Y (len x l, col-major, ld ldq) in place.
// passes = 2: BCGS2 with CholQR2 panels (orthonormal to fp64 rounding, for
// the final basis); passes = 1: one projection and one CholQR pass (a
// well-conditioned basis of the same span, enough for the power
// iteration's intermediate bases, which only carry the subspace).
static void orth(double2* Y, int ldq, int len, int l, RsvdWork& w, hipStream_t s, int passes) {
  // at most 16 row chunks (k_gsum sums them)
  const int rows_per_chunk = (int)round_up(std::max(64, ceil_div(len, 16)), 64);
  const int n_chunks = ceil_div(len, rows_per_chunk);
  RCS_REQUIRE(n_chunks >= 1 && n_chunks <= 16, "panel Gram split into more than 16 row chunks");
  for (int j0 = 0; j0 < l; j0 += 64) {
    const int pw = std::min(64, l - j0);
    if (j0 > 0) {
      for (int pass = 0; pass < passes; ++pass) {
        // split the length-len reduction over row chunks so ~256 workgroups run
        const int ny = ceil_div(j0, GT_M);
        const int n_kc = std::max(1, std::min({kMaxKChunks, 256 / ny, ceil_div(len, 128)}));
        const int rows_kc = (int)round_up(ceil_div(len, n_kc), 16);
        const int nk = ceil_div(len, rows_kc);
        hipLaunchKernelGGL(k_qhy, dim3(nk, ny), dim3(GT_THREADS), 0, s, Y, ldq, len, j0, pw, rows_kc, w.ldc,
                           w.Cpart);
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_csum, dim3(ceil_div(j0 * 64, 256)), dim3(256), 0, s, w.Cpart, nk, w.ldc, j0, w.C);
        HIP_LAUNCH_OK();
        const int nm = ceil_div(len, GT_M);
        const int n_pc = std::max(1, std::min({kMaxKChunks, 256 / nm, ceil_div(j0, 64)}));
        const int cols_kc = (int)round_up(ceil_div(j0, n_pc), 16);
        const int np = ceil_div(j0, cols_kc);
        hipLaunchKernelGGL(k_ysub, dim3(np, nm), dim3(GT_THREADS), 0, s, Y, ldq, len, j0, pw, w.C, cols_kc,
                           w.Ppart);
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_ysub_apply, dim3(ceil_div(pw * len, 256)), dim3(256), 0, s, Y, ldq, len, j0, pw, w.Ppart,
                           np);
        HIP_LAUNCH_OK();
      }
    }
    for (int pass = 0; pass < passes; ++pass) {
      hipLaunchKernelGGL(k_panel_gram, dim3(n_chunks), dim3(GT_THREADS), 0, s, Y, ldq, len, j0, pw, rows_per_chunk,
                         w.gpart);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_gsum, dim3(16), dim3(256), 0, s, w.gpart, n_chunks, w.gsum);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, s, w.gsum, pw, 1e-26, w.Rinv);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_panel_apply, dim3(1, ceil_div(len, GT_M)), dim3(GT_THREADS), 0, s, Y, ldq, len, j0, pw,
                         w.Rinv);
      HIP_LAUNCH_OK();
    }
  }
}

void rsvd_work_ensure(RsvdWork& w, int len, int cnt, int l) {
  const int ldq = (int)round_up(len, 64), ldz = (int)round_up(cnt, 64);
  w.bufQ.ensure((size_t)ldq * round_up(l, 64) * sizeof(double2));
  w.bufZ.ensure((size_t)ldz * round_up(l, 64) * sizeof(double2));
  w.bufC.ensure((size_t)round_up(l, 64) * 64 * sizeof(double2));
  w.ldc = (int)round_up(l, 64);
  w.bufCp.ensure((size_t)kMaxKChunks * w.ldc * 64 * sizeof(double2));
  w.Cpart = w.bufCp.as<double2>();
  w.bufPp.ensure((size_t)kMaxKChunks * 64 * std::max(ldq, ldz) * sizeof(double2));
  w.Ppart = w.bufPp.as<double2>();
  const int mx = std::max(len, cnt);
  const int n_chunks = ceil_div(mx, (int)round_up(std::max(64, ceil_div(mx, 64)), 64)) + 1;
  w.bufG.ensure((size_t)n_chunks * 4096 * sizeof(double2));
  w.bufR.ensure((size_t)4096 * sizeof(double2));
  w.bufGs.ensure((size_t)4096 * sizeof(double2));
  w.Q = w.bufQ.as<double2>();
  w.Z = w.bufZ.as<double2>();
  w.C = w.bufC.as<double2>();
  w.gpart = w.bufG.as<double2>();
  w.Rinv = w.bufR.as<double2>();
  w.gsum = w.bufGs.as<double2>();
  w.ldq = ldq;
  w.ldz = ldz;
}

void range_finder(const double2* M, int ldx, int len, int cnt, int l, int q, uint64_t seed, uint64_t step,
                  RsvdWork& w, hipStream_t s) {
  rsvd_work_ensure(w, len, cnt, l);
  const int grid_sk = (int)std::min<int64_t>(65535, std::max<int64_t>(1, ((int64_t)cnt * l + 255) / 256));
  hipLaunchKernelGGL(k_sketch, dim3(grid_sk), dim3(256), 0, s, w.Z, w.ldz, cnt, l, (uint32_t)seed,
                     (uint32_t)(seed >> 32), (uint32_t)step);
  HIP_LAUNCH_OK();
  const dim3 gy(ceil_div(l, FT_N), ceil_div(len, FT_M)), gz(ceil_div(l, FT_N), ceil_div(cnt, FT_M));
  {
    // nominal work of the first sketch product M Z (complex fp32 GEMM)
    Probe pr(kKcRange, s, 8.0 * len * (double)cnt * l, 16.0 * len * (double)cnt + 8.0 * (double)(len + cnt) * l);
    hipExtLaunchKernelGGL(k_mz32, gy, dim3(256), 0, s, pr.start(), pr.stop(), 0, M, ldx, len, cnt, w.Z, w.ldz, l,
                          w.Q, w.ldq);
  }
  HIP_LAUNCH_OK();
  orth(w.Q, w.ldq, len, l, w, s, q > 0 ? 1 : 2);
  for (int it = 0; it < q; ++it) {
    hipLaunchKernelGGL(k_mhq32, gz, dim3(256), 0, s, M, ldx, len, cnt, w.Q, w.ldq, l, w.Z, w.ldz);
    HIP_LAUNCH_OK();
    orth(w.Z, w.ldz, cnt, l, w, s, 1);
    hipLaunchKernelGGL(k_mz32, gy, dim3(256), 0, s, M, ldx, len, cnt, w.Z, w.ldz, l, w.Q, w.ldq);
    HIP_LAUNCH_OK();
    orth(w.Q, w.ldq, len, l, w, s, it + 1 == q ? 2 : 1);
  }
}

// X (cnt x l, col-major ld ldxo) = M^H Q in fp64, and a copy in X0.
__global__ __launch_bounds__(GT_THREADS) void k_mhq64(const double2* M, int ldx, int len, int cnt, const double2* Q,
                                                     int ldq, int l, double2* X, double2* X0, int ldxo) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int k) -> double2 {
    const double2 v = M[(int64_t)m * ldx + k];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int k, int n) -> double2 { return Q[(int64_t)n * ldq + k]; };
  LoadA<decltype(fa), true> la{fa, m0, cnt, len};
  LoadB<decltype(fb), false> lb{fb, n0, len, l};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, len, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r, n = n0 + c;
    if (m < cnt && n < l) {
      X[(int64_t)n * ldxo + m] = make_double2(re, im);
      X0[(int64_t)n * ldxo + m] = make_double2(re, im);
    }
  });
}

void project_to_basis(const double2* M, int ldx, int len, int cnt, int l, const RsvdWork& w, double2* X,
                      double2* X0, int ldxo, hipStream_t s) {
  hipLaunchKernelGGL(k_mhq64, dim3(ceil_div(l, GT_N), ceil_div(cnt, GT_M)), dim3(GT_THREADS), 0, s, M, ldx, len, cnt,
                     w.Q, w.ldq, l, X, X0, ldxo);
  HIP_LAUNCH_OK();
}

// A_i[s1][a][j] = sum_t Q[(s1,a)][t] conj(P[j][t])   (rows (s1,a) of M)
__global__ __launch_bounds__(GT_THREADS) void k_basis_times_pc(const double2* Q, int ldq, int len, int l,
                                                              const double2* P, int k, int dl, double2* Ai) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int t) -> double2 { return Q[(int64_t)t * ldq + m]; };
  auto fb = [&](int t, int n) -> double2 {
    const double2 v = P[(int64_t)n * l + t];
    return make_double2(v.x, -v.y);
  };
  LoadA<decltype(fa), false> la{fa, m0, len, l};
  LoadB<decltype(fb), false> lb{fb, n0, l, k};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, l, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    const int m = m0 + r, n = n0 + c;
    if (m < len && n < k) {
      const int s1 = m / dl, a = m % dl;
      Ai[((int64_t)s1 * dl + a) * k + n] = make_double2(re, im);
    }
  });
}

void basis_times_pc(const RsvdWork& w, int len, int l, const double2* P, int k, int dl, double2* Ai, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_times_pc, dim3(ceil_div(k, GT_N), ceil_div(len, GT_M)), dim3(GT_THREADS), 0, s, w.Q,
                     w.ldq, len, l, P, k, dl, Ai);
  HIP_LAUNCH_OK();
}

}  // namespace rcs
