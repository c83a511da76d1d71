// State construction (Section 3.2, stage 1) as a snake-ordered MPS.
//
// Schedule ops run in order on the state's stream:
//   single-qubit layer : A_p^s <- sum_t U[s,t] A_p^t on every site (one launch)
//   two-site update    : centre moves (exact SVD orthogonalisations) until the
//                        centre is in {i, i+1}; T^{s1' s2'} = A_i^{s1'} A_{i+1}^{s2'}
//                        on the matrix cores; theta' = G T mixed with the 4x4
//                        gate (fSim or SWAP of the swap network) while laying out
//                        the Jacobi input; one-sided Jacobi SVD in fp64;
//                        descending sort, rank rule, renormalisation; U_k and
//                        S_k V_k^H written back as the two site tensors.
//   end                : centre moved to position 0, A_0 normalised, so the
//                        state is right-canonical with unit norm.
// The Jacobi SVD orthogonalises whichever side of the two-site matrix has
// fewer columns; for square matrices it picks the side that leaves the
// orthogonality centre where the next update needs it.
#include <algorithm>
#include <array>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>
#include <cstdlib>
#include <chrono>
#include <cmath>

#include "build.h"
#include "chol.h"
#include "circuit.h"
#include "gemm_f64.h"
#include "jacobi.h"
#include "prof.h"
#include "rsvd.h"
#include "state.h"

namespace rcs {

// ------------------------------------------------------------- allocation
size_t site_capacity(const rcs_state_s& st, int) {
  int mx = 1;
  for (int c : st.cap) mx = std::max(mx, c);
  return (size_t)mx * 2 * mx;
}

void state_alloc(rcs_state_s& st, int n, int chi) {
  st.n = n;
  st.chi = chi;
  st.cap.assign(n + 1, 1);
  for (int b = 0; b <= n; ++b) {
    int e = std::min(b, n - b);
    int64_t c = (e >= 30) ? (int64_t)1 << 30 : (int64_t)1 << e;
    st.cap[b] = (int)std::min<int64_t>(c, chi);
  }
  st.dims.assign(n + 1, 1);
  st.pi.resize(n);
  for (int k = 0; k < n; ++k) st.pi[k] = k;
  const size_t per = site_capacity(st, 0);
  st.slab.ensure((size_t)n * per * sizeof(double2));
  st.spare.ensure(per * sizeof(double2));
  st.site.resize(n);
  for (int k = 0; k < n; ++k) st.site[k] = st.slab.as<double2>() + (size_t)k * per;
  st.spare_ptr = st.spare.as<double2>();
  HIP_OK(hipMemsetAsync(st.slab.p, 0, st.slab.bytes, st.stream));
  // |0>: A_k[s=0][0][0] = 1
  const double2 one = make_double2(1.0, 0.0);
  for (int k = 0; k < n; ++k)
    HIP_OK(hipMemcpyAsync(st.site[k], &one, sizeof(double2), hipMemcpyHostToDevice, st.stream));
  HIP_OK(hipStreamSynchronize(st.stream));
  st.center = 0;
  st.canonical = true;
}

// ---------------------------------------------------------------- kernels
struct Layer1q {
  double2* site[64];
  int dl[64], dr[64];
  uint8_t gate[64];
};
__constant__ double2 c_gates1q[3][4];

__global__ void k_apply_1q(Layer1q L) {
  const int k = blockIdx.y;
  const int64_t cnt = (int64_t)L.dl[k] * L.dr[k];
  double2* a = L.site[k];
  const double2* U = c_gates1q[L.gate[k]];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2 x0 = a[e], x1 = a[cnt + e];
    double2 y0 = make_double2(U[0].x * x0.x - U[0].y * x0.y + U[1].x * x1.x - U[1].y * x1.y,
                              U[0].x * x0.y + U[0].y * x0.x + U[1].x * x1.y + U[1].y * x1.x);
    double2 y1 = make_double2(U[2].x * x0.x - U[2].y * x0.y + U[3].x * x1.x - U[3].y * x1.y,
                              U[2].x * x0.y + U[2].y * x0.x + U[3].x * x1.y + U[3].y * x1.x);
    a[e] = y0;
    a[cnt + e] = y1;
  }
}

// T[q][a][c] = A_i^{s1'}[a][:] . A_{i+1}^{s2'}[:][c], q = 2 s1' + s2'
__global__ __launch_bounds__(GT_THREADS) void k_two_site_f64(const double2* A, const double2* B,
                                                            double2* T, int dl, int dm, int dr) {
  __shared__ SmemC64 sm;
  const int q = blockIdx.z, s1 = q >> 1, s2 = q & 1;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  const double2* a = A + (int64_t)s1 * dl * dm;
  const double2* b = B + (int64_t)s2 * dm * dr;
  auto fa = [&](int m, int k) -> double2 { return a[(int64_t)m * dm + k]; };
  auto fb = [&](int k, int n) -> double2 { return b[(int64_t)k * dr + n]; };
  LoadA<decltype(fa), true> la{fa, m0, dl, dm};
  LoadB<decltype(fb), true> lb{fb, n0, dm, dr};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, dm, sm, acc);
  double2* t = T + (int64_t)q * dl * dr;
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    int m = m0 + r, n = n0 + c;
    if (m < dl && n < dr) t[(int64_t)m * dr + n] = make_double2(re, im);
  });
}

// T = the four products A^{s1'} B^{s2'} in the requested contraction precision.
void contract_two_site(const double2* A, const double2* B, double2* T, int dl, int dm, int dr, int precision,
                       hipStream_t s) {
  Probe pr(kKcTwoSite, s, 32.0 * dl * (double)dm * dr, 16.0 * (2.0 * dl * dm + 2.0 * dm * dr + 4.0 * dl * dr));
  if (precision != RCS_PREC_C128) {
    contract_two_site_lowp(A, B, T, dl, dm, dr, precision, s, pr.start(), pr.stop());
    return;
  }
  hipExtLaunchKernelGGL(k_two_site_f64, dim3(ceil_div(dr, GT_N), ceil_div(dl, GT_M), 4), dim3(GT_THREADS), 0, s,
                        pr.start(), pr.stop(), 0, A, B, T, dl, dm, dr);
  HIP_LAUNCH_OK();
}

struct Gate4 {
  double2 g[16];
};

// theta'[s1][s2][a][c] = sum_q G[(s1 s2), q] T[q][a][c] written to X (and X0)
// column-major.  case 1: X = M (rows (s1,a), cols (s2,c)); case 2: X = M^H.
__global__ void k_mix_gate(const double2* T, Gate4 G, int dl, int dr, int orient, double2* X,
                           double2* X0, int ldx) {
  const int64_t tot = (int64_t)dl * dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int a, c;
    if (orient == 1) {  // a fastest: column-major writes along rows (s1, a)
      a = (int)(e % dl);
      c = (int)(e / dl);
    } else {            // c fastest: rows are (s2, c)
      c = (int)(e % dr);
      a = (int)(e / dr);
    }
    double2 t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = T[(int64_t)q * tot + (int64_t)a * dr + c];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double2 g = G.g[o * 4 + q];
        re += g.x * t[q].x - g.y * t[q].y;
        im += g.x * t[q].y + g.y * t[q].x;
      }
      const int s1 = o >> 1, s2 = o & 1;
      int64_t idx;
      double2 v;
      if (orient == 1) {
        idx = (int64_t)(s2 * dr + c) * ldx + (s1 * dl + a);
        v = make_double2(re, im);
      } else {
        idx = (int64_t)(s1 * dl + a) * ldx + (s2 * dr + c);
        v = make_double2(re, -im);
      }
      X[idx] = v;
      X0[idx] = v;
    }
  }
}

// Single-site orthogonalisation input.  right: X[b][(s,a)] = A[s][a][b];
// left: X[a][(s,b)] = conj(A[s][a][b]).
__global__ void k_load_site(const double2* A, int dl, int dr, int right, double2* X, double2* X0,
                            int ldx) {
  const int64_t tot = (int64_t)2 * dl * dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    // e enumerates the device layout [s][a][b]
    const int b = (int)(e % dr);
    const int a = (int)((e / dr) % dl);
    const int s = (int)(e / ((int64_t)dl * dr));
    double2 v = A[e];
    int64_t idx;
    if (right) {
      idx = (int64_t)b * ldx + s * dl + a;
    } else {
      idx = (int64_t)a * ldx + s * dr + b;
      v.y = -v.y;
    }
    X[idx] = v;
    X0[idx] = v;
  }
}

__global__ void k_colnorm(const double2* X, int ldx, int len, double* sigma) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const double2* col = X + (int64_t)j * ldx;
  double s = 0.0;
  for (int r = threadIdx.x; r < len; r += 256) s += col[r].x * col[r].x + col[r].y * col[r].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[j] = sqrt(red[0]);
}

// fp32 copies of fp64 columns, and column norms of fp32 columns (fp64 sums).
__global__ void k_to_c64(const double2* X, float2* Y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    Y[e] = make_float2((float)X[e].x, (float)X[e].y);
}
__global__ void k_scale_c128(double2* x, int64_t n, double a) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = make_double2(x[e].x * a, x[e].y * a);
}
__global__ void k_colnorm_c64(const float2* X, int ldx, int len, double* sigma) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const float2* col = X + (int64_t)j * ldx;
  double s = 0.0;
  for (int r = threadIdx.x; r < len; r += 256) {
    const double x = col[r].x, y = col[r].y;
    s += x * x + y * y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[j] = sqrt(red[0]);
}

// Permute columns of X (len x cnt) into Xs by descending norm (order from
// k_sort_rank); sorted columns converge faster under cyclic Jacobi.
__global__ void k_permute_cols(const double2* X, int ldx, int len, const int* order, double2* Xs) {
  const int j = blockIdx.y;
  const double2* src = X + (int64_t)order[j] * ldx;
  double2* dst = Xs + (int64_t)j * ldx;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < len; r += gridDim.x * blockDim.x) dst[r] = src[r];
}

// *out = sum of squares of v[0..n) (fixed-order tree)
__global__ void k_sum_sq(const double* v, int n, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m += v[i] * v[i];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Sort sigma descending (ties by index), apply the rank rule.
//  w = sum s^2; s^2 <= 1e-24 w counts as zero; tail(k) = sum_{r>=k} s_r^2
//  from the smallest upward; k_eps = min{k>=1 : tail(k) <= eps w};
//  k = min(k_eps, cap); eps_step = tail(k)/w; nrm = sqrt(sum_{r<k} s_r^2).
struct RankOut {
  int k;
  int nnz;
  double eps_step, w, nrm;
  int bad;
};

constexpr int SORT_MAX = 4096;

__global__ __launch_bounds__(1024) void k_sort_rank(const double* sigma, int cnt, int cap,
                                                   double eps, double* sorted, int* order,
                                                   RankOut* out, const double* extra_tail) {
  __shared__ double key[SORT_MAX];
  __shared__ int idx[SORT_MAX];
  int npow = 1;
  while (npow < cnt) npow <<= 1;
  for (int i = threadIdx.x; i < npow; i += blockDim.x) {
    key[i] = i < cnt ? sigma[i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  // bitonic sort: descending by key, ascending by index for equal keys
  for (int size = 2; size <= npow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < npow; i += blockDim.x) {
        int j = i ^ stride;
        if (j > i) {
          bool desc = ((i & size) == 0);
          double ki = key[i], kj = key[j];
          int ii = idx[i], ij = idx[j];
          bool i_first = (ki > kj) || (ki == kj && ii < ij);
          bool swap = desc ? !i_first : i_first;
          if (swap) {
            key[i] = kj;
            key[j] = ki;
            idx[i] = ij;
            idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    sorted[i] = key[i];
    order[i] = idx[i];
  }
  if (threadIdx.x == 0) {
    // extra: discarded weight that lies outside the decomposed subspace
    const double extra = extra_tail ? fmax(*extra_tail, 0.0) : 0.0;
    double w = extra;
    int bad = 0;
    for (int i = cnt - 1; i >= 0; --i) {
      double v = key[i];
      if (!(v == v) || v > 1e300) bad = 1;
      w += v * v;
    }
    const double floor = 1e-24 * w;
    int nnz = 0;
    for (int i = 0; i < cnt; ++i)
      if (key[i] * key[i] > floor) nnz = i + 1;
    // tail sums from the smallest upward; find the smallest k >= 1 with
    // tail(k) <= eps w by scanning k downward while the condition holds.
    double tail = extra;
    int k_eps = cnt;
    double tail_at[1];
    (void)tail_at;
    // walk down accumulating; tail(cnt) is the outside weight, so when even
    // that exceeds eps w the scan stops at once and k_eps = cnt discards it
    double tail_k = extra;
    for (int k = cnt; k >= 1; --k) {
      // tail currently = tail(k)
      if (tail <= eps * w) {
        k_eps = k;
        tail_k = tail;
      } else {
        break;
      }
      double v = key[k - 1];
      double v2 = v * v;
      tail += (v2 <= floor) ? 0.0 : v2;
    }
    int k = min(k_eps, cap);
    double tk = extra;
    if (k == k_eps) {
      tk = tail_k;
    } else {
      for (int i = cnt - 1; i >= k; --i) {
        double v2 = key[i] * key[i];
        tk += (v2 <= floor) ? 0.0 : v2;
      }
    }
    double kept = 0.0;
    for (int i = 0; i < k; ++i) kept += key[i] * key[i];
    out->k = k;
    out->nnz = nnz;
    out->eps_step = (w > 0.0) ? tk / w : 0.0;
    out->w = w;
    out->nrm = sqrt(kept);
    out->bad = bad || !(w > 0.0);
  }
}

// Wn[:, j] = X[:, order[j]] / sorted[j], j < k  (all ldx rows)
__global__ void k_gather_normalize(const double2* X, int ldx, const int* order, const double* sorted,
                                   double2* Wn) {
  const int j = blockIdx.y;
  const double inv = 1.0 / sorted[j];
  const double2* src = X + (int64_t)order[j] * ldx;
  double2* dst = Wn + (int64_t)j * ldx;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ldx; r += gridDim.x * blockDim.x) {
    double2 v = src[r];
    dst[r] = make_double2(v.x * inv, v.y * inv);
  }
}

__global__ void k_gather_normalize_c64(const float2* X, int ldx, const int* order, const double* sorted,
                                       double2* Wn) {
  const int j = blockIdx.y;
  const double inv = 1.0 / sorted[j];
  const float2* src = X + (int64_t)order[j] * ldx;
  double2* dst = Wn + (int64_t)j * ldx;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ldx; r += gridDim.x * blockDim.x) {
    const float2 v = src[r];
    dst[r] = make_double2(v.x * inv, v.y * inv);
  }
}

// Newton-Schulz orthonormalisation of the kept columns (the Jacobi stops at
// an absolute floor, so columns of small singular values are orthonormal
// only to ~floor / (s_i s_j)):  Wn <- Wn (3 I - Wn^H Wn) / 2.
// H (k x k, row-major) = (3 I - Wn^H Wn) / 2
__global__ __launch_bounds__(GT_THREADS) void k_ns_gram(const double2* Wn, int ldx, int len, int k,
                                                       double2* H) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int kk) -> double2 {
    double2 v = Wn[(int64_t)m * ldx + kk];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int kk, int n) -> double2 { return Wn[(int64_t)n * ldx + kk]; };
  LoadA<decltype(fa), true> la{fa, m0, k, len};
  LoadB<decltype(fb), false> lb{fb, n0, len, k};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, len, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    int m = m0 + r, n = n0 + c;
    if (m < k && n < k) H[(int64_t)m * k + n] = make_double2(((m == n) ? 1.5 : 0.0) - 0.5 * re, -0.5 * im);
  });
}

// Out (len x k, column-major, ld ldx) = Wn H
__global__ __launch_bounds__(GT_THREADS) void k_ns_apply(const double2* Wn, int ldx, int len, int k,
                                                        const double2* H, double2* Out) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int kk) -> double2 { return Wn[(int64_t)kk * ldx + m]; };
  auto fb = [&](int kk, int n) -> double2 { return H[(int64_t)kk * k + n]; };
  LoadA<decltype(fa), false> la{fa, m0, len, k};
  LoadB<decltype(fb), true> lb{fb, n0, k, k};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, k, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    int m = m0 + r, n = n0 + c;
    if (m < len && n < k) Out[(int64_t)n * ldx + m] = make_double2(re, im);
  });
}

// P (k x cnt, row-major) = scale * Wn^H X0
__global__ __launch_bounds__(GT_THREADS) void k_project(const double2* Wn, const double2* X0, int ldx,
                                                       int len, int k, int cnt, double scale,
                                                       double2* P) {
  __shared__ SmemC64 sm;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  auto fa = [&](int m, int kk) -> double2 {
    double2 v = Wn[(int64_t)m * ldx + kk];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int kk, int n) -> double2 { return X0[(int64_t)n * ldx + kk]; };
  LoadA<decltype(fa), true> la{fa, m0, k, len};
  LoadB<decltype(fb), false> lb{fb, n0, len, cnt};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, len, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) {
    int m = m0 + r, n = n0 + c;
    if (m < k && n < cnt) P[(int64_t)m * cnt + n] = make_double2(re * scale, im * scale);
  });
}

// Write the two factors of a split back into site layout.
//  case 1 (X = M):   A_i[s1][a][j] = Wn[j][(s1,a)],  A_{i+1}[s2][j][c] = P[j][(s2,c)]
//  case 2 (X = M^H): A_{i+1}[s2][j][c] = conj Wn[j][(s2,c)], A_i[s1][a][j] = conj P[j][(s1,a)]
__global__ void k_write_split(const double2* Wn, int ldx, const double2* P, int cnt, int k, int dl,
                              int dr, int orient, double2* Ai, double2* Aj) {
  const int64_t n1 = (int64_t)2 * dl * k, n2 = (int64_t)2 * k * dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n1 + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n1) {  // A_i element [s1][a][j]
      const int j = (int)(e % k);
      const int a = (int)((e / k) % dl);
      const int s1 = (int)(e / ((int64_t)k * dl));
      double2 v;
      if (orient == 1) {
        v = Wn[(int64_t)j * ldx + s1 * dl + a];
      } else {
        v = P[(int64_t)j * cnt + s1 * dl + a];
        v.y = -v.y;
      }
      Ai[e] = v;
    } else {       // A_{i+1} element [s2][j][c]
      const int64_t f = e - n1;
      const int c = (int)(f % dr);
      const int j = (int)((f / dr) % k);
      const int s2 = (int)(f / ((int64_t)dr * k));
      double2 v;
      if (orient == 1) {
        v = P[(int64_t)j * cnt + s2 * dr + c];
      } else {
        v = Wn[(int64_t)j * ldx + s2 * dr + c];
        v.y = -v.y;
      }
      Aj[f] = v;
    }
  }
}

// Orthonormal factor of a single-site split.  right: A[s][a][j] = Wn[j][(s,a)];
// left: A[s][j][b] = conj Wn[j][(s,b)].
__global__ void k_write_ortho(const double2* Wn, int ldx, int k, int dl, int dr, int right,
                              double2* A) {
  const int64_t tot = right ? (int64_t)2 * dl * k : (int64_t)2 * k * dr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2 v;
    if (right) {
      const int j = (int)(e % k);
      const int a = (int)((e / k) % dl);
      const int s = (int)(e / ((int64_t)k * dl));
      v = Wn[(int64_t)j * ldx + s * dl + a];
    } else {
      const int b = (int)(e % dr);
      const int j = (int)((e / dr) % k);
      const int s = (int)(e / ((int64_t)dr * k));
      v = Wn[(int64_t)j * ldx + s * dr + b];
      v.y = -v.y;
    }
    A[e] = v;
  }
}

// Absorb the non-orthonormal factor into the neighbour, batched over s.
//  right: out[s][j][c] = sum_b P[j][b] A[s][b][c]   (P: k x db)
//  left:  out[s][a][j] = sum_b A[s][a][b] conj P[j][b]
__global__ __launch_bounds__(GT_THREADS) void k_absorb(const double2* P, int pld, const double2* A,
                                                      int da, int db, int k, int right,
                                                      double2* out) {
  __shared__ SmemC64 sm;
  const int s = blockIdx.z;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  AccC64 acc;
  acc_zero(acc);
  if (right) {
    // A here is (db x da) per s: rows b, cols c
    const double2* a = A + (int64_t)s * db * da;
    auto fa = [&](int m, int kk) -> double2 { return P[(int64_t)m * pld + kk]; };
    auto fb = [&](int kk, int n) -> double2 { return a[(int64_t)kk * da + n]; };
    LoadA<decltype(fa), true> la{fa, m0, k, db};
    LoadB<decltype(fb), true> lb{fb, n0, db, da};
    cgemm_mainloop(la, lb, db, sm, acc);
    double2* o = out + (int64_t)s * k * da;
    acc_foreach(acc, [&](int r, int c, double re, double im) {
      int m = m0 + r, n = n0 + c;
      if (m < k && n < da) o[(int64_t)m * da + n] = make_double2(re, im);
    });
  } else {
    // A is (da x db) per s: rows a, cols b
    const double2* a = A + (int64_t)s * da * db;
    auto fa = [&](int m, int kk) -> double2 { return a[(int64_t)m * db + kk]; };
    auto fb = [&](int kk, int n) -> double2 {
      double2 v = P[(int64_t)n * pld + kk];
      return make_double2(v.x, -v.y);
    };
    LoadA<decltype(fa), true> la{fa, m0, da, db};
    LoadB<decltype(fb), false> lb{fb, n0, db, k};
    cgemm_mainloop(la, lb, db, sm, acc);
    double2* o = out + (int64_t)s * da * k;
    acc_foreach(acc, [&](int r, int c, double re, double im) {
      int m = m0 + r, n = n0 + c;
      if (m < da && n < k) o[(int64_t)m * k + n] = make_double2(re, im);
    });
  }
}

__global__ void k_normalize_site(double2* A, int64_t cnt, double* norm_out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += 256) s += A[e].x * A[e].x + A[e].y * A[e].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = 1.0 / nrm;
  for (int64_t e = threadIdx.x; e < cnt; e += 256) A[e] = make_double2(A[e].x * inv, A[e].y * inv);
  if (threadIdx.x == 0) *norm_out = nrm;
}

// Copy a column-major len x cnt matrix into the zero-padded Jacobi buffer.
__global__ void k_copy_in(const double2* x, int len, int cnt, double2* X, int ldx) {
  const int64_t tot = (int64_t)len * cnt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % len), c = (int)(e / len);
    X[(int64_t)c * ldx + r] = x[e];
  }
}

// The same from fp32 columns.
__global__ void k_copy_out_c64(const float2* X, int ldx, int len, int cnt, const int* order, const double* sorted,
                               double* s, double2* u) {
  const int j = blockIdx.y;
  const double sv = sorted[j];
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) s[j] = sv;
  const float2* src = X + (int64_t)order[j] * ldx;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < len; r += gridDim.x * blockDim.x) {
    const float2 v = src[r];
    u[(int64_t)j * len + r] = make_double2(v.x * inv, v.y * inv);
  }
}

// s[j] = sorted[j]; u[:, j] = X[:, order[j]] / sorted[j] (0 when sorted[j] = 0)
__global__ void k_copy_out(const double2* X, int ldx, int len, int cnt, const int* order,
                           const double* sorted, double* s, double2* u) {
  const int j = blockIdx.y;
  const double sv = sorted[j];
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) s[j] = sv;
  const double2* src = X + (int64_t)order[j] * ldx;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < len; r += gridDim.x * blockDim.x) {
    double2 v = src[r];
    u[(int64_t)j * len + r] = make_double2(v.x * inv, v.y * inv);
  }
}

// q[j * len + r] = Q[r][j] (Q: ld ldq) and r[c * cnt + j] = P[j][c] (P row-major
// cnt x cnt): the thin QR factors in column-major layout.
__global__ void k_export_qr(const double2* Q, int ldq, const double2* P, int len, int cnt, double2* q, double2* r) {
  const int64_t tot = (int64_t)len * cnt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % len), j = (int)(e / len);
    q[e] = Q[(int64_t)j * ldq + row];
    if (e < (int64_t)cnt * cnt) {
      const int jj = (int)(e % cnt), c = (int)(e / cnt);
      r[e] = P[(int64_t)jj * cnt + c];
    }
  }
}

// q_dev[j * len + r] = Q[r][j]: the fp64 basis the range finder leaves.
__global__ void k_copy_basis(const double2* Q, int ldq, int len, int l, double2* out) {
  const int64_t tot = (int64_t)len * l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % len), j = (int)(e / len);
    out[e] = Q[(int64_t)j * ldq + r];
  }
}

// Export layout (a, s, b) -> device layout [s][a][b]
__global__ void k_to_device_layout(const double2* in, int da, int db, double2* out) {
  const int64_t tot = (int64_t)2 * da * db;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e % db);
    const int s = (int)((e / db) % 2);
    const int a = (int)(e / (2 * (int64_t)db));
    out[((int64_t)s * da + a) * db + b] = in[e];
  }
}

// ------------------------------------------------------------ workspace
struct BuildWork {
  DevBuf T, X, X0, Wn, P, H, jac, sigma, sorted, order, scal, rot, tmp;
  DevBuf G, Rd, Y, order_x, cflag;   // preconditioned split
  DevBuf Y32;                         // its fp32 copy (RCS_SVD_F32)
  DevBuf Ri, Tq, qdev;                // CholeskyQR centre moves
  std::vector<double> host_sorted;
  double2* wn_final = nullptr;   // orthonormal kept columns after svd_split
  void* host_rank_dev() {
    tmp.ensure(64);
    return tmp.p;
  }
  RankOut* host_rank = nullptr;   // pinned
  int* host_rot = nullptr;        // pinned
  BuildWork() {
    HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&host_rank), sizeof(RankOut)));
    HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&host_rot), 2 * sizeof(int)));
  }
  ~BuildWork() {
    if (host_rank) (void)hipHostFree(host_rank);
    if (host_rot) (void)hipHostFree(host_rot);
  }
};

int grid1d(int64_t n, int per = 256) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65535));
}

static bool sort_columns_first() {
  static const bool v = [] {
    const char* e = std::getenv("RCS_JACOBI_SORT");
    return !(e && e[0] == '0');
  }();
  return v;
}

// Orthogonalise X (len x cnt) and produce Wn (k columns) and P (k x cnt).
struct SplitResult {
  int k, nnz, sweeps;
  double eps_step, w, nrm;
};

// ortho_only: the caller needs an exact factorisation X = Q P with Q
// orthonormal, not singular vectors (centre moves): the Jacobi iteration
// stops at a loose orthogonality (relative 1e-7) and two Newton-Schulz steps
// (error e -> ~3e^2/4 each, from e <= k 1e-7) make the kept columns
// orthonormal to fp64 rounding; P = Q^H X is then exact.
static SplitResult svd_split(rcs_state_s& st, BuildWork& ws, const JacobiPlan& pl, int cap,
                             double eps, bool renorm, std::vector<double>* spectrum_out,
                             const double* extra_dev = nullptr, bool ortho_only = false) {
  hipStream_t s = st.stream;
  // the rank kernel sorts at most SORT_MAX values in LDS
  RCS_REQUIRE(pl.cnt <= SORT_MAX, "matrix too wide for the rank kernel");
  double2* X = ws.X.as<double2>();
  // ||X||_F^2 scales the Jacobi's numerically-zero column threshold
  RCS_PROBED_LAUNCH(kKcFactor, k_colnorm, dim3(pl.cnt), dim3(256), 0, s, X, pl.ldx, pl.len, ws.sigma.as<double>());
  HIP_LAUNCH_OK();
  RCS_PROBED_LAUNCH(kKcFactor, k_sum_sq, dim3(1), dim3(256), 0, s, ws.sigma.as<double>(), pl.cnt,
                     reinterpret_cast<double*>(ws.host_rank_dev()));
  HIP_LAUNCH_OK();
  HIP_OK(hipMemcpyAsync(&ws.host_rank->w, ws.host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double fro2 = ws.host_rank->w;
  if (sort_columns_first()) {
    // order columns by norm (X0 keeps the original order for the projection)
    RCS_PROBED_LAUNCH(kKcFactor, k_sort_rank, dim3(1), dim3(1024), 0, s, ws.sigma.as<double>(), pl.cnt, pl.cnt, 0.0,
                       ws.sorted.as<double>(), ws.order.as<int>(), ws.scal.as<RankOut>(), nullptr);
    HIP_LAUNCH_OK();
    RCS_PROBED_LAUNCH(kKcFactor, k_permute_cols, dim3(ceil_div(pl.len, 256), pl.cnt), dim3(256), 0, s, ws.X0.as<double2>(),
                       pl.ldx, pl.len, ws.order.as<int>(), X);
    HIP_LAUNCH_OK();
  }
  int sweeps = jacobi_run(pl, X, ws.jac.p, ws.rot.as<int>(), ws.host_rot, fro2, s, 60, ortho_only ? 1e-7 : 0.0);
  st.jacobi_sweeps_max = std::max(st.jacobi_sweeps_max, sweeps);
  RCS_PROBED_LAUNCH(kKcFactor, k_colnorm, dim3(pl.cnt), dim3(256), 0, s, X, pl.ldx, pl.len, ws.sigma.as<double>());
  HIP_LAUNCH_OK();
  RCS_PROBED_LAUNCH(kKcFactor, k_sort_rank, dim3(1), dim3(1024), 0, s, ws.sigma.as<double>(), pl.cnt, cap, eps,
                     ws.sorted.as<double>(), ws.order.as<int>(), ws.scal.as<RankOut>(), extra_dev);
  HIP_LAUNCH_OK();
  HIP_OK(hipMemcpyAsync(ws.host_rank, ws.scal.p, sizeof(RankOut), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const RankOut r = *ws.host_rank;
  if (r.bad) fail(RCS_ERR_NUMERIC, "non-finite singular values");
  SplitResult out{r.k, r.nnz, sweeps, r.eps_step, r.w, r.nrm};
  if (spectrum_out) {
    spectrum_out->resize(pl.cnt);
    HIP_OK(hipMemcpyAsync(spectrum_out->data(), ws.sorted.p, pl.cnt * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  RCS_PROBED_LAUNCH(kKcFactor, k_gather_normalize, dim3(ceil_div(pl.ldx, 256), out.k), dim3(256), 0, s, X, pl.ldx,
                     ws.order.as<int>(), ws.sorted.as<double>(), ws.Wn.as<double2>());
  HIP_LAUNCH_OK();
  // orthonormalise: X <- Wn (3I - Wn^H Wn)/2 (X is free after the gather);
  // the Jacobi stops at an absolute floor, so kept columns of small singular
  // values are orthonormal only to ~floor / (s_i s_j); a second step, from X
  // back into Wn, after the loose iteration of a centre move
  double2* src = ws.Wn.as<double2>();
  double2* dst = X;
  for (int it = 0; it < (ortho_only ? 2 : 1); ++it) {
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_gram, dim3(ceil_div(out.k, GT_N), ceil_div(out.k, GT_M)), dim3(GT_THREADS), 0, s, src,
                       pl.ldx, pl.len, out.k, ws.H.as<double2>());
    HIP_LAUNCH_OK();
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_apply, dim3(ceil_div(out.k, GT_N), ceil_div(pl.len, GT_M)), dim3(GT_THREADS), 0, s,
                       src, pl.ldx, pl.len, out.k, ws.H.as<double2>(), dst);
    HIP_LAUNCH_OK();
    std::swap(src, dst);
  }
  ws.wn_final = src;
  const double scale = renorm ? 1.0 / out.nrm : 1.0;
  RCS_PROBED_LAUNCH(kKcFactor, k_project, dim3(ceil_div(pl.cnt, GT_N), ceil_div(out.k, GT_M)), dim3(GT_THREADS), 0, s,
                     ws.wn_final, ws.X0.as<double2>(), pl.ldx, pl.len, out.k, pl.cnt, scale,
                     ws.P.as<double2>());
  HIP_LAUNCH_OK();
  return out;
}

static bool svd_precondition_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("RCS_SVD_PRECOND");
    return !(e && e[0] == '0');
  }();
  return v;
}

// Preconditioned split of X (len x cnt, X0 its copy): the Jacobi runs on
// Y = R^H with R the Cholesky factor of X^H X (chol.hip), so it yields the
// right singular vectors V of X and its singular values.  On success
// ws.wn_final holds V_k (cnt x k, ld *ldw, X's column order) and ws.P the
// k x len factor (X V_k)^H / nrm; the orthonormal factor is on X's column
// side.  Returns false, with the caller free to run the plain split on the
// untouched X0, when the Cholesky breaks down (X numerically rank
// deficient) or when the Gram's rounding (about 1e-13 of ||X||_F^2 in each
// squared singular value) could move the truncation: the last kept squared
// singular value must exceed 1e-10 of the weight, and the discarded weight
// must clear the eps threshold by 1e-9 of the weight on the side the rank
// rule decided.
//
// f32: the Jacobi first runs on an fp32 copy of Y.  Its result is used when
// the bond cap decides the rank by a clear margin (discarded weight above
// the eps threshold by 1e-4 of the weight, or nothing discarded) and the
// last kept squared singular value is at least 1e-7 of the weight: fp32
// singular values carry absolute errors of a few u32 ||Y||, so these
// margins keep the rank and the kept subspace those of the fp64 split up to
// fp32 accuracy.  The kept columns then get two fp64 Newton-Schulz steps
// (orthogonality ~1e-5 -> ~1e-10 -> rounding).  Otherwise the fp64 Jacobi
// runs on Y, which the fp32 attempt left untouched.
static bool svd_split_chol(rcs_state_s& st, BuildWork& ws, const JacobiPlan& pl, int cap, double eps, bool renorm,
                           std::vector<double>* spectrum_out, SplitResult& out, int* ldw, bool f32) {
  hipStream_t s = st.stream;
  const int n = pl.cnt, len = pl.len;
  RCS_REQUIRE(n <= SORT_MAX, "matrix too wide for the rank kernel");
  double2* X = ws.X.as<double2>();
  double2* X0 = ws.X0.as<double2>();
  RCS_PROBED_LAUNCH(kKcFactor, k_colnorm, dim3(n), dim3(256), 0, s, X0, pl.ldx, len, ws.sigma.as<double>());
  HIP_LAUNCH_OK();
  RCS_PROBED_LAUNCH(kKcFactor, k_sum_sq, dim3(1), dim3(256), 0, s, ws.sigma.as<double>(), n,
                     reinterpret_cast<double*>(ws.host_rank_dev()));
  HIP_LAUNCH_OK();
  // columns in descending-norm order (the pivoting of the QR preconditioner)
  ws.order_x.ensure((size_t)n * sizeof(int));
  RCS_PROBED_LAUNCH(kKcFactor, k_sort_rank, dim3(1), dim3(1024), 0, s, ws.sigma.as<double>(), n, n, 0.0,
                     ws.sorted.as<double>(), ws.order_x.as<int>(), ws.scal.as<RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  RCS_PROBED_LAUNCH(kKcFactor, k_permute_cols, dim3(ceil_div(len, 256), n), dim3(256), 0, s, X0, pl.ldx, len,
                     ws.order_x.as<int>(), X);
  HIP_LAUNCH_OK();
  const int ldg = (int)round_up(n, 64);
  JacobiPlan py = jacobi_plan(n, n);
  ws.G.ensure((size_t)ldg * ldg * sizeof(double2));
  ws.Rd.ensure((size_t)ldg * 64 * sizeof(double2));
  ws.Y.ensure((size_t)py.ldx * py.cnt_pad * sizeof(double2));
  ws.jac.ensure(jacobi_work_bytes(py));
  ws.cflag.ensure(sizeof(int));
  HIP_OK(hipMemsetAsync(ws.cflag.p, 0, sizeof(int), s));
  chol_precondition(X, pl.ldx, len, n, ws.G.as<double2>(), ldg, ws.Rd.as<double2>(), ws.Y.as<double2>(), py.ldx,
                    py.cnt_pad, ws.cflag.as<int>(), s);
  HIP_OK(hipMemcpyAsync(&ws.host_rank->w, ws.host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(ws.host_rot, ws.cflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double fro2 = ws.host_rank->w;
  if (*ws.host_rot != 0) return false;
  double2* Y = ws.Y.as<double2>();
  ws.host_sorted.resize(n);
  // rank rule on the Jacobi's columns; fills host_rank and host_sorted
  auto rank = [&](const void* cols, bool c64) {
    if (c64)
      RCS_PROBED_LAUNCH(kKcFactor, k_colnorm_c64, dim3(n), dim3(256), 0, s, static_cast<const float2*>(cols), py.ldx, n,
                        ws.sigma.as<double>());
    else
      RCS_PROBED_LAUNCH(kKcFactor, k_colnorm, dim3(n), dim3(256), 0, s, static_cast<const double2*>(cols), py.ldx, n,
                        ws.sigma.as<double>());
    HIP_LAUNCH_OK();
    RCS_PROBED_LAUNCH(kKcFactor, k_sort_rank, dim3(1), dim3(1024), 0, s, ws.sigma.as<double>(), n, cap, eps,
                       ws.sorted.as<double>(), ws.order.as<int>(), ws.scal.as<RankOut>(), nullptr);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(ws.host_rank, ws.scal.p, sizeof(RankOut), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ws.host_sorted.data(), ws.sorted.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return *ws.host_rank;
  };
  // discarded weight beyond the rank rule's k and the last kept squared value
  auto tail = [&](const RankOut& r, double* sk2) {
    double tk = 0.0;
    for (int i = n - 1; i >= r.k; --i) tk += ws.host_sorted[i] * ws.host_sorted[i];
    *sk2 = ws.host_sorted[r.k - 1] * ws.host_sorted[r.k - 1];
    return tk;
  };
  float2* Y32 = nullptr;
  RankOut r{};
  int sweeps = 0;
  bool use32 = false;
  if (f32) {
    ws.Y32.ensure((size_t)py.ldx * py.cnt_pad * sizeof(float2));
    Y32 = ws.Y32.as<float2>();
    const int64_t ne = (int64_t)py.ldx * py.cnt_pad;
    RCS_PROBED_LAUNCH(kKcFactor, k_to_c64, dim3(grid1d(ne)), dim3(256), 0, s, Y, Y32, ne);
    HIP_LAUNCH_OK();
    sweeps = jacobi_run_f32(py, Y32, ws.jac.p, ws.rot.as<int>(), ws.host_rot, fro2, s, 60);
    r = rank(Y32, true);
    if (!r.bad && r.k >= 1) {
      double sk2;
      const double tk = tail(r, &sk2), W = r.w;
      use32 = (r.k == n || tk > eps * W + 1e-4 * W) && sk2 >= 1e-7 * W;
    }
    if (use32)
      st.n_svd_f32 += 1;
    else
      st.n_svd_f32_redone += 1;
  }
  if (!use32) {
    sweeps = jacobi_run(py, Y, ws.jac.p, ws.rot.as<int>(), ws.host_rot, fro2, s, 60);
    r = rank(Y, false);
    if (r.bad || r.k < 1) return false;
    double sk2;
    const double tk = tail(r, &sk2), W = r.w;
    const double thr = eps * W, delta = 1e-9 * W;
    const bool decided = r.k == n || tk > thr + delta || (tk <= thr - delta && tk + sk2 > thr + delta);
    if (!(sk2 >= 1e-10 * W) || !decided) return false;
  }
  st.jacobi_sweeps_max = std::max(st.jacobi_sweeps_max, sweeps);
  out = SplitResult{r.k, r.nnz, sweeps, r.eps_step, r.w, r.nrm};
  if (spectrum_out) spectrum_out->assign(ws.host_sorted.begin(), ws.host_sorted.end());
  const int k = r.k;
  // kept columns of Y J, normalised: V_k in the sorted basis.  The accepted
  // fp64 split keeps only squared values >= 1e-10 of the weight, far above
  // the Jacobi's noise floor, so every kept pair is orthogonal to the
  // relative tolerance and the columns are orthonormal to fp64 accuracy as
  // they are; after the fp32 Jacobi two Newton-Schulz steps (Wn -> Y -> Wn,
  // Y is free after the gather) make them orthonormal to fp64 rounding.
  double2* Wn = ws.Wn.as<double2>();
  if (use32)
    RCS_PROBED_LAUNCH(kKcFactor, k_gather_normalize_c64, dim3(ceil_div(py.ldx, 256), k), dim3(256), 0, s, Y32,
                       py.ldx, ws.order.as<int>(), ws.sorted.as<double>(), Wn);
  else
    RCS_PROBED_LAUNCH(kKcFactor, k_gather_normalize, dim3(ceil_div(py.ldx, 256), k), dim3(256), 0, s, Y, py.ldx,
                       ws.order.as<int>(), ws.sorted.as<double>(), Wn);
  HIP_LAUNCH_OK();
  double2* src = Wn;
  double2* dst = Y;
  for (int it = 0; it < (use32 ? 2 : 0); ++it) {
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_gram, dim3(ceil_div(k, GT_N), ceil_div(k, GT_M)), dim3(GT_THREADS), 0, s, src,
                       py.ldx, n, k, ws.H.as<double2>());
    HIP_LAUNCH_OK();
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_apply, dim3(ceil_div(k, GT_N), ceil_div(n, GT_M)), dim3(GT_THREADS), 0, s, src,
                       py.ldx, n, k, ws.H.as<double2>(), dst);
    HIP_LAUNCH_OK();
    std::swap(src, dst);
  }
  // P = (X_sorted V_k)^H / nrm, and V_k back in X's column order (into the
  // other buffer)
  if (!use32) {
    project_rows(src, py.ldx, X, pl.ldx, len, n, k, renorm ? 1.0 / r.nrm : 1.0, ws.P.as<double2>(), s);
  } else {
    // the kept weight ||X V_k||_F^2 of the fp64 projection gives nrm and the
    // discarded fraction (fp32 singular values drift by ~1e-4 of the largest)
    double2* P = ws.P.as<double2>();
    project_rows(src, py.ldx, X, pl.ldx, len, n, k, 1.0, P, s);
    RCS_PROBED_LAUNCH(kKcFactor, k_colnorm, dim3(k), dim3(256), 0, s, P, len, len, ws.sigma.as<double>());
    HIP_LAUNCH_OK();
    RCS_PROBED_LAUNCH(kKcFactor, k_sum_sq, dim3(1), dim3(256), 0, s, ws.sigma.as<double>(), k,
                       reinterpret_cast<double*>(ws.host_rank_dev()));
    HIP_LAUNCH_OK();
    double kept = 0.0;
    HIP_OK(hipMemcpyAsync(&kept, ws.host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (!(kept > 0.0)) fail(RCS_ERR_NUMERIC, "non-finite or zero kept weight");
    out.nrm = std::sqrt(kept);
    out.w = fro2;
    out.eps_step = std::max(0.0, 1.0 - kept / fro2);
    if (renorm) {
      const int64_t ne = (int64_t)k * len;
      RCS_PROBED_LAUNCH(kKcFactor, k_scale_c128, dim3(grid1d(ne)), dim3(256), 0, s, P, ne, 1.0 / out.nrm);
      HIP_LAUNCH_OK();
    }
  }
  unpermute_rows(src, py.ldx, n, k, ws.order_x.as<int>(), dst, s);
  ws.wn_final = dst;
  *ldw = py.ldx;
  return true;
}

void ensure_work(BuildWork& ws, const JacobiPlan& pl, int64_t t_elems) {
  const size_t xbytes = (size_t)pl.ldx * pl.cnt_pad * sizeof(double2);
  ws.X.ensure(xbytes);
  ws.X0.ensure(xbytes);
  ws.Wn.ensure(xbytes);
  ws.P.ensure((size_t)pl.cnt_pad * pl.cnt_pad * sizeof(double2) + (size_t)pl.ldx * pl.cnt * sizeof(double2));
  ws.H.ensure((size_t)pl.cnt_pad * pl.cnt_pad * sizeof(double2));
  ws.jac.ensure(jacobi_work_bytes(pl));
  ws.sigma.ensure((size_t)pl.cnt_pad * sizeof(double));
  ws.sorted.ensure((size_t)pl.cnt_pad * sizeof(double));
  ws.order.ensure((size_t)pl.cnt_pad * sizeof(int));
  ws.scal.ensure(sizeof(RankOut));
  ws.rot.ensure(2 * sizeof(int));
  if (t_elems > 0) ws.T.ensure((size_t)t_elems * sizeof(double2));
}

// Nominal work of the factorisations (real flops, complex counted as 4x
// real): thin SVD with U, Golub & Van Loan's count 14 m n^2 + 8 n^3, and
// Householder QR 2 m n^2 - 2 n^3 / 3, m >= n.
static double nominal_svd_flops(int a, int b) {
  const double m = std::max(a, b), n = std::min(a, b);
  return 4.0 * (14.0 * m * n * n + 8.0 * n * n * n);
}
static double nominal_qr_flops(int a, int b) {
  const double m = std::max(a, b), n = std::min(a, b);
  return 4.0 * (2.0 * m * n * n - 2.0 * n * n * n / 3.0);
}

static bool cholqr_moves_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("RCS_CHOLQR_MOVES");
    return !(e && e[0] == '0');
  }();
  return v;
}

// CholeskyQR of the loaded site matrix X (len x cnt): Q1 = X R^{-1} with R
// the Cholesky factor of X^H X, then Newton-Schulz steps Q <- Q (3I -
// Q^H Q) / 2.  Q1's orthogonality defect is about u cond(X)^2; the first
// step measures it and the move is left to the Jacobi path (false) when it
// exceeds 1e-4 (cond(X) above about 1e6) or the Cholesky breaks down
// (X rank deficient).  From 1e-4 two more steps reach rounding level
// (e -> 3e^2/4 each).  On success ws.wn_final holds Q (ld pl.ldx).
static bool move_cholqr(rcs_state_s& st, BuildWork& ws, const JacobiPlan& pl) {
  hipStream_t s = st.stream;
  const int len = pl.len, n = pl.cnt;
  const int ldg = (int)round_up(n, 64);
  ws.G.ensure((size_t)ldg * ldg * sizeof(double2));
  ws.Rd.ensure((size_t)ldg * 64 * sizeof(double2));
  ws.Ri.ensure((size_t)ldg * ldg * sizeof(double2));
  ws.Tq.ensure((size_t)ldg * ldg * sizeof(double2));
  ws.cflag.ensure(sizeof(int));
  ws.qdev.ensure(sizeof(double));
  HIP_OK(hipMemsetAsync(ws.cflag.p, 0, sizeof(int), s));
  double2* Wn = ws.Wn.as<double2>();
  double2* X = ws.X.as<double2>();
  cholqr(ws.X0.as<double2>(), pl.ldx, len, n, ws.G.as<double2>(), ldg, ws.Rd.as<double2>(), ws.Ri.as<double2>(),
         ws.Tq.as<double2>(), Wn, pl.ldx, ws.cflag.as<int>(), s);
  double2* src = Wn;
  double2* dst = X;
  for (int it = 0; it < 3; ++it) {
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_gram, dim3(ceil_div(n, GT_N), ceil_div(n, GT_M)), dim3(GT_THREADS), 0, s, src, pl.ldx,
                       len, n, ws.H.as<double2>());
    HIP_LAUNCH_OK();
    if (it == 0) {
      max_dev_identity(ws.H.as<double2>(), n, ws.qdev.as<double>(), s);
      double dev = 0.0;
      HIP_OK(hipMemcpyAsync(ws.host_rot, ws.cflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_OK(hipMemcpyAsync(&ws.host_rank->w, ws.qdev.p, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      dev = ws.host_rank->w;      // max |H - I| = max |I - Q^H Q| / 2
      if (*ws.host_rot != 0 || !(dev <= 0.5e-4)) return false;
    }
    RCS_PROBED_LAUNCH(kKcFactor, k_ns_apply, dim3(ceil_div(n, GT_N), ceil_div(len, GT_M)), dim3(GT_THREADS), 0, s, src,
                       pl.ldx, len, n, ws.H.as<double2>(), dst);
    HIP_LAUNCH_OK();
    std::swap(src, dst);
  }
  ws.wn_final = src;
  return true;
}

// Move the orthogonality centre one step: X = Q P with Q orthonormal
// (CholeskyQR, or, when X is rank deficient or too ill-conditioned for it,
// the Jacobi orthogonalisation that drops exact zeros); Q stays, P is
// absorbed into the neighbour.
static void move_center(rcs_state_s& st, BuildWork& ws, bool right) {
  hipStream_t s = st.stream;
  const int c = st.center;
  const int dl = st.dims[c], dr = st.dims[c + 1];
  const int len = right ? 2 * dl : 2 * dr;
  const int cnt = right ? dr : dl;
  JacobiPlan pl = jacobi_plan(len, cnt);
  ensure_work(ws, pl, 0);
  HIP_OK(hipMemsetAsync(ws.X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws.X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  hipLaunchKernelGGL(k_load_site, dim3(grid1d((int64_t)2 * dl * dr)), dim3(256), 0, s, st.site[c], dl, dr,
                     right ? 1 : 0, ws.X.as<double2>(), ws.X0.as<double2>(), pl.ldx);
  HIP_LAUNCH_OK();
  int k;
  if (cholqr_moves_enabled() && cnt >= 64 && cnt <= len && move_cholqr(st, ws, pl)) {
    k = cnt;
    st.n_moves_cholqr += 1;
    RCS_PROBED_LAUNCH(kKcFactor, k_project, dim3(ceil_div(cnt, GT_N), ceil_div(k, GT_M)), dim3(GT_THREADS), 0, s,
                       ws.wn_final, ws.X0.as<double2>(), pl.ldx, len, k, cnt, 1.0, ws.P.as<double2>());
    HIP_LAUNCH_OK();
  } else {
    // the CholeskyQR attempt (if any) left X untouched only where it ran
    // out of steps: reload it
    HIP_OK(hipMemcpyAsync(ws.X.p, ws.X0.p, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), hipMemcpyDeviceToDevice, s));
    SplitResult r = svd_split(st, ws, pl, right ? st.cap[c + 1] : st.cap[c], 0.0, false, nullptr, nullptr, true);
    k = r.k;
  }
  st.n_moves += 1;
  st.nominal_qr_flops += nominal_qr_flops(len, cnt);
  hipLaunchKernelGGL(k_write_ortho, dim3(grid1d((int64_t)2 * k * std::max(dl, dr))), dim3(256), 0, s,
                     ws.wn_final, pl.ldx, k, dl, dr, right ? 1 : 0, st.site[c]);
  HIP_LAUNCH_OK();
  if (right) {
    const int d2 = st.dims[c + 2];
    hipLaunchKernelGGL(k_absorb, dim3(ceil_div(d2, GT_N), ceil_div(k, GT_M), 2), dim3(GT_THREADS), 0, s,
                       ws.P.as<double2>(), pl.cnt, st.site[c + 1], d2, dr, k, 1, st.spare_ptr);
    HIP_LAUNCH_OK();
    std::swap(st.site[c + 1], st.spare_ptr);
    st.dims[c + 1] = k;
    st.center = c + 1;
  } else {
    const int d0 = st.dims[c - 1];
    hipLaunchKernelGGL(k_absorb, dim3(ceil_div(k, GT_N), ceil_div(d0, GT_M), 2), dim3(GT_THREADS), 0, s,
                       ws.P.as<double2>(), pl.cnt, st.site[c - 1], d0, dl, k, 0, st.spare_ptr);
    HIP_LAUNCH_OK();
    std::swap(st.site[c - 1], st.spare_ptr);
    st.dims[c] = k;
    st.center = c - 1;
  }
}

// Per-build state of the learned / randomized rank modes.
struct UpdateCtx {
  const BuildOptions* o = nullptr;
  int n_cycles = 0;
  int update_index = 0;
  DevBuf w_mlp, feat, yhat, bond_spec, scal2;
  std::vector<int> bond_k;          // kept count of each bond's last truncation
  std::vector<double> prev_eps;     // discarded fraction of each bond's last truncation
  RsvdWork rw;
  DevBuf M;
  int chi_cap = 0;
  bool pred_capped = true;          // learned mode: the network predicted k_hat >= cap for this update
  double* dev_scalars() { return scal2.as<double>(); }
};

__global__ void k_sub_scalar(const double* a, const double* b, double* out) { *out = *a - *b; }

// k_hat = ceil(m f*), f* the first f where the interpolated prediction y(f)
// drops to log10(eps) (y(0) = 0, knots at j/32); clamped to [1, min(cap, m)].
static int predict_rank(const float* y, int m, int cap, double eps) {
  const double target = eps > 0.0 ? std::log10(eps) : -20.0;
  double fstar = 1.0, yprev = 0.0;
  for (int j = 1; j <= 32; ++j) {
    const double yj = y[j - 1];
    if (yj <= target) {
      const double f0 = (j - 1) / 32.0, f1 = j / 32.0;
      fstar = (yj == yprev) ? f1 : f0 + (target - yprev) / (yj - yprev) * (f1 - f0);
      break;
    }
    yprev = yj;
  }
  int k = (int)std::ceil(m * fstar - 1e-12);
  return std::max(1, std::min({cap, k, m}));
}

static double predicted_eps(const float* y, int k, int m) {
  const double f = (double)k / m;
  const int j = std::min(31, (int)std::floor(f * 32.0));
  const double f0 = j / 32.0, f1 = (j + 1) / 32.0;
  const double y0 = j == 0 ? 0.0 : y[j - 1], y1 = y[j];
  return std::pow(10.0, y0 + (f - f0) / (f1 - f0) * (y1 - y0));
}

static void record_bond_spectrum(rcs_state_s& st, BuildWork& ws, UpdateCtx& ctx, int i, int k) {
  if (!ctx.o || ctx.o->rank_mode == RCS_RANK_FULL_SVD) return;
  const int kk = std::min(k, ctx.chi_cap);
  HIP_OK(hipMemcpyAsync(ctx.bond_spec.as<double>() + (size_t)i * ctx.chi_cap, ws.sorted.p, kk * sizeof(double),
                        hipMemcpyDeviceToDevice, st.stream));
  ctx.bond_k[i] = kk;
}

// Randomized split of the two-site matrix (T already holds the products).
// Returns false when the randomized path does not apply or the judge rejects.
static bool randomized_split(rcs_state_s& st, BuildWork& ws, UpdateCtx& ctx, int i, const double2* gate16,
                             int cap, double eps, int cycle, bool log_spectra) {
  hipStream_t s = st.stream;
  const BuildOptions& o = *ctx.o;
  const int dl = st.dims[i], dm = st.dims[i + 1], dr = st.dims[i + 2];
  const int len = 2 * dl, cnt = 2 * dr, m = std::min(len, cnt);
  RsvdRecord rec{};
  rec.update = ctx.update_index - 1;
  rec.pos = i;
  rec.cycle = cycle;
  rec.m = m;
  rec.k = -1;
  float* y = rec.y;
  int k_hat;
  if (o.rank_mode == RCS_RANK_LEARNED) {
    spectrum_features(ctx.bond_spec.as<double>() + (size_t)i * ctx.chi_cap, ctx.bond_k[i], i, st.n, cycle,
                      ctx.n_cycles, ctx.feat.as<float>(), s);
    mlp_forward(ctx.w_mlp.as<float>(), ctx.feat.as<float>(), 1, ctx.yhat.as<float>(), nullptr, s);
    HIP_OK(hipMemcpyAsync(rec.y, ctx.yhat.p, sizeof(rec.y), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(rec.feat, ctx.feat.p, sizeof(rec.feat), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    k_hat = predict_rank(y, m, cap, eps);
  } else {
    k_hat = std::min(cap, m);
  }
  const int l = std::min(k_hat + std::max(0, o.rsvd_p), m);
  rec.k_hat = k_hat;
  rec.l = l;
  ctx.pred_capped = k_hat >= cap;
  if (l >= m) return false;   // the sketch would cover the whole space: plain split
  // predicted cap-limited cut with the fp32 full SVD available: no sketch
  if (o.svd_f32 && o.rank_mode == RCS_RANK_LEARNED && k_hat >= cap) return false;
  // M (len x cnt, column-major) from the products
  const int ldm = (int)round_up(len, 64);
  ctx.M.ensure((size_t)ldm * round_up(cnt, 64) * sizeof(double2));
  double2* M = ctx.M.as<double2>();
  Gate4 G;
  for (int e = 0; e < 16; ++e) G.g[e] = gate16[e];
  hipLaunchKernelGGL(k_mix_gate, dim3(grid1d((int64_t)dl * dr)), dim3(256), 0, s, ws.T.as<double2>(), G, dl, dr, 1,
                     M, M, ldm);
  HIP_LAUNCH_OK();
  range_finder(M, ldm, len, cnt, l, std::max(0, o.rsvd_q), o.rsvd_seed, (uint64_t)ctx.update_index, ctx.rw, s);
  JacobiPlan pl = jacobi_plan(cnt, l);
  ensure_work(ws, pl, 0);
  ws.sigma.ensure((size_t)std::max(cnt, pl.cnt_pad) * sizeof(double));
  HIP_OK(hipMemsetAsync(ws.X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws.X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  project_to_basis(M, ldm, len, cnt, l, ctx.rw, ws.X.as<double2>(), ws.X0.as<double2>(), pl.ldx, s);
  // weight outside span(Q): ||M||_F^2 - ||B||_F^2 (fp64)
  double* sc = ctx.dev_scalars();
  hipLaunchKernelGGL(k_colnorm, dim3(cnt), dim3(256), 0, s, M, ldm, len, ws.sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sum_sq, dim3(1), dim3(256), 0, s, ws.sigma.as<double>(), cnt, sc + 0);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_colnorm, dim3(l), dim3(256), 0, s, ws.X.as<double2>(), pl.ldx, cnt, ws.sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sum_sq, dim3(1), dim3(256), 0, s, ws.sigma.as<double>(), l, sc + 1);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sub_scalar, dim3(1), dim3(1), 0, s, sc + 0, sc + 1, sc + 2);
  HIP_LAUNCH_OK();
  // Early rejection, the same decision as the judge below.  When the weight
  // outside span(Q) exceeds eps times the total, no rank meets eps, so the
  // rank rule keeps k = min(l, cap).  The discarded fraction is then at
  // least (outside weight) / (total), and if that alone exceeds the judge's
  // threshold the split would be rejected after its projected SVD anyway.
  // The 1e-9 relative margins cover the rounding between ||B||_F^2 and the
  // sum of B's squared singular values.
  {
    double h[3];
    HIP_OK(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double outside = std::max(h[2], 0.0), wb = outside + h[1];
    rec.outside = outside;
    rec.total = wb;
    if (o.fallback_tau >= 0.0 && wb > 0.0 && outside > eps * wb * (1.0 + 1e-9)) {
      const int k_forced = std::min(l, cap);
      const double ep = (o.rank_mode == RCS_RANK_LEARNED) ? predicted_eps(y, k_forced, m) : ctx.prev_eps[i];
      if (outside / wb > (std::max(eps, ep) + o.fallback_tau) * (1.0 + 1e-9)) {
        st.n_fallback += 1;
        st.n_rsvd_early += 1;
        rec.early = 1;
        rec.k = k_forced;
        rec.eps_pred = ep;
        rec.eps_rand = outside / wb;
        st.rsvd_log.push_back(rec);
        return false;
      }
    }
  }
  std::vector<double> spec;
  SplitResult r = svd_split(st, ws, pl, cap, eps, true, log_spectra ? &spec : nullptr, sc + 2);
  const double eps_pred = (o.rank_mode == RCS_RANK_LEARNED) ? predicted_eps(y, r.k, m) : ctx.prev_eps[i];
  const bool accept = o.fallback_tau >= 0.0 && r.eps_step <= std::max(eps, eps_pred) + o.fallback_tau;
  rec.k = r.k;
  rec.eps_pred = eps_pred;
  rec.eps_rand = r.eps_step;
  rec.accepted = accept ? 1 : 0;
  st.rsvd_log.push_back(rec);
  if (!accept) {
    st.n_fallback += 1;
    if (log_spectra) st.rsvd_log.back().values = std::move(spec);
    return false;
  }
  const int k = r.k;
  // A_{i+1} = V_k^H (conjugated kept columns), A_i = Q (B V_k) / nrm
  hipLaunchKernelGGL(k_write_ortho, dim3(grid1d((int64_t)2 * k * dr)), dim3(256), 0, s, ws.wn_final, pl.ldx, k, dl,
                     dr, 0, st.site[i + 1]);
  HIP_LAUNCH_OK();
  basis_times_pc(ctx.rw, len, l, ws.P.as<double2>(), k, dl, st.site[i], s);
  st.dims[i + 1] = k;
  st.center = i;
  st.log_fest += std::log1p(-r.eps_step);
  st.sum_eps += r.eps_step;
  st.n_trunc += 1;
  st.n_rsvd_ok += 1;
  ctx.prev_eps[i] = r.eps_step;
  record_bond_spectrum(st, ws, ctx, i, k);
  st.updates.push_back(UpdateRecord{i, cycle, dl, dm, dr, k, 1});
  if (log_spectra) {
    st.rsvd_log.back().values = spec;
    SpectrumRecord srec{i, cycle, l, k, dl, dr, std::move(spec)};
    st.spectra.push_back(std::move(srec));
  }
  return true;
}

static void two_site_update(rcs_state_s& st, BuildWork& ws, UpdateCtx& ctx, int i, const double2* gate16, int cap,
                            double eps, int prefer_left, int cycle, bool log_spectra, int precision) {
  hipStream_t s = st.stream;
  while (st.center < i) move_center(st, ws, true);
  while (st.center > i + 1) move_center(st, ws, false);
  const int dl = st.dims[i], dm = st.dims[i + 1], dr = st.dims[i + 2];
  const int cap_eff = std::min(cap, st.cap[i + 1]);
  ctx.update_index += 1;
  ws.T.ensure((size_t)4 * dl * dr * sizeof(double2));
  contract_two_site(st.site[i], st.site[i + 1], ws.T.as<double2>(), dl, dm, dr, precision, s);
  const size_t n_log = st.rsvd_log.size();
  ctx.pred_capped = true;
  if (ctx.o && ctx.o->rank_mode != RCS_RANK_FULL_SVD &&
      randomized_split(st, ws, ctx, i, gate16, cap_eff, eps, cycle, log_spectra))
    return;
  const bool randomized_tried = st.rsvd_log.size() > n_log;
  // X = M (orient 1, rows (s1, a)) or M^H (orient 2, rows (s2, c)), with
  // no more columns than rows.  The plain split puts the orthonormal factor
  // on X's row side, the preconditioned one on its column side; a square M
  // is oriented so that the preferred one leaves the centre where the next
  // update needs it.
  const bool precond = svd_precondition_enabled() && std::min(dl, dr) >= 64;
  int orient;
  if (dr < dl)
    orient = 1;
  else if (dl < dr)
    orient = 2;
  else
    orient = (prefer_left != 0) == precond ? 1 : 2;
  const int len = orient == 1 ? 2 * dl : 2 * dr;
  const int cnt = orient == 1 ? 2 * dr : 2 * dl;
  JacobiPlan pl = jacobi_plan(len, cnt);
  ensure_work(ws, pl, 0);
  HIP_OK(hipMemsetAsync(ws.X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws.X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  Gate4 G;
  for (int e = 0; e < 16; ++e) G.g[e] = gate16[e];
  hipLaunchKernelGGL(k_mix_gate, dim3(grid1d((int64_t)dl * dr)), dim3(256), 0, s, ws.T.as<double2>(), G, dl,
                     dr, orient, ws.X.as<double2>(), ws.X0.as<double2>(), pl.ldx);
  HIP_LAUNCH_OK();
  std::vector<double> spec;
  SplitResult r{};
  int ldw = pl.ldx, p_row = pl.cnt, side = orient;
  // fp32 first, unless the network predicted an eps-limited rank (the fp32
  // result would be redone in fp64)
  const bool try32 =
      ctx.o && ctx.o->svd_f32 && (ctx.o->rank_mode != RCS_RANK_LEARNED || ctx.pred_capped);
  if (precond && svd_split_chol(st, ws, pl, cap_eff, eps, true, log_spectra ? &spec : nullptr, r, &ldw, try32)) {
    // orthonormal factor on X's column side: the other orientation's layout
    side = 3 - orient;
    p_row = len;
    st.n_precond += 1;
  } else {
    if (precond) {
      // X may hold the column-sorted copy: restore it from X0
      HIP_OK(hipMemcpyAsync(ws.X.p, ws.X0.p, (size_t)pl.ldx * pl.cnt * sizeof(double2), hipMemcpyDeviceToDevice, s));
      st.n_precond_fallback += 1;
    }
    r = svd_split(st, ws, pl, cap_eff, eps, true, log_spectra ? &spec : nullptr);
    ldw = pl.ldx;
  }
  const int k = r.k;
  st.nominal_svd_flops += nominal_svd_flops(len, cnt);
  record_bond_spectrum(st, ws, ctx, i, k);
  if (ctx.o) ctx.prev_eps[i] = r.eps_step;
  hipLaunchKernelGGL(k_write_split, dim3(grid1d((int64_t)2 * k * (dl + dr))), dim3(256), 0, s,
                     ws.wn_final, ldw, ws.P.as<double2>(), p_row, k, dl, dr, side,
                     st.site[i], st.site[i + 1]);
  HIP_LAUNCH_OK();
  st.updates.push_back(UpdateRecord{i, cycle, dl, dm, dr, k, randomized_tried ? 2 : 0});
  st.dims[i + 1] = k;
  st.center = side == 1 ? i + 1 : i;
  st.log_fest += std::log1p(-r.eps_step);
  st.sum_eps += r.eps_step;
  st.n_trunc += 1;
  if (log_spectra) {
    SpectrumRecord rec;
    rec.pos = i;
    rec.cycle = cycle;
    rec.m = cnt;
    rec.kept = k;
    rec.chi_l = dl;
    rec.chi_r = dr;
    rec.values = std::move(spec);
    st.spectra.push_back(std::move(rec));
  }
}

static void apply_layer(rcs_state_s& st, const rcs_circuit_s& c, int layer) {
  Layer1q L;
  int64_t mx = 1;
  for (int k = 0; k < st.n; ++k) {
    L.site[k] = st.site[k];
    L.dl[k] = st.dims[k];
    L.dr[k] = st.dims[k + 1];
    L.gate[k] = (uint8_t)c.layers_1q[layer][st.pi[k]];
    mx = std::max<int64_t>(mx, (int64_t)L.dl[k] * L.dr[k]);
  }
  hipLaunchKernelGGL(k_apply_1q, dim3(grid1d(mx), st.n), dim3(256), 0, st.stream, L);
  HIP_LAUNCH_OK();
}

static void upload_gates_once() {
  static std::mutex mu;
  static std::vector<int> done_devices;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (std::find(done_devices.begin(), done_devices.end(), dev) != done_devices.end()) return;
  double2 g[3][4];
  for (int i = 0; i < 3; ++i)
    for (int e = 0; e < 4; ++e) {
      auto v = one_qubit_gate(i)[e];
      g[i][e] = make_double2(v.real(), v.imag());
    }
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_gates1q), g, sizeof(g)));
  done_devices.push_back(dev);
}

void canonicalize(rcs_state_s& st, BuildWork& ws) {
  while (st.center > 0) move_center(st, ws, false);
  DevBuf nrm;
  nrm.ensure(sizeof(double));
  hipLaunchKernelGGL(k_normalize_site, dim3(1), dim3(256), 0, st.stream, st.site[0],
                     (int64_t)2 * st.dims[0] * st.dims[1], nrm.as<double>());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(st.stream));
  st.canonical = true;
}

void build_one(rcs_state_s& st, const rcs_circuit_s& c, int chi, double eps, const BuildOptions& o,
               BuildWork& ws) {
  upload_gates_once();
  RCS_REQUIRE(c.n <= 64, "too many qubits");
  st.pi = c.snake;
  std::array<double2, 16> fs, sw;
  auto sg = swap_gate();
  for (int e = 0; e < 16; ++e) {
    fs[e] = make_double2(c.fsim[e].real(), c.fsim[e].imag());
    sw[e] = make_double2(sg[e].real(), sg[e].imag());
  }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  HIP_OK(hipEventRecord(e0, st.stream));
  st.canonical = false;
  UpdateCtx ctx;
  ctx.o = &o;
  ctx.n_cycles = c.n_cycles;
  ctx.chi_cap = chi;
  ctx.bond_k.assign(st.n, 0);
  ctx.prev_eps.assign(st.n, eps);
  ctx.scal2.ensure(8 * sizeof(double));
  if (o.rank_mode != RCS_RANK_FULL_SVD) {
    ctx.bond_spec.ensure((size_t)st.n * chi * sizeof(double));
    ctx.feat.ensure(66 * sizeof(float));
    ctx.yhat.ensure(32 * sizeof(float));
    if (o.rank_mode == RCS_RANK_LEARNED) {
      ctx.w_mlp.ensure(o.mlp.size() * sizeof(float));
      HIP_OK(hipMemcpyAsync(ctx.w_mlp.p, o.mlp.data(), o.mlp.size() * sizeof(float), hipMemcpyHostToDevice,
                            st.stream));
    }
  }
  const int nops = (int)c.ops.size();
  const int stop = (o.max_ops < 0) ? nops : std::min(nops, o.max_ops);
  // optional progress lines on stderr (RCS_PROGRESS = seconds between lines)
  const char* pe = std::getenv("RCS_PROGRESS");
  const double every = pe ? std::atof(pe) : 0.0;
  const auto t_start = std::chrono::steady_clock::now();
  double next_report = every;
  for (int oi = 0; oi < stop; ++oi) {
    if (every > 0.0) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      if (el >= next_report) {
        std::fprintf(stderr, "rcs build: op %d/%d, %.1f s (randomized: %d accepted, %d rejected, %d of them early)\n",
                     oi, stop, el, st.n_rsvd_ok, st.n_fallback, st.n_rsvd_early);
        std::fflush(stderr);
        next_report = el + every;
      }
    }
    const Op& op = c.ops[oi];
    if (op.kind == 0) {
      apply_layer(st, c, op.arg);
      continue;
    }
    // where does the next update want the centre?
    int prefer_left = 0;
    for (int nj = oi + 1; nj < nops; ++nj)
      if (c.ops[nj].kind == 1) {
        prefer_left = c.ops[nj].arg < op.arg ? 1 : 0;
        break;
      }
    two_site_update(st, ws, ctx, op.arg, op.gate == 0 ? fs.data() : sw.data(), chi, eps, prefer_left,
                    op.cycle, o.log_spectra, o.contraction);
    if (op.gate == 1) std::swap(st.pi[op.arg], st.pi[op.arg + 1]);
  }
  if (o.canonicalize) canonicalize(st, ws);
  HIP_OK(hipEventRecord(e1, st.stream));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  st.build_seconds = ms * 1e-3;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

BuildWork* new_work() { return new BuildWork(); }
void delete_work(BuildWork* w) { delete w; }

}  // namespace rcs

// ------------------------------------------------------------------ C ABI
#define RCS_API_BEGIN try {
#define RCS_API_END                                   \
  }                                                   \
  catch (const rcs::Error& e) {                       \
    rcs::set_last_error(e.what());                    \
    return e.status;                                  \
  }                                                   \
  catch (const std::exception& e) {                   \
    rcs::set_last_error(e.what());                    \
    return RCS_ERR_DEVICE;                            \
  }                                                   \
  return RCS_OK;

extern "C" {

void rcs_build_opts_default(rcs_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->contraction = RCS_PREC_C128;
  o->rank_mode = RCS_RANK_FULL_SVD;
  o->fallback_tau = 1e-6;
  o->rsvd_oversample = 16;
  o->rsvd_power_iters = 2;
  o->rsvd_seed = 0x5eed;
  o->max_ops = -1;
  o->canonicalize = 1;
  o->svd_precision = RCS_SVD_F64;
}

static rcs::BuildOptions to_options(const rcs_build_opts* opts) {
  rcs_build_opts d;
  rcs_build_opts_default(&d);
  const rcs_build_opts& o = opts ? *opts : d;
  rcs::BuildOptions b;
  RCS_REQUIRE(o.contraction >= 0 && o.contraction <= 2, "bad contraction precision");
  RCS_REQUIRE(o.rank_mode >= 0 && o.rank_mode <= 2, "bad rank mode");
  RCS_REQUIRE(o.svd_precision == RCS_SVD_F64 || o.svd_precision == RCS_SVD_F32, "bad SVD precision");
  b.contraction = o.contraction;
  b.rank_mode = o.rank_mode;
  b.fallback_tau = o.fallback_tau;
  if (o.mlp_weights_host && o.mlp_count > 0)
    b.mlp.assign(o.mlp_weights_host, o.mlp_weights_host + o.mlp_count);
  b.rsvd_p = o.rsvd_oversample;
  b.rsvd_q = o.rsvd_power_iters;
  b.rsvd_seed = o.rsvd_seed;
  b.stream = o.stream;
  b.log_spectra = o.log_spectra != 0;
  b.max_ops = o.max_ops;
  b.canonicalize = o.canonicalize != 0;
  b.svd_f32 = o.svd_precision == RCS_SVD_F32;
  if (b.rank_mode == RCS_RANK_LEARNED)
    RCS_REQUIRE((int64_t)b.mlp.size() == RCS_MLP_PARAMS, "learned mode needs the packed network weights");
  return b;
}

rcs_status rcs_build_state_ex(rcs_circuit circuit, int32_t chi, double trunc_eps,
                              const rcs_build_opts* opts, rcs_state* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(circuit && out, "null argument");
  *out = nullptr;
  RCS_REQUIRE(chi >= 1 && chi <= 2048, "chi must be in [1, 2048]");
  RCS_REQUIRE(trunc_eps >= 0.0 && trunc_eps < 1.0, "trunc_eps must be in [0, 1)");
  rcs::BuildOptions b = to_options(opts);
  auto st = std::make_unique<rcs_state_s>();
  st->stream = rcs::as_stream(b.stream);
  HIP_OK(hipGetDevice(&st->device));
  rcs::state_alloc(*st, circuit->n, chi);
  std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
  rcs::build_one(*st, *circuit, chi, trunc_eps, b, *ws);
  *out = st.release();
  RCS_API_END
}

rcs_status rcs_svd_jacobi(int32_t len, int32_t cnt, double* x_dev, double* s_dev, double* u_dev,
                          void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(x_dev && s_dev && u_dev, "null device pointer");
  RCS_REQUIRE(len >= 1 && cnt >= 1 && cnt <= rcs::SORT_MAX && len <= 16384, "bad matrix shape");
  hipStream_t s = rcs::as_stream(stream);
  rcs::JacobiPlan pl = rcs::jacobi_plan(len, cnt);
  std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
  rcs::ensure_work(*ws, pl, 0);
  HIP_OK(hipMemsetAsync(ws->X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  double2* X = ws->X.as<double2>();
  HIP_OK(hipMemsetAsync(ws->X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  hipLaunchKernelGGL(rcs::k_copy_in, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x_dev), len, cnt, ws->X0.as<double2>(), pl.ldx);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(cnt), dim3(256), 0, s, ws->X0.as<double2>(), pl.ldx, len,
                     ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  // columns in descending-norm order
  hipLaunchKernelGGL(rcs::k_sort_rank, dim3(1), dim3(1024), 0, s, ws->sigma.as<double>(), cnt, cnt, 0.0,
                     ws->sorted.as<double>(), ws->order.as<int>(), ws->scal.as<rcs::RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_permute_cols, dim3(rcs::ceil_div(len, 256), cnt), dim3(256), 0, s,
                     ws->X0.as<double2>(), pl.ldx, len, ws->order.as<int>(), X);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(cnt), dim3(256), 0, s, X, pl.ldx, len, ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sum_sq, dim3(1), dim3(256), 0, s, ws->sigma.as<double>(), cnt,
                     reinterpret_cast<double*>(ws->host_rank_dev()));
  HIP_LAUNCH_OK();
  double fro2 = 0.0;
  HIP_OK(hipMemcpyAsync(&fro2, ws->host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  rcs::jacobi_run(pl, X, ws->jac.p, ws->rot.as<int>(), ws->host_rot, fro2, s, 60);
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(cnt), dim3(256), 0, s, X, pl.ldx, len, ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sort_rank, dim3(1), dim3(1024), 0, s, ws->sigma.as<double>(), cnt, cnt, 0.0,
                     ws->sorted.as<double>(), ws->order.as<int>(), ws->scal.as<rcs::RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_copy_out, dim3(rcs::ceil_div(len, 256), cnt), dim3(256), 0, s, X, pl.ldx, len, cnt,
                     ws->order.as<int>(), ws->sorted.as<double>(), s_dev, reinterpret_cast<double2*>(u_dev));
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_svd_jacobi_f32(int32_t len, int32_t cnt, const double* x_dev, double* s_dev, double* u_dev,
                              void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(x_dev && s_dev && u_dev, "null device pointer");
  RCS_REQUIRE(len >= 1 && cnt >= 1 && cnt <= rcs::SORT_MAX && len <= 16384, "bad matrix shape");
  hipStream_t s = rcs::as_stream(stream);
  rcs::JacobiPlan pl = rcs::jacobi_plan(len, cnt);
  std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
  rcs::ensure_work(*ws, pl, 0);
  HIP_OK(hipMemsetAsync(ws->X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws->X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  double2* X = ws->X.as<double2>();
  hipLaunchKernelGGL(rcs::k_copy_in, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x_dev), len, cnt, ws->X0.as<double2>(), pl.ldx);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(cnt), dim3(256), 0, s, ws->X0.as<double2>(), pl.ldx, len,
                     ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  // columns in descending-norm order, then the fp32 copy
  hipLaunchKernelGGL(rcs::k_sort_rank, dim3(1), dim3(1024), 0, s, ws->sigma.as<double>(), cnt, cnt, 0.0,
                     ws->sorted.as<double>(), ws->order.as<int>(), ws->scal.as<rcs::RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_permute_cols, dim3(rcs::ceil_div(len, 256), cnt), dim3(256), 0, s,
                     ws->X0.as<double2>(), pl.ldx, len, ws->order.as<int>(), X);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sum_sq, dim3(1), dim3(256), 0, s, ws->sigma.as<double>(), cnt,
                     reinterpret_cast<double*>(ws->host_rank_dev()));
  HIP_LAUNCH_OK();
  const int64_t ne = (int64_t)pl.ldx * pl.cnt_pad;
  ws->Y32.ensure((size_t)ne * sizeof(float2));
  float2* X32 = ws->Y32.as<float2>();
  hipLaunchKernelGGL(rcs::k_to_c64, dim3(rcs::grid1d(ne)), dim3(256), 0, s, X, X32, ne);
  HIP_LAUNCH_OK();
  double fro2 = 0.0;
  HIP_OK(hipMemcpyAsync(&fro2, ws->host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  rcs::jacobi_run_f32(pl, X32, ws->jac.p, ws->rot.as<int>(), ws->host_rot, fro2, s, 60);
  hipLaunchKernelGGL(rcs::k_colnorm_c64, dim3(cnt), dim3(256), 0, s, X32, pl.ldx, len, ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sort_rank, dim3(1), dim3(1024), 0, s, ws->sigma.as<double>(), cnt, cnt, 0.0,
                     ws->sorted.as<double>(), ws->order.as<int>(), ws->scal.as<rcs::RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_copy_out_c64, dim3(rcs::ceil_div(len, 256), cnt), dim3(256), 0, s, X32, pl.ldx, len,
                     cnt, ws->order.as<int>(), ws->sorted.as<double>(), s_dev, reinterpret_cast<double2*>(u_dev));
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_cholqr(int32_t len, int32_t cnt, const double* x_dev, double* q_dev, double* r_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(x_dev && q_dev && r_dev, "null device pointer");
  RCS_REQUIRE(cnt >= 64 && cnt <= len && cnt <= rcs::SORT_MAX && len <= 16384, "bad matrix shape");
  hipStream_t s = rcs::as_stream(stream);
  rcs::JacobiPlan pl = rcs::jacobi_plan(len, cnt);
  std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
  rcs::ensure_work(*ws, pl, 0);
  HIP_OK(hipMemsetAsync(ws->X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws->X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  hipLaunchKernelGGL(rcs::k_copy_in, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x_dev), len, cnt, ws->X0.as<double2>(), pl.ldx);
  HIP_LAUNCH_OK();
  rcs_state_s tmp;
  tmp.stream = s;
  if (!rcs::move_cholqr(tmp, *ws, pl))
    rcs::fail(RCS_ERR_NUMERIC, "CholeskyQR: matrix rank deficient or too ill-conditioned");
  // Q out (len x cnt), R = Q^H X (cnt x cnt) as a row-major P then transposed out
  hipLaunchKernelGGL(rcs::k_project, dim3(rcs::ceil_div(cnt, rcs::GT_N), rcs::ceil_div(cnt, rcs::GT_M)),
                     dim3(rcs::GT_THREADS), 0, s, ws->wn_final, ws->X0.as<double2>(), pl.ldx, len, cnt, cnt, 1.0,
                     ws->P.as<double2>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_export_qr, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s, ws->wn_final, pl.ldx,
                     ws->P.as<double2>(), len, cnt, reinterpret_cast<double2*>(q_dev), reinterpret_cast<double2*>(r_dev));
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_rsvd(int32_t len, int32_t cnt, const double* x_dev, int32_t l, int32_t q, uint64_t seed,
                    uint64_t step, double* s_dev, double* fro2_host, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(x_dev && s_dev && fro2_host, "null pointer");
  RCS_REQUIRE(len >= 1 && cnt >= 1 && l >= 1 && l <= cnt && l <= len && q >= 0 && cnt <= rcs::SORT_MAX,
              "bad sizes");
  hipStream_t s = rcs::as_stream(stream);
  std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
  rcs::RsvdWork rw;
  const int ldm = (int)rcs::round_up(len, 64);
  rcs::DevBuf M;
  M.ensure((size_t)ldm * cnt * sizeof(double2));
  hipLaunchKernelGGL(rcs::k_copy_in, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x_dev), len, cnt, M.as<double2>(), ldm);
  HIP_LAUNCH_OK();
  rcs::range_finder(M.as<double2>(), ldm, len, cnt, l, q, seed, step, rw, s);
  rcs::JacobiPlan pl = rcs::jacobi_plan(cnt, l);
  rcs::ensure_work(*ws, pl, 0);
  ws->sigma.ensure((size_t)std::max(cnt, pl.cnt_pad) * sizeof(double));
  HIP_OK(hipMemsetAsync(ws->X.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  HIP_OK(hipMemsetAsync(ws->X0.p, 0, (size_t)pl.ldx * pl.cnt_pad * sizeof(double2), s));
  rcs::project_to_basis(M.as<double2>(), ldm, len, cnt, l, rw, ws->X.as<double2>(), ws->X0.as<double2>(), pl.ldx, s);
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(cnt), dim3(256), 0, s, M.as<double2>(), ldm, len, ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sum_sq, dim3(1), dim3(256), 0, s, ws->sigma.as<double>(), cnt,
                     reinterpret_cast<double*>(ws->host_rank_dev()));
  HIP_LAUNCH_OK();
  HIP_OK(hipMemcpyAsync(fro2_host, ws->host_rank_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  rcs::jacobi_run(pl, ws->X.as<double2>(), ws->jac.p, ws->rot.as<int>(), ws->host_rot, *fro2_host, s, 60);
  hipLaunchKernelGGL(rcs::k_colnorm, dim3(l), dim3(256), 0, s, ws->X.as<double2>(), pl.ldx, cnt,
                     ws->sigma.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_sort_rank, dim3(1), dim3(1024), 0, s, ws->sigma.as<double>(), l, l, 0.0,
                     ws->sorted.as<double>(), ws->order.as<int>(), ws->scal.as<rcs::RankOut>(), nullptr);
  HIP_LAUNCH_OK();
  HIP_OK(hipMemcpyAsync(s_dev, ws->sorted.p, l * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_rsvd_basis(int32_t len, int32_t cnt, const double* x_dev, int32_t l, int32_t q, uint64_t seed,
                          uint64_t step, double* q_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(x_dev && q_dev, "null pointer");
  RCS_REQUIRE(len >= 1 && cnt >= 1 && l >= 1 && l <= cnt && l <= len && q >= 0 && cnt <= rcs::SORT_MAX,
              "bad sizes");
  hipStream_t s = rcs::as_stream(stream);
  rcs::RsvdWork rw;
  const int ldm = (int)rcs::round_up(len, 64);
  rcs::DevBuf M;
  M.ensure((size_t)ldm * cnt * sizeof(double2));
  hipLaunchKernelGGL(rcs::k_copy_in, dim3(rcs::grid1d((int64_t)len * cnt)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(x_dev), len, cnt, M.as<double2>(), ldm);
  HIP_LAUNCH_OK();
  rcs::range_finder(M.as<double2>(), ldm, len, cnt, l, q, seed, step, rw, s);
  hipLaunchKernelGGL(rcs::k_copy_basis, dim3(rcs::grid1d((int64_t)len * l)), dim3(256), 0, s, rw.Q, rw.ldq, len, l,
                     reinterpret_cast<double2*>(q_dev));
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_two_site(int32_t dl, int32_t dm, int32_t dr, const double* a_dev, const double* b_dev,
                        const double* gate_host, int32_t precision, double* out_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(a_dev && b_dev && gate_host && out_dev, "null pointer");
  RCS_REQUIRE(dl >= 1 && dm >= 1 && dr >= 1 && dl <= 4096 && dm <= 4096 && dr <= 4096, "bad dimensions");
  RCS_REQUIRE(precision >= 0 && precision <= 2, "bad precision");
  hipStream_t s = rcs::as_stream(stream);
  rcs::DevBuf A, B, T;
  A.ensure((size_t)2 * dl * dm * sizeof(double2));
  B.ensure((size_t)2 * dm * dr * sizeof(double2));
  T.ensure((size_t)4 * dl * dr * sizeof(double2));
  hipLaunchKernelGGL(rcs::k_to_device_layout, dim3(rcs::grid1d((int64_t)2 * dl * dm)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(a_dev), dl, dm, A.as<double2>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_to_device_layout, dim3(rcs::grid1d((int64_t)2 * dm * dr)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(b_dev), dm, dr, B.as<double2>());
  HIP_LAUNCH_OK();
  rcs::contract_two_site(A.as<double2>(), B.as<double2>(), T.as<double2>(), dl, dm, dr, precision, s);
  rcs::Gate4 G;
  for (int e = 0; e < 16; ++e) G.g[e] = make_double2(gate_host[2 * e], gate_host[2 * e + 1]);
  hipLaunchKernelGGL(rcs::k_mix_gate, dim3(rcs::grid1d((int64_t)dl * dr)), dim3(256), 0, s, T.as<double2>(), G,
                     dl, dr, 1, reinterpret_cast<double2*>(out_dev), reinterpret_cast<double2*>(out_dev), 2 * dl);
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_build_state(rcs_circuit circuit, int32_t chi, double trunc_eps, rcs_state* out) {
  return rcs_build_state_ex(circuit, chi, trunc_eps, nullptr, out);
}

rcs_status rcs_build_batch(const rcs_circuit* circuits, const int32_t* chi, const double* eps,
                           int32_t n, const rcs_build_opts* opts, rcs_state* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(circuits && chi && eps && out && n >= 0, "null argument");
  for (int i = 0; i < n; ++i) out[i] = nullptr;
  for (int i = 0; i < n; ++i) {
    RCS_REQUIRE(circuits[i], "null circuit in batch");
    RCS_REQUIRE(chi[i] >= 1 && chi[i] <= 2048, "chi must be in [1, 2048]");
    RCS_REQUIRE(eps[i] >= 0.0 && eps[i] < 1.0, "eps must be in [0, 1)");
  }
  rcs::BuildOptions b = to_options(opts);
  hipStream_t caller = rcs::as_stream(b.stream);
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  // Circuits are built concurrently by worker threads, each with its own
  // stream and workspaces, taking circuits longest-first (cost ~ updates x
  // bond cap^3): the latency-bound SVD sweeps of small bonds then overlap.
  std::vector<int> order(n);
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    const double c = std::min<double>(chi[i], std::ldexp(1.0, circuits[i]->n / 2));
    cost[i] = (double)circuits[i]->ops.size() * c * c * c;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  // as many streams as the runtime's hardware queues per process (four by
  // default): more would share queues and serialise behind each other
  int n_workers = 4;
  if (const char* e = std::getenv("RCS_BATCH_STREAMS")) n_workers = std::max(1, std::min(32, std::atoi(e)));
  n_workers = std::max(1, std::min(n_workers, n));
  hipEvent_t ready;
  HIP_OK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIP_OK(hipEventRecord(ready, caller));
  std::vector<std::unique_ptr<rcs_state_s>> states(n);
  std::atomic<int> next{0};
  std::atomic<bool> stop{false};
  std::mutex err_mu;
  rcs_status err_status = RCS_OK;
  std::string err_msg;
  auto worker = [&]() {
    hipStream_t s = nullptr;
    try {
      HIP_OK(hipSetDevice(dev));
      HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      HIP_OK(hipStreamWaitEvent(s, ready, 0));
      std::unique_ptr<rcs::BuildWork, void (*)(rcs::BuildWork*)> ws(rcs::new_work(), rcs::delete_work);
      rcs::BuildOptions bo = b;
      bo.stream = s;
      for (int j = next++; j < n && !stop; j = next++) {
        const int i = order[j];
        auto st = std::make_unique<rcs_state_s>();
        st->stream = s;
        st->device = dev;
        try {
          rcs::state_alloc(*st, circuits[i]->n, chi[i]);
          rcs::build_one(*st, *circuits[i], chi[i], eps[i], bo, *ws);
          HIP_OK(hipStreamSynchronize(s));
        } catch (...) {
          // let queued work finish before the state and workspaces are freed
          (void)hipStreamSynchronize(s);
          throw;
        }
        st->stream = caller;
        states[i] = std::move(st);
      }
      HIP_OK(hipStreamSynchronize(s));
    } catch (const rcs::Error& e) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (err_status == RCS_OK) {
        err_status = e.status;
        err_msg = e.what();
      }
      stop = true;
    } catch (const std::exception& e) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (err_status == RCS_OK) {
        err_status = RCS_ERR_DEVICE;
        err_msg = e.what();
      }
      stop = true;
    }
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < n_workers; ++w) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  (void)hipEventDestroy(ready);
  if (err_status != RCS_OK) rcs::fail(err_status, err_msg);
  for (int i = 0; i < n; ++i) out[i] = states[i].release();
  RCS_API_END
}

}  // extern "C"
