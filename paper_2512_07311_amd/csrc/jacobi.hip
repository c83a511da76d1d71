// One-sided block Jacobi SVD in fp64 (Hestenes; block variant with a
// Gram-matrix inner eigensolver).
//
// X (len x cnt, complex, column-major, leading dimension ldx, zero padded to
// ldx rows and nbp*32 columns) is rotated from the right by unitary 64x64
// block rotations until every pair of columns is orthogonal to a relative
// tolerance; the columns are then sigma_j u_j.  Per sweep the nbp column
// blocks (32 columns each) meet pairwise in round-robin order (nbp-1 rounds,
// nbp/2 disjoint pairs per round).  Each round:
//   gram   : G_p = Y_p^H Y_p for Y_p = [X_bi | X_bj], split over row chunks
//            (complex MFMA GEMMs, partial Grams summed later in fixed order);
//   solve  : one workgroup per pair diagonalises the 64x64 Hermitian G_p in
//            LDS by cyclic two-sided Jacobi (parallel ordering), giving the
//            unitary V_p, unless G_p is already diagonal to tolerance;
//   update : Y_p <- Y_p V_p on the matrix cores, in place by row tiles.
// A sweep that rotates nothing ends the iteration.
#include "gemm_f64.h"
#include "jacobi.h"

namespace rcs {

constexpr int JB = 32;        // columns per block
constexpr int JP = 2 * JB;    // columns per pair (64)

__device__ inline int rr_block(int slot, int round, int nbp) {
  return slot == 0 ? 0 : ((slot - 1 + round) % (nbp - 1)) + 1;
}

__device__ inline int pair_col(int c, int bi, int bj) { return c < JB ? bi * JB + c : bj * JB + (c - JB); }

struct JacArgs {
  double2* x;
  int ldx, len, nbp, round, rows_per_chunk, n_chunks;
  double2* part;   // [pair][chunk][64][64]
  double2* v;      // [pair][64][64]
  int* flags;      // [pair]
  int* rot_count;
  double tol;
  double tiny;     // absolute floor on |g_ij|
};

__global__ __launch_bounds__(GT_THREADS) void k_jac_gram(JacArgs a) {
  __shared__ SmemC64 sm;
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  const int row0 = chunk * a.rows_per_chunk;
  const int K = min(a.rows_per_chunk, a.len - row0);
  double2* part = a.part + ((int64_t)p * a.n_chunks + chunk) * JP * JP;
  if (K <= 0) {
    for (int e = threadIdx.x; e < JP * JP; e += GT_THREADS) part[e] = make_double2(0.0, 0.0);
    return;
  }
  const double2* x = a.x;
  const int ldx = a.ldx;
  auto fa = [&](int m, int k) -> double2 {
    double2 v = x[(int64_t)pair_col(m, bi, bj) * ldx + row0 + k];
    return make_double2(v.x, -v.y);
  };
  auto fb = [&](int k, int n) -> double2 { return x[(int64_t)pair_col(n, bi, bj) * ldx + row0 + k]; };
  LoadA<decltype(fa), true> la{fa, 0, JP, K};
  LoadB<decltype(fb), false> lb{fb, 0, K, JP};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, K, sm, acc);
  acc_foreach(acc, [&](int r, int c, double re, double im) { part[r * JP + c] = make_double2(re, im); });
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Inner solver.  LDS: G and V 64x64 complex (64 KiB each).
__global__ __launch_bounds__(GT_THREADS) void k_jac_solve(JacArgs a) {
  extern __shared__ double2 lds[];
  double2* G = lds;               // [64][64]
  double2* V = lds + JP * JP;     // [64][64]
  __shared__ double rc[JP / 2], rs[JP / 2];
  __shared__ double2 re_[JP / 2];
  __shared__ int ri[JP / 2], rj[JP / 2];
  __shared__ int any_flag;
  const int p = blockIdx.x, tid = threadIdx.x;
  const double2* part = a.part + (int64_t)p * a.n_chunks * JP * JP;
  for (int e = tid; e < JP * JP; e += GT_THREADS) {
    double2 s = make_double2(0.0, 0.0);
    for (int c = 0; c < a.n_chunks; ++c) {
      double2 t = part[(int64_t)c * JP * JP + e];
      s.x += t.x;
      s.y += t.y;
    }
    G[e] = s;
    V[e] = make_double2((e / JP) == (e % JP) ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) any_flag = 0;
  __syncthreads();
  // does any pair need a rotation?
  for (int e = tid; e < JP * JP; e += GT_THREADS) {
    int i = e / JP, j = e % JP;
    if (i < j) {
      double h = sqrt(cabs2(G[e]));
      double d = sqrt(G[i * JP + i].x * G[j * JP + j].x);
      if (h > a.tol * d && h > a.tiny) any_flag = 1;
    }
  }
  __syncthreads();
  if (!any_flag) {
    if (tid == 0) a.flags[p] = 0;
    return;
  }
  const int max_inner = 20;
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    for (int round = 0; round < JP - 1; ++round) {
      if (tid < JP / 2) {
        // round-robin pairing of 64 indices
        int s0 = tid, s1 = JP - 1 - tid;
        int i = (s0 == 0) ? 0 : ((s0 - 1 + round) % (JP - 1)) + 1;
        int j = ((s1 - 1 + round) % (JP - 1)) + 1;
        if (i > j) {
          int t = i;
          i = j;
          j = t;
        }
        ri[tid] = i;
        rj[tid] = j;
        double gii = G[i * JP + i].x, gjj = G[j * JP + j].x;
        double2 g = G[i * JP + j];
        double h = sqrt(cabs2(g));
        double c = 1.0, s = 0.0;
        double2 e = make_double2(1.0, 0.0);
        if (h > a.tiny && h > 1e-300 && h > 0.5 * a.tol * sqrt(fabs(gii * gjj))) {
          double tau = (gjj - gii) / (2.0 * h);
          double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          e = make_double2(g.x / h, g.y / h);
        }
        rc[tid] = c;
        rs[tid] = s;
        re_[tid] = e;
      }
      __syncthreads();
      // columns: G <- G J, V <- V J
      for (int job = tid; job < (JP / 2) * JP; job += GT_THREADS) {
        int q = job / JP, r = job % JP;
        if (rs[q] == 0.0) continue;
        int i = ri[q], j = rj[q];
        double c = rc[q], s = rs[q];
        double2 e = re_[q], ec = cconj(e);
        double2 gi = G[r * JP + i], gj = G[r * JP + j];
        double2 t1 = cmul(ec, gj), t2 = cmul(e, gi);
        G[r * JP + i] = make_double2(c * gi.x - s * t1.x, c * gi.y - s * t1.y);
        G[r * JP + j] = make_double2(s * t2.x + c * gj.x, s * t2.y + c * gj.y);
        double2 vi = V[r * JP + i], vj = V[r * JP + j];
        double2 u1 = cmul(ec, vj), u2 = cmul(e, vi);
        V[r * JP + i] = make_double2(c * vi.x - s * u1.x, c * vi.y - s * u1.y);
        V[r * JP + j] = make_double2(s * u2.x + c * vj.x, s * u2.y + c * vj.y);
      }
      __syncthreads();
      // rows: G <- J^H G
      for (int job = tid; job < (JP / 2) * JP; job += GT_THREADS) {
        int q = job / JP, col = job % JP;
        if (rs[q] == 0.0) continue;
        int i = ri[q], j = rj[q];
        double c = rc[q], s = rs[q];
        double2 e = re_[q], ec = cconj(e);
        double2 gi = G[i * JP + col], gj = G[j * JP + col];
        double2 t1 = cmul(e, gj), t2 = cmul(ec, gi);
        G[i * JP + col] = make_double2(c * gi.x - s * t1.x, c * gi.y - s * t1.y);
        G[j * JP + col] = make_double2(s * t2.x + c * gj.x, s * t2.y + c * gj.y);
      }
      __syncthreads();
    }
    // converged?
    if (tid == 0) any_flag = 0;
    __syncthreads();
    for (int e = tid; e < JP * JP; e += GT_THREADS) {
      int i = e / JP, j = e % JP;
      if (i < j) {
        double h = sqrt(cabs2(G[e]));
        double d = sqrt(fabs(G[i * JP + i].x * G[j * JP + j].x));
        if (h > 0.5 * a.tol * d && h > a.tiny) any_flag = 1;
      }
    }
    __syncthreads();
    if (!any_flag) break;
    __syncthreads();
  }
  double2* vout = a.v + (int64_t)p * JP * JP;
  for (int e = tid; e < JP * JP; e += GT_THREADS) vout[e] = V[e];
  if (tid == 0) {
    a.flags[p] = 1;
    atomicAdd(a.rot_count, 1);
  }
}

__global__ __launch_bounds__(GT_THREADS) void k_jac_update(JacArgs a) {
  __shared__ SmemC64 sm;
  const int p = blockIdx.x, chunk = blockIdx.y;
  if (a.flags[p] == 0) return;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  const int rbeg = chunk * a.rows_per_chunk;
  const int rend = min(a.len, rbeg + a.rows_per_chunk);
  double2* x = a.x;
  const int ldx = a.ldx;
  const double2* v = a.v + (int64_t)p * JP * JP;
  for (int row0 = rbeg; row0 < rend; row0 += GT_M) {
    const int M = min(GT_M, rend - row0);
    auto fa = [&](int m, int k) -> double2 { return x[(int64_t)pair_col(k, bi, bj) * ldx + row0 + m]; };
    auto fb = [&](int k, int n) -> double2 { return v[k * JP + n]; };
    LoadA<decltype(fa), false> la{fa, 0, M, JP};
    LoadB<decltype(fb), true> lb{fb, 0, JP, JP};
    AccC64 acc;
    acc_zero(acc);
    cgemm_mainloop(la, lb, JP, sm, acc);
    // every thread finished reading this row tile (mainloop ends in a barrier)
    acc_foreach(acc, [&](int r, int c, double re, double im) {
      if (r < M) x[(int64_t)pair_col(c, bi, bj) * ldx + row0 + r] = make_double2(re, im);
    });
    __syncthreads();
  }
}

// ------------------------------------------------------------- driver
JacobiPlan jacobi_plan(int len, int cnt) {
  JacobiPlan pl;
  pl.len = len;
  pl.cnt = cnt;
  pl.ldx = (int)round_up(std::max(len, 1), 64);
  int nb = ceil_div(std::max(cnt, 1), JB);
  pl.nbp = std::max(2, nb + (nb & 1));
  pl.cnt_pad = pl.nbp * JB;
  pl.n_pairs = pl.nbp / 2;
  int target_chunks = std::max(1, 512 / pl.n_pairs);
  int max_chunks = ceil_div(len, 64);
  pl.n_chunks = std::max(1, std::min(target_chunks, max_chunks));
  pl.rows_per_chunk = (int)round_up(ceil_div(len, pl.n_chunks), 64);
  pl.n_chunks = ceil_div(len, pl.rows_per_chunk);
  return pl;
}

size_t jacobi_work_bytes(const JacobiPlan& pl) {
  return (size_t)pl.n_pairs * pl.n_chunks * JP * JP * sizeof(double2) +
         (size_t)pl.n_pairs * JP * JP * sizeof(double2) + (size_t)pl.n_pairs * sizeof(int) + 256;
}

int jacobi_run(const JacobiPlan& pl, double2* x, void* work, int* rot_count_dev,
               int* rot_count_host, double fro2, hipStream_t stream, int max_sweeps) {
  JacArgs a;
  a.x = x;
  a.ldx = pl.ldx;
  a.len = pl.len;
  a.nbp = pl.nbp;
  a.rows_per_chunk = pl.rows_per_chunk;
  a.n_chunks = pl.n_chunks;
  char* w = reinterpret_cast<char*>(work);
  a.part = reinterpret_cast<double2*>(w);
  w += (size_t)pl.n_pairs * pl.n_chunks * JP * JP * sizeof(double2);
  a.v = reinterpret_cast<double2*>(w);
  w += (size_t)pl.n_pairs * JP * JP * sizeof(double2);
  a.flags = reinterpret_cast<int*>(w);
  a.rot_count = rot_count_dev;
  a.tol = std::max(1e-15, 2.3e-16 * std::sqrt((double)pl.len));
  a.tiny = 1e-30 * std::max(fro2, 1e-300);
  const size_t solve_lds = 2 * JP * JP * sizeof(double2);
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    HIP_OK(hipMemsetAsync(rot_count_dev, 0, sizeof(int), stream));
    for (int r = 0; r < pl.nbp - 1; ++r) {
      a.round = r;
      hipLaunchKernelGGL(k_jac_gram, dim3(pl.n_pairs, pl.n_chunks), dim3(GT_THREADS), 0, stream, a);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_jac_solve, dim3(pl.n_pairs), dim3(GT_THREADS), solve_lds, stream, a);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_jac_update, dim3(pl.n_pairs, pl.n_chunks), dim3(GT_THREADS), 0, stream, a);
      HIP_LAUNCH_OK();
    }
    HIP_OK(hipMemcpyAsync(rot_count_host, rot_count_dev, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (*rot_count_host == 0) return sweep;
  }
  fail(RCS_ERR_NUMERIC, "one-sided Jacobi SVD did not converge");
}

void jacobi_init_attributes() {
  static bool done = false;
  if (done) return;
  HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_jac_solve),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(2 * JP * JP * sizeof(double2))));
  done = true;
}

}  // namespace rcs
