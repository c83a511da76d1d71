// One-sided block Jacobi SVD in fp64 (Hestenes method, block variant with a
// Gram-matrix inner eigensolver).
//
// X (len x cnt, complex, column-major, leading dimension ldx, zero padded to
// nbp*16 columns) is rotated from the right by unitary 32x32 block rotations
// until every pair of columns is orthogonal to the relative tolerance
// tol = 16 u sqrt(len) (fresh Grams keep relative accuracy; the margin over
// the rounding noise of a length-len inner product keeps noise from
// re-triggering rotations among millions of pairs), ignoring columns
// below the fp64 noise level delta ||X||_F; the columns are then
// sigma_j u_j.  Per sweep the nbp column blocks (16 columns each) meet
// pairwise in round-robin order: nbp-1 rounds of nbp/2 disjoint pairs.  A
// round is two launches:
//   gram   : G_p = Y_p^H Y_p, Y_p = [X_bi | X_bj], as partial Grams over row
//            chunks (fp64 MFMA; waves reduce in fixed order);
//   rotate : every (pair, chunk) workgroup sums the partial Grams in fixed
//            order, diagonalises the 32x32 Hermitian G_p in LDS by cyclic
//            two-sided Jacobi (all workgroups of a pair compute the same
//            unitary V_p), and applies Y_p <- Y_p V_p to its own rows on the
//            matrix cores.
// A pair whose two blocks were not rotated since the pair last met is
// skipped (it is still orthogonal), so late sweeps cost almost nothing.  A
// sweep that rotates nothing ends the iteration.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "gemm_f64.h"
#include "jacobi.h"
#include "prof.h"

namespace rcs {

constexpr int TR = 16;        // rows per wave tile

__device__ inline int rr_block(int slot, int round, int nbp) {
  return slot == 0 ? 0 : ((slot - 1 + round) % (nbp - 1)) + 1;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

struct JacArgs {
  double2* x;
  int ldx, len, nbp, round, rows_per_chunk, n_chunks;
  double2* part;      // [pair][chunk][JP][JP]
  int* rot_prev;      // [nbp] block rotated during the previous sweep
  int* rot_cur;       // [nbp] block rotated during this sweep
  int* rot_count;
  double tol;         // relative orthogonality tolerance
  double neg2;        // squared column norm below which a column counts as zero
  int max_inner;      // inner two-sided sweeps per pair meeting
};

__device__ inline bool pair_skipped(const JacArgs& a, int bi, int bj) {
  return a.rot_prev[bi] == 0 && a.rot_prev[bj] == 0 && a.rot_cur[bi] == 0 && a.rot_cur[bj] == 0;
}

template <int JP>
__device__ inline int pair_col(int c, int bi, int bj) {
  return c < JP / 2 ? bi * (JP / 2) + c : bj * (JP / 2) + (c - JP / 2);
}

// Load a 16-row x JP-column tile of Y_p (rows row0.., masked at rend) into a
// wave's LDS tile.  Each lane takes 16*JP/64 consecutive rows of one column.
template <int JP>
__device__ inline void load_tile(const double2* x, int ldx, int bi, int bj, int row0, int rend,
                                 double2 (*tile)[JP + 1], int lane) {
  constexpr int LPC = 64 / JP;          // lanes per column
  constexpr int RPL = TR / LPC;         // rows per lane
  const int c = lane / LPC, h = (lane % LPC) * RPL;
  const double2* col = x + (int64_t)pair_col<JP>(c, bi, bj) * ldx;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = row0 + h + t;
    tile[h + t][c] = (r < rend) ? col[r] : make_double2(0.0, 0.0);
  }
}

// Partial Grams.  The JP x JP output is split into 16x16 MFMA blocks; wave w
// owns blocks w, w+4, ... and all waves walk the chunk's rows together
// through per-wave LDS tiles (every wave reads every tile).
template <int JP>
__global__ __launch_bounds__(256) void k_jac_gram(JacArgs a) {
  constexpr int NB = JP / 16, NBLK = NB * NB, PER = (NBLK + 3) / 4;
  __shared__ double2 tile[4][TR][JP + 1];
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  if (pair_skipped(a, bi, bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rbeg = chunk * a.rows_per_chunk;
  const int rend = min(a.len, rbeg + a.rows_per_chunk);
  const int ngroups = (rend - rbeg + TR - 1) / TR;
  double4_t gr[PER], gi[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    gr[i] = double4_t{0, 0, 0, 0};
    gi[i] = double4_t{0, 0, 0, 0};
  }
  for (int g0 = 0; g0 < ngroups; g0 += 4) {
    const int g = g0 + w;
    if (g < ngroups) load_tile<JP>(a.x, a.ldx, bi, bj, rbeg + g * TR, rend, tile[w], lane);
    __syncthreads();
    const int nt_here = min(4, ngroups - g0);
    for (int tt = 0; tt < nt_here; ++tt) {
#pragma unroll
      for (int kk = 0; kk < TR; kk += 4) {
        const int r = kk + (lane >> 4);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int blk = w + 4 * q;
          if (blk < NBLK) {
            const int mb = blk / NB, nb = blk % NB;
            const double2 ym = tile[tt][r][mb * 16 + (lane & 15)];
            const double2 yn = tile[tt][r][nb * 16 + (lane & 15)];
            gr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ym.x, yn.x, gr[q], 0, 0, 0);
            gr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ym.y, yn.y, gr[q], 0, 0, 0);
            gi[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ym.x, yn.y, gi[q], 0, 0, 0);
            gi[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ym.y, yn.x, gi[q], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  double2* part = a.part + ((int64_t)p * a.n_chunks + chunk) * JP * JP;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int blk = w + 4 * q;
    if (blk < NBLK) {
      const int mb = blk / NB, nb = blk % NB;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mb * 16 + f64_row(lane, r), col = nb * 16 + (lane & 15);
        part[row * JP + col] = make_double2(gr[q][r], gi[q][r]);
      }
    }
  }
}

// Sum partial Grams (fixed order), diagonalise by cyclic two-sided Jacobi,
// rotate this chunk's rows.  LDS: V, and G aliased with the row tiles (G is
// dead once V is known).
template <int JP>
__global__ __launch_bounds__(256) void k_jac_rotate(JacArgs a) {
  constexpr int GS = JP + 1, NP = JP / 2, NB = JP / 16;
  constexpr int G_BYTES = JP * GS * 16, T_BYTES = 4 * TR * GS * 16;
  __shared__ double2 V[JP][GS];
  __shared__ __align__(16) char gt_raw[G_BYTES > T_BYTES ? G_BYTES : T_BYTES];
  __shared__ double rc[NP], rs[NP];
  __shared__ double2 re_[NP];
  __shared__ int ri[NP], rj[NP];
  __shared__ int any_flag;
  double2 (*G)[GS] = reinterpret_cast<double2 (*)[GS]>(gt_raw);
  double2 (*tile)[TR][GS] = reinterpret_cast<double2 (*)[TR][GS]>(gt_raw);
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  if (pair_skipped(a, bi, bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double2* part = a.part + (int64_t)p * a.n_chunks * JP * JP;
  for (int e = tid; e < JP * JP; e += 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int c = 0; c < a.n_chunks; ++c) {
      const double2 t = part[(int64_t)c * JP * JP + e];
      s.x += t.x;
      s.y += t.y;
    }
    const int i = e / JP, j = e % JP;
    G[i][j] = s;
    V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) any_flag = 0;
  __syncthreads();
  for (int e = tid; e < JP * JP; e += 256) {
    const int i = e / JP, j = e % JP;
    if (i < j) {
      const double h = sqrt(cabs2(G[i][j]));
      const double d = sqrt(fabs(G[i][i].x * G[j][j].x));
      if (h > a.tol * d && G[i][i].x > a.neg2 && G[j][j].x > a.neg2) any_flag = 1;
    }
  }
  __syncthreads();
  if (!any_flag) return;
  const double tol_in = 0.5 * a.tol, neg2 = a.neg2;
  for (int sweep = 0; sweep < a.max_inner; ++sweep) {
    for (int round = 0; round < JP - 1; ++round) {
      if (tid < NP) {
        int i = (tid == 0) ? 0 : ((tid - 1 + round) % (JP - 1)) + 1;
        int j = ((JP - 2 - tid + round) % (JP - 1)) + 1;
        if (i > j) {
          const int t = i;
          i = j;
          j = t;
        }
        ri[tid] = i;
        rj[tid] = j;
        const double gii = G[i][i].x, gjj = G[j][j].x;
        const double2 g = G[i][j];
        const double h = sqrt(cabs2(g));
        double c = 1.0, s = 0.0;
        double2 e = make_double2(1.0, 0.0);
        if (h > 1e-300 && gii > neg2 && gjj > neg2 && h > tol_in * sqrt(gii * gjj)) {
          const double tau = (gjj - gii) / (2.0 * h);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          e = make_double2(g.x / h, g.y / h);
        }
        rc[tid] = c;
        rs[tid] = s;
        re_[tid] = e;
      }
      __syncthreads();
      for (int job = tid; job < NP * JP; job += 256) {   // G <- G J, V <- V J
        const int q = job / JP, r = job % JP;
        const double s = rs[q];
        if (s == 0.0) continue;
        const int i = ri[q], j = rj[q];
        const double c = rc[q];
        const double2 e = re_[q], ec = cconj(e);
        const double2 gi = G[r][i], gj = G[r][j];
        const double2 t1 = cmul(ec, gj), t2 = cmul(e, gi);
        G[r][i] = make_double2(c * gi.x - s * t1.x, c * gi.y - s * t1.y);
        G[r][j] = make_double2(s * t2.x + c * gj.x, s * t2.y + c * gj.y);
        const double2 vi = V[r][i], vj = V[r][j];
        const double2 u1 = cmul(ec, vj), u2 = cmul(e, vi);
        V[r][i] = make_double2(c * vi.x - s * u1.x, c * vi.y - s * u1.y);
        V[r][j] = make_double2(s * u2.x + c * vj.x, s * u2.y + c * vj.y);
      }
      __syncthreads();
      for (int job = tid; job < NP * JP; job += 256) {   // G <- J^H G
        const int q = job / JP, col = job % JP;
        const double s = rs[q];
        if (s == 0.0) continue;
        const int i = ri[q], j = rj[q];
        const double c = rc[q];
        const double2 e = re_[q], ec = cconj(e);
        const double2 gi = G[i][col], gj = G[j][col];
        const double2 t1 = cmul(e, gj), t2 = cmul(ec, gi);
        G[i][col] = make_double2(c * gi.x - s * t1.x, c * gi.y - s * t1.y);
        G[j][col] = make_double2(s * t2.x + c * gj.x, s * t2.y + c * gj.y);
      }
      __syncthreads();
    }
    if (sweep + 1 == a.max_inner) break;
    if (tid == 0) any_flag = 0;
    __syncthreads();
    for (int e = tid; e < JP * JP; e += 256) {
      const int i = e / JP, j = e % JP;
      if (i < j) {
        const double h = sqrt(cabs2(G[i][j]));
        const double d = sqrt(fabs(G[i][i].x * G[j][j].x));
        if (h > tol_in * d && G[i][i].x > neg2 && G[j][j].x > neg2) any_flag = 1;
      }
    }
    __syncthreads();
    if (!any_flag) break;
    __syncthreads();
  }
  __syncthreads();   // G is dead from here on: its LDS becomes the row tiles
  const int rbeg = chunk * a.rows_per_chunk;
  const int rend = min(a.len, rbeg + a.rows_per_chunk);
  const int ngroups = (rend - rbeg + TR - 1) / TR;
  for (int g0 = 0; g0 < ngroups; g0 += 4) {
    const int g = g0 + w;
    const int row0 = rbeg + g * TR;
    if (g < ngroups) load_tile<JP>(a.x, a.ldx, bi, bj, row0, rend, tile[w], lane);
    __syncthreads();
    if (g < ngroups) {
      double4_t cr[NB], ci[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        cr[t] = double4_t{0, 0, 0, 0};
        ci[t] = double4_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int kk = 0; kk < JP; kk += 4) {
        const int k = kk + (lane >> 4);
        const double2 y = tile[w][lane & 15][k];
#pragma unroll
        for (int nt = 0; nt < NB; ++nt) {
          const double2 v = V[k][nt * 16 + (lane & 15)];
          cr[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, v.x, cr[nt], 0, 0, 0);
          cr[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.y, v.y, cr[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, v.y, ci[nt], 0, 0, 0);
          ci[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, v.x, ci[nt], 0, 0, 0);
        }
      }
#pragma unroll
      for (int nt = 0; nt < NB; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + f64_row(lane, r);
          const int col = nt * 16 + (lane & 15);
          if (row < rend)
            a.x[(int64_t)pair_col<JP>(col, bi, bj) * a.ldx + row] = make_double2(cr[nt][r], ci[nt][r]);
        }
    }
    __syncthreads();
  }
  if (chunk == 0 && tid == 0) {
    a.rot_cur[bi] = 1;
    a.rot_cur[bj] = 1;
    atomicAdd(a.rot_count, 1);
  }
}

// rot_prev <- rot_cur (or all ones before the first sweep), rot_cur <- 0,
// rot_count <- 0.
__global__ void k_jac_roll(int* rot_prev, int* rot_cur, int* rot_count, int nbp, int first) {
  for (int i = threadIdx.x; i < nbp; i += blockDim.x) {
    rot_prev[i] = first ? 1 : rot_cur[i];
    rot_cur[i] = 0;
  }
  if (threadIdx.x == 0) *rot_count = 0;
}

// ------------------------------------------------------------- driver
static bool debug_jacobi() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("RCS_DEBUG_JACOBI");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

// Tuning table: buckets (cnt_max ascending) -> block width, inner sweeps.
namespace {
struct TuneEntry {
  int cnt_max, jb, inner;
};
std::vector<TuneEntry> g_tune;
std::mutex g_tune_mu;
}  // namespace

void tuning_set(int cnt_max, int jb, int inner) {
  RCS_REQUIRE(jb == 16 || jb == 32, "block width must be 16 or 32");
  RCS_REQUIRE(inner >= 1 && inner <= 8, "inner sweeps must be in [1, 8]");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.cnt_max == cnt_max) {
      e.jb = jb;
      e.inner = inner;
      return;
    }
  g_tune.push_back({cnt_max, jb, inner});
  std::sort(g_tune.begin(), g_tune.end(), [](const TuneEntry& a, const TuneEntry& b) { return a.cnt_max < b.cnt_max; });
}

void tuning_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

static void tuned(int cnt, int* jb, int* inner) {
  *jb = cnt >= 512 ? 32 : 16;
  *inner = 1;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : g_tune)
      if (cnt <= e.cnt_max) {
        *jb = e.jb;
        *inner = e.inner;
        break;
      }
  }
  const char* b = std::getenv("RCS_JACOBI_BLOCK");
  if (b && (std::atoi(b) == 16 || std::atoi(b) == 32)) *jb = std::atoi(b);
  const char* i = std::getenv("RCS_JACOBI_INNER");
  if (i && std::atoi(i) >= 1 && std::atoi(i) <= 8) *inner = std::atoi(i);
}

JacobiPlan jacobi_plan(int len, int cnt, int jb) {
  JacobiPlan pl;
  int tjb, tin;
  tuned(cnt, &tjb, &tin);
  if (jb <= 0) jb = tjb;
  pl.inner = tin;
  RCS_REQUIRE(jb == 16 || jb == 32, "Jacobi block must be 16 or 32 columns");
  pl.jb = jb;
  pl.len = len;
  pl.cnt = cnt;
  pl.ldx = (int)round_up(std::max(len, 1), 64);
  int nb = ceil_div(std::max(cnt, 1), jb);
  pl.nbp = std::max(2, nb + (nb & 1));
  pl.cnt_pad = pl.nbp * jb;
  pl.n_pairs = pl.nbp / 2;
  const int target_chunks = std::max(1, 256 / pl.n_pairs);
  const int max_chunks = ceil_div(len, 64);
  pl.n_chunks = std::max(1, std::min(target_chunks, max_chunks));
  pl.rows_per_chunk = (int)round_up(ceil_div(len, pl.n_chunks), TR);
  pl.n_chunks = ceil_div(len, pl.rows_per_chunk);
  return pl;
}

size_t jacobi_work_bytes(const JacobiPlan& pl) {
  const int JP = 2 * pl.jb;
  return (size_t)pl.n_pairs * pl.n_chunks * JP * JP * sizeof(double2) + 2 * (size_t)pl.nbp * sizeof(int) +
         256;
}

static void launch_sweep(const JacobiPlan& pl, JacArgs a, hipStream_t stream, bool first) {
  hipLaunchKernelGGL(k_jac_roll, dim3(1), dim3(256), 0, stream, a.rot_prev, a.rot_cur, a.rot_count, pl.nbp,
                     first ? 1 : 0);
  HIP_LAUNCH_OK();
  for (int r = 0; r < pl.nbp - 1; ++r) {
    a.round = r;
    // nominal algorithmic work of a round with every pair active: Gram and
    // update are each n_pairs complex GEMMs of len x JP x JP
    const double JPd = 2.0 * pl.jb;
    const double fl = 8.0 * pl.len * JPd * JPd * pl.n_pairs;
    const double by = 16.0 * (double)pl.len * JPd * pl.n_pairs;
    {
      Probe pr(kKcJacGram, stream, fl, by);
      if (pl.jb == 16)
        hipLaunchKernelGGL(k_jac_gram<32>, dim3(pl.n_pairs, pl.n_chunks), dim3(256), 0, stream, a);
      else
        hipLaunchKernelGGL(k_jac_gram<64>, dim3(pl.n_pairs, pl.n_chunks), dim3(256), 0, stream, a);
    }
    HIP_LAUNCH_OK();
    {
      Probe pr(kKcJacRotate, stream, fl, 2.0 * by);
      if (pl.jb == 16)
        hipLaunchKernelGGL(k_jac_rotate<32>, dim3(pl.n_pairs, pl.n_chunks), dim3(256), 0, stream, a);
      else
        hipLaunchKernelGGL(k_jac_rotate<64>, dim3(pl.n_pairs, pl.n_chunks), dim3(256), 0, stream, a);
    }
    HIP_LAUNCH_OK();
  }
}

static bool use_graphs() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("RCS_JACOBI_GRAPH");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

// Cached executable graphs of one sweep (not the first), keyed by the plan
// and the buffers they were captured with.
namespace {
struct SweepGraph {
  int len, cnt, jb, inner;
  void *x, *work;
  int* rc;
  hipGraphExec_t exec;
};
std::vector<SweepGraph> g_graphs;
std::mutex g_graph_mu;
}  // namespace

static hipGraphExec_t sweep_graph(const JacobiPlan& pl, const JacArgs& a, void* work, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& g : g_graphs)
    if (g.len == pl.len && g.cnt == pl.cnt && g.jb == pl.jb && g.inner == a.max_inner && g.x == a.x &&
        g.work == work && g.rc == a.rot_count)
      return g.exec;
  hipStream_t cs;
  HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  launch_sweep(pl, a, cs, false);
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  HIP_OK(e);
  if (g_graphs.size() > 64) {
    for (auto& g : g_graphs) (void)hipGraphExecDestroy(g.exec);
    g_graphs.clear();
  }
  g_graphs.push_back({pl.len, pl.cnt, pl.jb, a.max_inner, a.x, work, a.rot_count, exec});
  (void)stream;
  return exec;
}

int jacobi_run(const JacobiPlan& pl, double2* x, void* work, int* rot_count_dev, int* rot_count_host,
               double fro2, hipStream_t stream, int max_sweeps) {
  JacArgs a;
  a.x = x;
  a.ldx = pl.ldx;
  a.len = pl.len;
  a.nbp = pl.nbp;
  a.rows_per_chunk = pl.rows_per_chunk;
  a.n_chunks = pl.n_chunks;
  a.round = 0;
  char* w = reinterpret_cast<char*>(work);
  a.part = reinterpret_cast<double2*>(w);
  w += (size_t)pl.n_pairs * pl.n_chunks * (2 * pl.jb) * (2 * pl.jb) * sizeof(double2);
  a.rot_prev = reinterpret_cast<int*>(w);
  a.rot_cur = a.rot_prev + pl.nbp;
  a.rot_count = rot_count_dev;
  a.tol = 16.0 * 1.11e-16 * std::sqrt((double)std::max(pl.len, 16));
  // columns shorter than delta ||X||_F (delta = 8 u sqrt(len)) are numerically
  // zero: below the absolute accuracy of any fp64 SVD, and they must not be
  // required to be mutually orthogonal (a wide matrix has more columns than
  // its rank)
  const double delta = 8.0 * 1.11e-16 * std::sqrt((double)pl.len);
  a.neg2 = delta * delta * std::max(fro2, 1e-300);
  a.max_inner = pl.inner;
  const bool graphs = use_graphs() && pl.nbp > 4;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    if (graphs && sweep > 1) {
      HIP_OK(hipGraphLaunch(sweep_graph(pl, a, work, stream), stream));
    } else {
      launch_sweep(pl, a, stream, sweep == 1);
    }
    HIP_OK(hipMemcpyAsync(rot_count_host, rot_count_dev, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (debug_jacobi())
      std::fprintf(stderr, "jacobi %dx%d sweep %d: %d pair rotations\n", pl.len, pl.cnt, sweep, *rot_count_host);
    if (*rot_count_host == 0) return sweep;
  }
  fail(RCS_ERR_NUMERIC, "one-sided Jacobi SVD did not converge");
}

void jacobi_init_attributes() {}

}  // namespace rcs

extern "C" {

rcs_status rcs_tuning_set(int32_t cnt_max, int32_t block, int32_t inner_sweeps) {
  try {
    rcs::tuning_set(cnt_max, block, inner_sweeps);
  } catch (const rcs::Error& e) {
    rcs::set_last_error(e.what());
    return e.status;
  }
  return RCS_OK;
}

void rcs_tuning_clear(void) { rcs::tuning_clear(); }

}  // extern "C"
