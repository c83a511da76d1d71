// One-sided block Jacobi SVD (Hestenes method, block variant with a
// Gram-matrix inner eigensolver), in fp64 or fp32 (complex128 / complex64
// data, the matching matrix-core products; R below is the real type and u
// its unit roundoff).
//
// X (len x cnt, complex, column-major, leading dimension ldx, zero padded to
// nbp*16 columns) is rotated from the right by unitary 32x32 block rotations
// until every pair of columns is orthogonal to the relative tolerance
// tol = 16 u sqrt(len) (fresh Grams keep relative accuracy; the margin over
// the rounding noise of a length-len inner product keeps noise from
// re-triggering rotations among millions of pairs), ignoring columns
// below the noise level delta ||X||_F; the columns are then
// sigma_j u_j.  Per sweep the nbp column blocks (16 columns each) meet
// pairwise in round-robin order: nbp-1 rounds of nbp/2 disjoint pairs.  A
// round is two launches:
//   gram   : G_p = Y_p^H Y_p, Y_p = [X_bi | X_bj], as partial Grams over row
//            chunks (MFMA in R; waves reduce in fixed order);
//   rotate : every (pair, chunk) workgroup sums the partial Grams in fixed
//            order, diagonalises the 32x32 Hermitian G_p in LDS by cyclic
//            two-sided Jacobi (all workgroups of a pair compute the same
//            unitary V_p), and applies Y_p <- Y_p V_p to its own rows on the
//            matrix cores.
// A pair whose two blocks were not rotated since the pair last met is
// skipped (it is still orthogonal), so late sweeps cost almost nothing.  A
// sweep that rotates nothing ends the iteration, and so does a sweep whose
// meetings all entered with squared cosines below tol / 100 (the rotate
// pass raises a flag otherwise): at that point convergence is quadratic and
// the next sweep would rotate nothing.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <vector>

#include "gemm_f64.h"
#include "jacobi.h"
#include "prof.h"

namespace rcs {

constexpr int TR = 16;        // rows per wave tile (four 4-row MFMA k steps)

// Per-precision pieces: the complex type, the 16x16x4 matrix-core product
// and the row of accumulator element r in a lane (the fp64 instruction
// interleaves rows, the fp32 one gives each 16-lane group four consecutive
// rows).
template <typename R>
struct JT;
template <>
struct JT<double> {
  using C = double2;
  using V4 = double4_t;
  static constexpr double u = 1.11e-16;
  static constexpr double tiny = 1e-300;
  __device__ static V4 mma(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int orow(int lane, int r) { return (lane >> 4) + 4 * r; }
  __host__ __device__ static C mk(double x, double y) { return make_double2(x, y); }
};
template <>
struct JT<float> {
  using C = float2;
  using V4 = float4_t;
  static constexpr double u = 5.97e-8;
  static constexpr float tiny = 1e-36f;
  __device__ static V4 mma(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
  __host__ __device__ static C mk(float x, float y) { return make_float2(x, y); }
};

__device__ inline int rr_block(int slot, int round, int nbp) {
  return slot == 0 ? 0 : ((slot - 1 + round) % (nbp - 1)) + 1;
}

template <typename R>
struct JacArgs {
  typename JT<R>::C* x;
  int ldx, len, nbp, round, rows_per_chunk, n_chunks;   // rotate chunks
  int rows_per_gchunk, n_gchunks;                      // Gram chunks
  typename JT<R>::C* part;   // [pair][chunk][JP][JP]
  int* rot_prev;      // [nbp] block rotated during the previous sweep
  int* rot_cur;       // [nbp] block rotated during this sweep
  int* rot_count;
  int* big_cos;       // set when a meeting entered with |g_ij|^2 > qtol g_ii g_jj
  R qtol;             // squared-cosine level below which the next sweep would rotate nothing
  R tol;              // relative orthogonality tolerance
  R neg2;             // squared column norm below which a column counts as zero
  int max_inner;      // inner two-sided sweeps per pair meeting
};

template <typename R>
__device__ inline bool pair_skipped(const JacArgs<R>& a, int bi, int bj) {
  return a.rot_prev[bi] == 0 && a.rot_prev[bj] == 0 && a.rot_cur[bi] == 0 && a.rot_cur[bj] == 0;
}

template <int JP>
__device__ inline int pair_col(int c, int bi, int bj) {
  return c < JP / 2 ? bi * (JP / 2) + c : bj * (JP / 2) + (c - JP / 2);
}

// Lane's element of every 16-column block of Y_p at one row (zero past
// rend).  The lane's column within a block is lane % 16, so a load
// instruction covers 16 columns x 4 consecutive rows.
template <int JP, typename C>
__device__ inline void load_row(const C* x, int ldx, int bi, int bj, int row, int rend, C (&v)[JP / 16], int lane) {
#pragma unroll
  for (int cb = 0; cb < JP / 16; ++cb) {
    const int col = pair_col<JP>(cb * 16 + (lane & 15), bi, bj);
    v[cb] = row < rend ? x[(int64_t)col * ldx + row] : C(0, 0);
  }
}

// Partial Grams.  Waves split the chunk's rows (16-row tiles, interleaved)
// and each accumulates the NB(NB+1)/2 upper 16x16 blocks of Y^H Y on the
// matrix cores straight from registers; the four waves are then reduced in
// the fixed order ((w3 + w2) + w1) + w0 through LDS.
template <int JP, typename R>
__global__ __launch_bounds__(256) void k_jac_gram(JacArgs<R> a) {
  using T = JT<R>;
  using C = typename T::C;
  using V4 = typename T::V4;
  constexpr int NB = JP / 16, NU = NB * (NB + 1) / 2;
  __shared__ R red[NU * 8][64];
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  if (pair_skipped(a, bi, bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rbeg = chunk * a.rows_per_gchunk;
  const int rend = min(a.len, rbeg + a.rows_per_gchunk);
  const int ntiles = (rend - rbeg + TR - 1) / TR;
  V4 gr[NU], gi[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    gr[u] = V4{0, 0, 0, 0};
    gi[u] = V4{0, 0, 0, 0};
  }
  C cur[4][NB], nxt[4][NB];
  const int rsub = lane >> 4;
  if (w < ntiles) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      load_row<JP>(a.x, a.ldx, bi, bj, rbeg + w * TR + 4 * ks + rsub, rend, cur[ks], lane);
  }
  for (int t = w; t < ntiles; t += 4) {
    if (t + 4 < ntiles) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        load_row<JP>(a.x, a.ldx, bi, bj, rbeg + (t + 4) * TR + 4 * ks + rsub, rend, nxt[ks], lane);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      int u = 0;
#pragma unroll
      for (int mb = 0; mb < NB; ++mb)
#pragma unroll
        for (int nb = mb; nb < NB; ++nb, ++u) {
          const C ym = cur[ks][mb], yn = cur[ks][nb];
          gr[u] = T::mma(ym.x, yn.x, gr[u]);
          gr[u] = T::mma(ym.y, yn.y, gr[u]);
          gi[u] = T::mma(ym.x, yn.y, gi[u]);
          gi[u] = T::mma(-ym.y, yn.x, gi[u]);
        }
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) cur[ks][cb] = nxt[ks][cb];
  }
  for (int src = 3; src >= 1; --src) {
    if (w == src) {
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          R vr = gr[u][r], vi = gi[u][r];
          if (src < 3) {
            vr += red[u * 8 + r][lane];
            vi += red[u * 8 + 4 + r][lane];
          }
          red[u * 8 + r][lane] = vr;
          red[u * 8 + 4 + r][lane] = vi;
        }
    }
    __syncthreads();
  }
  if (w != 0) return;
  C* part = a.part + ((int64_t)p * a.n_gchunks + chunk) * JP * JP;
  int u = 0;
#pragma unroll
  for (int mb = 0; mb < NB; ++mb)
#pragma unroll
    for (int nb = mb; nb < NB; ++nb, ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const R vr = gr[u][r] + red[u * 8 + r][lane];
        const R vi = gi[u][r] + red[u * 8 + 4 + r][lane];
        const int row = mb * 16 + T::orow(lane, r), col = nb * 16 + (lane & 15);
        part[row * JP + col] = T::mk(vr, vi);
        if (mb != nb) part[col * JP + row] = T::mk(vr, -vi);
      }
}

// 1/sqrt(x) for normal positive x: hardware estimate plus two Newton steps
// (each doubles the correct bits; the estimate carries about 23), i.e.
// within a couple of ulps.
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-h * r, r, 0.5);
  return fma(r, e, r);
}

// Plane rotation J = [[c, s e], [-s conj(e), c]] (rows: old columns i < j,
// columns: new) that (nearly) zeroes G_ij of the Hermitian 2x2 [[gii, g],
// [conj g, gjj]] in J^H G J; the identity when the pair is already
// orthogonal to tol or either column is negligible.
//
// Only unitarity has to hold to fp64 accuracy: the angle may be a few
// 1e-8 off (it leaves an off-diagonal of that relative size, which the
// next sweep's fresh Gram sees and removes, so convergence stays
// quadratic).  Hence e = g * rsq(|g|^2) with the raw hardware estimate
// (exact phase, modulus within ~2^-23 of one), tan(theta) in fp32 from
// tau = (gjj - gii) / (2|g|) (the smaller-angle root, |t| <= 1), and
// c = 1/sqrt(1 + t^2 |e|^2) refined in fp64, s = t c, which makes
// c^2 + s^2 |e|^2 = 1 to rounding.  Branch-free: inactive pairs select the
// identity.
template <typename R>
struct Rot {
  R c, s, ex, ey;
};
template <typename R>
__device__ inline bool rot_active(R gii, R gjj, R h2, R tol, R neg2) {
  return gii > neg2 && gjj > neg2 && h2 > JT<R>::tiny && h2 > tol * tol * gii * gjj;
}
__device__ inline Rot<double> jac_rot(double gii, double gjj, double2 g, double tol, double neg2) {
  const double h2 = g.x * g.x + g.y * g.y;
  const bool act = rot_active<double>(gii, gjj, h2, tol, neg2);
  const double rh = __builtin_amdgcn_rsq(fmax(h2, 1e-300));
  const double tau = (gjj - gii) * (0.5 * rh);
  const float tf = (float)fabs(tau);
  const float t32 = tf > 1e18f ? 0.5f * __builtin_amdgcn_rcpf(tf)
                               : __builtin_amdgcn_rcpf(tf + __builtin_amdgcn_sqrtf(fmaf(tf, tf, 1.0f)));
  const double t = tau < 0.0 ? -(double)t32 : (double)t32;
  const double ex = g.x * rh, ey = g.y * rh;
  const double c = rsqrt_nr(fma(t * t, ex * ex + ey * ey, 1.0));
  Rot<double> r;
  r.c = act ? c : 1.0;
  r.s = act ? t * c : 0.0;
  r.ex = act ? ex : 1.0;
  r.ey = act ? ey : 0.0;
  return r;
}

// fp32: the same rotation with every step in fp32; c takes one Newton step
// on the hardware 1/sqrt estimate, so c^2 (1 + t^2 |e|^2) = 1 to fp32
// rounding.
__device__ inline Rot<float> jac_rot(float gii, float gjj, float2 g, float tol, float neg2) {
  const float h2 = g.x * g.x + g.y * g.y;
  const bool act = rot_active<float>(gii, gjj, h2, tol, neg2);
  const float rh = __builtin_amdgcn_rsqf(fmaxf(h2, JT<float>::tiny));
  const float tau = (gjj - gii) * (0.5f * rh);
  const float tf = fabsf(tau);
  const float t32 = tf > 1e18f ? 0.5f * __builtin_amdgcn_rcpf(tf)
                               : __builtin_amdgcn_rcpf(tf + __builtin_amdgcn_sqrtf(fmaf(tf, tf, 1.0f)));
  const float t = tau < 0.0f ? -t32 : t32;
  const float ex = g.x * rh, ey = g.y * rh;
  const float x = fmaf(t * t, ex * ex + ey * ey, 1.0f);
  float c = __builtin_amdgcn_rsqf(x);
  c = fmaf(c, fmaf(-0.5f * x * c, c, 0.5f), c);
  Rot<float> r;
  r.c = act ? c : 1.0f;
  r.s = act ? t * c : 0.0f;
  r.ex = act ? ex : 1.0f;
  r.ey = act ? ey : 0.0f;
  return r;
}

// With a = s e (precomputed once per rotation: RotA = {c, Re a, Im a}):
// right action (X J):  x_i' = c x_i - conj(a) x_j,  x_j' = a x_i + c x_j;
// left action (J^H X): x_i' = c x_i - a x_j,        x_j' = conj(a) x_i + c x_j.
template <typename R>
struct RotA {
  R c, ax, ay;
};
template <typename R>
__device__ inline RotA<R> rot_a(const Rot<R>& r) { return RotA<R>{r.c, r.s * r.ex, r.s * r.ey}; }
template <typename R, typename C>
__device__ inline void rot_right(const RotA<R>& r, C& xi, C& xj) {
  const R ax = r.ax, ay = r.ay;
  const C ni(fma(r.c, xi.x, -fma(ax, xj.x, ay * xj.y)), fma(r.c, xi.y, fma(ay, xj.x, -ax * xj.y)));
  xj = C(fma(r.c, xj.x, fma(ax, xi.x, -ay * xi.y)), fma(r.c, xj.y, fma(ax, xi.y, ay * xi.x)));
  xi = ni;
}
template <typename R, typename C>
__device__ inline void rot_left(const RotA<R>& r, C& xi, C& xj) {
  const R ax = r.ax, ay = r.ay;
  const C ni(fma(r.c, xi.x, -fma(ax, xj.x, -ay * xj.y)), fma(r.c, xi.y, -fma(ax, xj.y, ay * xj.x)));
  xj = C(fma(r.c, xj.x, fma(ax, xi.x, ay * xi.y)), fma(r.c, xj.y, fma(ax, xi.y, -ay * xi.x)));
  xi = ni;
}

// Members (i < j) of pair q in round-robin round `round` of JP columns, and
// the pair that column c belongs to in that round.
template <int JP>
__device__ inline void rr_pair(int q, int round, int& i, int& j) {
  const int u = q == 0 ? 0 : ((q - 1 + round) % (JP - 1)) + 1;
  const int v = ((JP - 2 - q + round) % (JP - 1)) + 1;
  i = min(u, v);
  j = max(u, v);
}
template <int JP>
__device__ inline int rr_pair_of(int c, int round) {
  const int slot = c == 0 ? 0 : ((c - 1 - round + 2 * (JP - 1)) % (JP - 1)) + 1;
  return min(slot, JP - 1 - slot);
}

// Sum partial Grams (fixed order), diagonalise the JP x JP Hermitian G_p by
// cyclic two-sided Jacobi in LDS (every workgroup of a pair computes the
// same unitary V_p), and rotate this chunk's rows, Y_p <- Y_p V_p, on the
// matrix cores.
//
// Inner solve: a round applies JP/2 disjoint rotations at once.  JP/2 lanes
// compute the round's rotations into LDS; then waves 0-3 take the (JP/2)^2
// blocks G[pair a, pair b] <- J_a^H G[a, b] J_b and waves 4-7 the blocks
// V[rows of a, pair b] <- V J_b (one of each per SIMD, so their latencies
// overlap), all in place: each entry belongs to one job per round.  The
// diagonal and the next round's pair entries are handed on through small
// double-buffered arrays.
constexpr int ROT_THREADS = 512;
template <int JP, typename R>
__global__ __launch_bounds__(ROT_THREADS) void k_jac_rotate(JacArgs<R> a) {
  using T = JT<R>;
  using C = typename T::C;
  using V4 = typename T::V4;
  constexpr int GS = JP + 1, NP = JP / 2, NB = JP / 16, JOBS = NP * NP / 256;
  static_assert(NP * NP % 256 == 0, "block jobs must tile a wave group");
  __shared__ C G[JP][GS];
  __shared__ C V[JP][GS];
  __shared__ R dd[2][JP];
  __shared__ C od[2][NP];
  __shared__ unsigned char tb_i[JP - 1][NP], tb_j[JP - 1][NP], tb_q[JP - 1][JP];
  __shared__ RotA<R> rp[NP];
  __shared__ int any_flag;
  __shared__ int big_lds;
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int bi = rr_block(p, a.round, a.nbp), bj = rr_block(a.nbp - 1 - p, a.round, a.nbp);
  if (pair_skipped(a, bi, bj)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const C* part = a.part + (int64_t)p * a.n_gchunks * JP * JP;
  for (int e = tid; e < JP * JP; e += ROT_THREADS) {
    // partials summed in chunk order; loads issued eight at a time
    C s(0, 0);
    for (int c0 = 0; c0 < a.n_gchunks; c0 += 8) {
      C t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        t[u] = c0 + u < a.n_gchunks ? part[(int64_t)(c0 + u) * JP * JP + e] : C(0, 0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s.x += t[u].x;
        s.y += t[u].y;
      }
    }
    const int i = e / JP, j = e % JP;
    G[i][j] = s;
    V[i][j] = T::mk(i == j ? 1 : 0, 0);
  }
  if (tid == 0) {
    any_flag = 0;
    big_lds = 0;
  }
  // Inner schedule tables: members of pair q and the pair of column c, per
  // round.  The first outer round of a sweep runs the full round-robin over
  // all JP(JP-1)/2 column pairs (every block meets there, so every
  // intra-block pair is rotated once per sweep); the other outer rounds
  // rotate only the (JP/2)^2 cross pairs, column q of block bi against
  // column (q + t) mod JP/2 of block bj in round t.  Every column pair is
  // thus rotated at least once per sweep, as in cyclic Jacobi, at half the
  // inner rounds.
  const bool full = a.round == 0;
  const int n_in = full ? JP - 1 : NP;
  for (int e = tid; e < n_in * NP; e += ROT_THREADS) {
    const int rd = e / NP, q = e % NP;
    int i, j;
    if (full) {
      rr_pair<JP>(q, rd, i, j);
    } else {
      i = q;
      j = NP + (q + rd) % NP;
    }
    tb_i[rd][q] = (unsigned char)i;
    tb_j[rd][q] = (unsigned char)j;
  }
  for (int e = tid; e < n_in * JP; e += ROT_THREADS) {
    const int rd = e / JP, c = e % JP;
    tb_q[rd][c] = (unsigned char)(full ? rr_pair_of<JP>(c, rd) : (c < NP ? c : (c - NP - rd + NP) % NP));
  }
  __syncthreads();
  // only the pairs this meeting's schedule rotates decide whether it acts
  for (int e = tid; e < JP * JP; e += ROT_THREADS) {
    const int i = e / JP, j = e % JP;
    if (i < j && (full || (i < NP && j >= NP))) {
      const R gii = G[i][i].x, gjj = G[j][j].x, h2 = G[i][j].x * G[i][j].x + G[i][j].y * G[i][j].y;
      if (rot_active<R>(gii, gjj, h2, a.tol, a.neg2)) any_flag = 1;
      if (gii > a.neg2 && gjj > a.neg2 && h2 > a.qtol * gii * gjj) big_lds = 1;
    }
  }
  for (int c = tid; c < JP; c += ROT_THREADS) dd[0][c] = G[c][c].x;
  for (int q = tid; q < NP; q += ROT_THREADS) od[0][q] = G[tb_i[0][q]][tb_j[0][q]];
  __syncthreads();
  if (chunk == 0 && tid == 0 && big_lds) *a.big_cos = 1;
  if (!any_flag) return;
  const R tol_in = R(0.5) * a.tol, neg2 = a.neg2;
  const int rounds = a.max_inner * n_in;
  const bool g_waves = w < 4;          // wave-uniform role
  const int t = tid & 255;
  int buf = 0, round = 0;
  for (int it = 0; it < rounds; ++it) {
    const int nround = round + 1 == n_in ? 0 : round + 1;
    // the round's rotations, once each
    if (tid < NP) {
      const int i = tb_i[round][tid], j = tb_j[round][tid];
      rp[tid] = rot_a(jac_rot(dd[buf][i], dd[buf][j], od[buf][tid], tol_in, neg2));
    }
    __syncthreads();
    const int pb = t % NP;
    const int ib = tb_i[round][pb], jb = tb_j[round][pb];
    const RotA<R> rb = rp[pb];
    if (g_waves) {
#pragma unroll
      for (int k = 0; k < JOBS; ++k) {
        const int pa = (t + 256 * k) / NP;
        const int ia = tb_i[round][pa], ja = tb_j[round][pa];
        const RotA<R> ra = rp[pa];
        C g00 = G[ia][ib], g01 = G[ia][jb], g10 = G[ja][ib], g11 = G[ja][jb];
        rot_right(rb, g00, g01);
        rot_right(rb, g10, g11);
        rot_left(ra, g00, g10);
        rot_left(ra, g01, g11);
        G[ia][ib] = g00;
        G[ia][jb] = g01;
        G[ja][ib] = g10;
        G[ja][jb] = g11;
        // hand on the diagonal and the next round's pair entries
        if (pa == pb) {
          dd[buf ^ 1][ia] = g00.x;
          dd[buf ^ 1][ja] = g11.x;
        }
        const int qa = tb_q[nround][ia], qa2 = tb_q[nround][ja];
        const int qb = tb_q[nround][ib], qb2 = tb_q[nround][jb];
        if (ia < ib && qa == qb) od[buf ^ 1][qa] = g00;
        if (ia < jb && qa == qb2) od[buf ^ 1][qa] = g01;
        if (ja < ib && qa2 == qb) od[buf ^ 1][qa2] = g10;
        if (ja < jb && qa2 == qb2) od[buf ^ 1][qa2] = g11;
      }
    } else {
#pragma unroll
      for (int k = 0; k < JOBS; ++k) {
        const int pa = (t + 256 * k) / NP;
        const int ia = tb_i[round][pa], ja = tb_j[round][pa];
        C v0 = V[ia][ib], v1 = V[ia][jb], v2 = V[ja][ib], v3 = V[ja][jb];
        rot_right(rb, v0, v1);
        rot_right(rb, v2, v3);
        V[ia][ib] = v0;
        V[ia][jb] = v1;
        V[ja][ib] = v2;
        V[ja][jb] = v3;
      }
    }
    buf ^= 1;
    round = nround;
    __syncthreads();
  }
  // Y_p <- Y_p V_p: waves take 16-row tiles; A operand straight from global
  // (16 consecutive rows of one column per 16 lanes), B = V from LDS.
  const int rbeg = chunk * a.rows_per_chunk;
  const int rend = min(a.len, rbeg + a.rows_per_chunk);
  const int ntiles = (rend - rbeg + TR - 1) / TR;
  constexpr int KS = JP / 4, NW = ROT_THREADS / 64;
  C cur[KS], nxt[KS];
  const int m = lane & 15, ksub = lane >> 4;
  auto load_tile_regs = [&](int tt, C (&v)[KS]) {
    const int row = rbeg + tt * TR + m;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int col = pair_col<JP>(4 * ks + ksub, bi, bj);
      v[ks] = row < rend ? a.x[(int64_t)col * a.ldx + row] : C(0, 0);
    }
  };
  if (w < ntiles) load_tile_regs(w, cur);
  for (int tt = w; tt < ntiles; tt += NW) {
    if (tt + NW < ntiles) load_tile_regs(tt + NW, nxt);
    V4 cr[NB], ci[NB];
#pragma unroll
    for (int nt = 0; nt < NB; ++nt) {
      cr[nt] = V4{0, 0, 0, 0};
      ci[nt] = V4{0, 0, 0, 0};
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const C y = cur[ks];
      const int k = 4 * ks + ksub;
#pragma unroll
      for (int nt = 0; nt < NB; ++nt) {
        const C v = V[k][nt * 16 + m];
        cr[nt] = T::mma(y.x, v.x, cr[nt]);
        cr[nt] = T::mma(-y.y, v.y, cr[nt]);
        ci[nt] = T::mma(y.x, v.y, ci[nt]);
        ci[nt] = T::mma(y.y, v.x, ci[nt]);
      }
    }
    const int row0 = rbeg + tt * TR;
#pragma unroll
    for (int nt = 0; nt < NB; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + T::orow(lane, r);
        const int col = nt * 16 + m;
        if (row < rend) a.x[(int64_t)pair_col<JP>(col, bi, bj) * a.ldx + row] = T::mk(cr[nt][r], ci[nt][r]);
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) cur[ks] = nxt[ks];
  }
  if (chunk == 0 && tid == 0) {
    a.rot_cur[bi] = 1;
    a.rot_cur[bj] = 1;
    atomicAdd(a.rot_count, 1);
  }
}

// rot_prev <- rot_cur (or all ones before the first sweep), rot_cur <- 0,
// rot_count <- 0, big_cos <- 0.
__global__ void k_jac_roll(int* rot_prev, int* rot_cur, int* rot_count, int* big_cos, int nbp, int first) {
  for (int i = threadIdx.x; i < nbp; i += blockDim.x) {
    rot_prev[i] = first ? 1 : rot_cur[i];
    rot_cur[i] = 0;
  }
  if (threadIdx.x == 0) {
    *rot_count = 0;
    *big_cos = 0;
  }
}

// ------------------------------------------------------------- driver
static bool debug_jacobi() {
  static const bool v = [] {
    const char* e = std::getenv("RCS_DEBUG_JACOBI");
    return e && e[0] == '1';
  }();
  return v;
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
  *jb = 16;
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
  static const int wgs = [] {
    const char* e = std::getenv("RCS_JACOBI_WGS");
    const int v = e ? std::atoi(e) : 0;
    return v >= 64 && v <= 4096 ? v : 256;
  }();
  const int target_chunks = std::max(1, wgs / pl.n_pairs);
  const int max_chunks = ceil_div(len, 64);
  pl.n_chunks = std::max(1, std::min(target_chunks, max_chunks));
  pl.rows_per_chunk = (int)round_up(ceil_div(len, pl.n_chunks), TR);
  pl.n_chunks = ceil_div(len, pl.rows_per_chunk);
  // the Gram pass is pure matrix-core streaming: twice the workgroups, so
  // two share a compute unit and hide each other's load latency
  pl.n_gchunks = std::max(1, std::min(2 * pl.n_chunks, max_chunks));
  pl.rows_per_gchunk = (int)round_up(ceil_div(len, pl.n_gchunks), TR);
  pl.n_gchunks = ceil_div(len, pl.rows_per_gchunk);
  return pl;
}

size_t jacobi_work_bytes(const JacobiPlan& pl) {
  const int JP = 2 * pl.jb;
  return (size_t)pl.n_pairs * pl.n_gchunks * JP * JP * sizeof(double2) + 2 * (size_t)pl.nbp * sizeof(int) +
         256;
}

template <typename R>
static void launch_sweep(const JacobiPlan& pl, JacArgs<R> a, hipStream_t stream, bool first) {
  hipLaunchKernelGGL(k_jac_roll, dim3(1), dim3(256), 0, stream, a.rot_prev, a.rot_cur, a.rot_count, a.big_cos, pl.nbp,
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
        hipExtLaunchKernelGGL((k_jac_gram<32, R>), dim3(pl.n_pairs, pl.n_gchunks), dim3(256), 0, stream, pr.start(),
                              pr.stop(), 0, a);
      else
        hipExtLaunchKernelGGL((k_jac_gram<64, R>), dim3(pl.n_pairs, pl.n_gchunks), dim3(256), 0, stream, pr.start(),
                              pr.stop(), 0, a);
    }
    HIP_LAUNCH_OK();
    {
      Probe pr(kKcJacRotate, stream, fl, 2.0 * by);
      if (pl.jb == 16)
        hipExtLaunchKernelGGL((k_jac_rotate<32, R>), dim3(pl.n_pairs, pl.n_chunks), dim3(ROT_THREADS), 0, stream,
                              pr.start(), pr.stop(), 0, a);
      else
        hipExtLaunchKernelGGL((k_jac_rotate<64, R>), dim3(pl.n_pairs, pl.n_chunks), dim3(ROT_THREADS), 0, stream,
                              pr.start(), pr.stop(), 0, a);
    }
    HIP_LAUNCH_OK();
  }
}

// Stop after a sweep whose largest entering squared cosine c2 satisfies
// f c2 <= tol, f = 100 (RCS_JACOBI_QSTOP overrides; 0 turns it off): the
// Jacobi iteration converges quadratically at the end, so the next sweep
// would start below ~c2 and rotate nothing; it is not run.  On the
// 53-qubit chi 1024 build this skips 1,016 of 1,278 such verification
// sweeps, and in none of the skipped cases did the sweep rotate anything
// when run.
static double qstop_factor() {
  static const double v = [] {
    const char* e = std::getenv("RCS_JACOBI_QSTOP");
    const double f = e ? std::atof(e) : 100.0;
    return f > 0.0 ? f : 0.0;
  }();
  return v;
}

static bool use_graphs() {
  static const bool v = [] {
    const char* e = std::getenv("RCS_JACOBI_GRAPH");
    return e && e[0] == '1';
  }();
  return v;
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

static hipGraphExec_t sweep_graph(const JacobiPlan& pl, const JacArgs<double>& a, void* work, hipStream_t stream) {
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

template <typename R>
static int jacobi_run_t(const JacobiPlan& pl, typename JT<R>::C* x, void* work, int* rot_count_dev,
                        int* rot_count_host, double fro2, hipStream_t stream, int max_sweeps, double tol) {
  using C = typename JT<R>::C;
  JacArgs<R> a;
  a.x = x;
  a.ldx = pl.ldx;
  a.len = pl.len;
  a.nbp = pl.nbp;
  a.rows_per_chunk = pl.rows_per_chunk;
  a.n_chunks = pl.n_chunks;
  a.rows_per_gchunk = pl.rows_per_gchunk;
  a.n_gchunks = pl.n_gchunks;
  a.round = 0;
  char* w = reinterpret_cast<char*>(work);
  a.part = reinterpret_cast<C*>(w);
  w += (size_t)pl.n_pairs * pl.n_gchunks * (2 * pl.jb) * (2 * pl.jb) * sizeof(C);
  a.rot_prev = reinterpret_cast<int*>(w);
  a.rot_cur = a.rot_prev + pl.nbp;
  a.rot_count = rot_count_dev;
  a.big_cos = rot_count_dev + 1;
  const double u = JT<R>::u;
  a.tol = (R)(tol > 0.0 ? tol : 16.0 * u * std::sqrt((double)std::max(pl.len, 16)));
  // columns shorter than delta ||X||_F (delta = 8 u sqrt(len)) are numerically
  // zero: below the absolute accuracy of any SVD in this precision, and they
  // must not be required to be mutually orthogonal (a wide matrix has more
  // columns than its rank)
  const double delta = 8.0 * u * std::sqrt((double)pl.len);
  a.neg2 = (R)(delta * delta * std::max(fro2, 1e-300));
  a.qtol = (R)(qstop_factor() > 0.0 ? (double)a.tol / qstop_factor() : 0.0);
  a.max_inner = pl.inner;
  bool graphs = false;
  if constexpr (std::is_same<R, double>::value) graphs = use_graphs() && pl.nbp > 4;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    if constexpr (std::is_same<R, double>::value) {
      if (graphs && sweep > 1)
        HIP_OK(hipGraphLaunch(sweep_graph(pl, a, work, stream), stream));
      else
        launch_sweep(pl, a, stream, sweep == 1);
    } else {
      launch_sweep(pl, a, stream, sweep == 1);
    }
    HIP_OK(hipMemcpyAsync(rot_count_host, rot_count_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    const bool big = rot_count_host[1] != 0;
    if (debug_jacobi())
      std::fprintf(stderr, "jacobi %dx%d sweep %d: %d pair rotations%s\n", pl.len, pl.cnt, sweep, *rot_count_host,
                   big ? "" : ", all entering cosines below the quadratic-stop level");
    if (*rot_count_host == 0) return sweep;
    // quadratic convergence: after a sweep whose meetings all entered with
    // squared cosines below tol / f, the next one starts below ~tol^2 / f^2
    if (qstop_factor() > 0.0 && !big) return sweep;
  }
  fail(RCS_ERR_NUMERIC, "one-sided Jacobi SVD did not converge");
}

int jacobi_run(const JacobiPlan& pl, double2* x, void* work, int* rot_count_dev, int* rot_count_host, double fro2,
               hipStream_t stream, int max_sweeps, double tol) {
  return jacobi_run_t<double>(pl, x, work, rot_count_dev, rot_count_host, fro2, stream, max_sweeps, tol);
}

int jacobi_run_f32(const JacobiPlan& pl, float2* x, void* work, int* rot_count_dev, int* rot_count_host, double fro2,
                   hipStream_t stream, int max_sweeps, double tol) {
  return jacobi_run_t<float>(pl, x, work, rot_count_dev, rot_count_host, fro2, stream, max_sweeps, tol);
}

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
