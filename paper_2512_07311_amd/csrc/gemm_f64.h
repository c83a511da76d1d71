// Complex fp64 tile GEMM engine on CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup of 256 threads (4 wave64) computes a 64x64 complex output
// tile; wave w owns the 32x32 quadrant (w&1, w>>1) as 2x2 MFMA blocks with
// separate real and imaginary accumulators.  Operands are staged through LDS
// in split real/imaginary planes, 16 k-values per stage, so that each MFMA
// fragment read is 16 consecutive doubles.  A complex product is four real
// MFMAs:  Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br.
//
// MFMA f64 16x16x4 operand layout (lane l of 64):
//   A (16x4):  A[l % 16][l / 16]      B (4x16): B[l / 16][l % 16]
//   D (16x16): D[(l / 16) + 4 r][l % 16], r = 0..3 in the four result regs
//   (measured on gfx950; the fp32/bf16 16x16 forms use row 4 (l / 16) + r).
//
// Operands come from loader functors so that each caller can gather rows or
// columns in its own way (row-indirect shot vectors, pairs of column blocks,
// conjugated transposes) while keeping global loads coalesced along the
// operand's unit-stride dimension.
#pragma once

#include "common.h"

namespace rcs {

constexpr int GT_M = 64, GT_N = 64, GT_K = 16;
constexpr int GT_THREADS = 256;

struct SmemC64 {
  double ar[GT_K][GT_M];
  double ai[GT_K][GT_M];
  double br[GT_K][GT_N];
  double bi[GT_K][GT_N];
};

struct AccC64 {
  double4_t re[2][2];
  double4_t im[2][2];
};

__device__ inline void acc_zero(AccC64& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      a.re[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
      a.im[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
}

// Multiply the staged 64x16 A tile by the 16x64 B tile into the wave's
// quadrant.
__device__ inline void mma_stage(const SmemC64& s, AccC64& acc, int wm, int wn, int lane) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < GT_K; kk += 4) {
    const int k = kk + lk;
    double ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      ar[t] = s.ar[k][wm + t * 16 + lr];
      ai[t] = s.ai[k][wm + t * 16 + lr];
      nai[t] = -ai[t];
      br[t] = s.br[k][wn + t * 16 + lr];
      bi[t] = s.bi[k][wn + t * 16 + lr];
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        acc.re[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[mt], br[nt], acc.re[mt][nt], 0, 0, 0);
        acc.re[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[mt], bi[nt], acc.re[mt][nt], 0, 0, 0);
        acc.im[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[mt], bi[nt], acc.im[mt][nt], 0, 0, 0);
        acc.im[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[mt], br[nt], acc.im[mt][nt], 0, 0, 0);
      }
  }
}

// Output row (within a 16x16 block) of result register r in lane `lane`.
__device__ inline int f64_row(int lane, int r) { return (lane >> 4) + 4 * r; }

// Generic A loader: element functor f(m, k) -> double2 for rows m of the
// tile (absolute indices), with M x K bounds.  KFAST selects which index
// consecutive threads walk (the operand's unit-stride dimension).  fetch()
// reads a stage into registers, commit() writes them to LDS, so that the
// main loop can have the next stage's loads in flight during the current
// stage's matrix-core work.
template <class F, bool KFAST>
struct LoadA {
  static constexpr int PER = (GT_M * GT_K) / GT_THREADS;
  F f;
  int m0, M, K;
  __device__ inline void index(int j, int tid, int& m, int& k) const {
    const int e = tid + j * GT_THREADS;
    if (KFAST) {
      k = e % GT_K;
      m = e / GT_K;
    } else {
      m = e % GT_M;
      k = e / GT_M;
    }
  }
  __device__ inline void fetch(double2 (&r)[PER], int k0, int tid) const {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int m, k;
      index(j, tid, m, k);
      r[j] = (m0 + m < M && k0 + k < K) ? f(m0 + m, k0 + k) : make_double2(0.0, 0.0);
    }
  }
  __device__ inline void commit(SmemC64& s, const double2 (&r)[PER], int tid) const {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int m, k;
      index(j, tid, m, k);
      s.ar[k][m] = r[j].x;
      s.ai[k][m] = r[j].y;
    }
  }
};

// Generic B loader: f(k, n) -> double2, K x N bounds; NFAST: n is the
// unit-stride index.
template <class F, bool NFAST>
struct LoadB {
  static constexpr int PER = (GT_N * GT_K) / GT_THREADS;
  F f;
  int n0, K, N;
  __device__ inline void index(int j, int tid, int& k, int& n) const {
    const int e = tid + j * GT_THREADS;
    if (NFAST) {
      n = e % GT_N;
      k = e / GT_N;
    } else {
      k = e % GT_K;
      n = e / GT_K;
    }
  }
  __device__ inline void fetch(double2 (&r)[PER], int k0, int tid) const {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int k, n;
      index(j, tid, k, n);
      r[j] = (k0 + k < K && n0 + n < N) ? f(k0 + k, n0 + n) : make_double2(0.0, 0.0);
    }
  }
  __device__ inline void commit(SmemC64& s, const double2 (&r)[PER], int tid) const {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      int k, n;
      index(j, tid, k, n);
      s.br[k][n] = r[j].x;
      s.bi[k][n] = r[j].y;
    }
  }
};

// K loop: stage k0 goes from registers to LDS, then the loads of stage
// k0 + 16 are issued before the matrix cores work on stage k0, so global
// latency overlaps the MFMAs (one LDS buffer, one register stage).
template <class LA, class LB>
__device__ inline void cgemm_mainloop(const LA& la, const LB& lb, int K, SmemC64& s, AccC64& acc) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  double2 ra[LA::PER], rb[LB::PER];
  if (K > 0) {
    la.fetch(ra, 0, tid);
    lb.fetch(rb, 0, tid);
  }
  for (int k0 = 0; k0 < K; k0 += GT_K) {
    la.commit(s, ra, tid);
    lb.commit(s, rb, tid);
    __syncthreads();
    if (k0 + GT_K < K) {
      la.fetch(ra, k0 + GT_K, tid);
      lb.fetch(rb, k0 + GT_K, tid);
    }
    mma_stage(s, acc, wm, wn, lane);
    __syncthreads();
  }
}

// Visit each output element held by this thread: g(row_in_tile, col_in_tile,
// re, im).
template <class G>
__device__ inline void acc_foreach(const AccC64& acc, G g) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = wm + mt * 16 + f64_row(lane, r);
        int col = wn + nt * 16 + (lane & 15);
        g(row, col, acc.re[mt][nt][r], acc.im[mt][nt][r]);
      }
}

}  // namespace rcs
