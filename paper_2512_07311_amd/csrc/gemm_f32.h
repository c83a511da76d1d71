// Complex fp32 tile GEMM engine on CDNA matrix cores (v_mfma_f32_16x16x4f32).
//
// Same organisation as the fp64 engine: 256 threads, 64x64 complex output
// tile, wave w owns the 32x32 quadrant (w&1, w>>1), operands staged through
// LDS as fp32 real/imaginary planes (32 k-values per stage).  Loader functors
// return complex128 values, rounded to fp32 as they are staged.
// Output layout of the fp32 16x16x4 form: D[4 (l / 16) + r][l % 16].
#pragma once

#include "common.h"

namespace rcs {

constexpr int FT_M = 64, FT_N = 64, FT_K = 32;

struct SmemF32C {
  float ar[FT_K][FT_M];
  float ai[FT_K][FT_M];
  float br[FT_K][FT_N];
  float bi[FT_K][FT_N];
};

struct AccF32C {
  float4_t re[2][2];
  float4_t im[2][2];
};

__device__ inline void acc_zero(AccF32C& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      a.re[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      a.im[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    }
}

template <class F, bool KFAST>
struct LoadA32 {
  F f;
  int m0, M, K;
  __device__ inline void operator()(SmemF32C& s, int k0, int tid) const {
#pragma unroll
    for (int j = 0; j < (FT_M * FT_K) / 256; ++j) {
      const int e = tid + j * 256;
      int m, k;
      if (KFAST) {
        k = e % FT_K;
        m = e / FT_K;
      } else {
        m = e % FT_M;
        k = e / FT_M;
      }
      double2 v = make_double2(0.0, 0.0);
      if (m0 + m < M && k0 + k < K) v = f(m0 + m, k0 + k);
      s.ar[k][m] = (float)v.x;
      s.ai[k][m] = (float)v.y;
    }
  }
};

template <class F, bool NFAST>
struct LoadB32 {
  F f;
  int n0, K, N;
  __device__ inline void operator()(SmemF32C& s, int k0, int tid) const {
#pragma unroll
    for (int j = 0; j < (FT_N * FT_K) / 256; ++j) {
      const int e = tid + j * 256;
      int n, k;
      if (NFAST) {
        n = e % FT_N;
        k = e / FT_N;
      } else {
        k = e % FT_K;
        n = e / FT_K;
      }
      double2 v = make_double2(0.0, 0.0);
      if (k0 + k < K && n0 + n < N) v = f(k0 + k, n0 + n);
      s.br[k][n] = (float)v.x;
      s.bi[k][n] = (float)v.y;
    }
  }
};

template <class LA, class LB>
__device__ inline void cgemm32_mainloop(const LA& la, const LB& lb, int K, SmemF32C& s, AccF32C& acc) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += FT_K) {
    la(s, k0, tid);
    lb(s, k0, tid);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < FT_K; kk += 4) {
      const int k = kk + lk;
      float ar[2], ai[2], nai[2], br[2], bi[2];
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
          acc.re[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], br[nt], acc.re[mt][nt], 0, 0, 0);
          acc.re[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[mt], bi[nt], acc.re[mt][nt], 0, 0, 0);
          acc.im[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], bi[nt], acc.im[mt][nt], 0, 0, 0);
          acc.im[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mt], br[nt], acc.im[mt][nt], 0, 0, 0);
        }
    }
    __syncthreads();
  }
}

template <class G>
__device__ inline void acc32_foreach(const AccF32C& acc, G g) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm + mt * 16 + 4 * (lane >> 4) + r;
        const int col = wn + nt * 16 + (lane & 15);
        g(row, col, acc.re[mt][nt][r], acc.im[mt][nt][r]);
      }
}

}  // namespace rcs
