// Two-site contraction T^{s1 s2} = A_i^{s1} A_{i+1}^{s2} in reduced precision.
//
//  complex64 : operands rounded to fp32, v_mfma_f32_16x16x4f32, fp32 sums;
//  split-bf16: each fp32 operand x = hi + lo with hi = bf16(x), lo =
//              bf16(x - hi) (round to nearest even); every real product is
//              hi*hi' + hi*lo' + lo*hi' on v_mfma_f32_16x16x32_bf16 with fp32
//              accumulation (Henry, Tang, Heinecke, ARITH 2019), complex
//              products in the four-real-product form.
// Site tensors stay complex128 in HBM; operands are converted while staged
// into LDS (fp32 planes), the bf16 split happens in registers.  The result
// is written as complex128 for the fp64 SVD.
//
// MFMA layouts (lane l): f32 16x16x4: A[l%16][l/16], B[l/16][l%16];
// bf16 16x16x32: A[l%16][8(l/16)+j], B[8(l/16)+j][l%16], j = 0..7;
// both: D[4(l/16)+r][l%16].
#include <hip/hip_ext.h>

#include "build.h"
#include "gemm_f64.h"

namespace rcs {

constexpr int CT_M = 64, CT_N = 64, CT_K = 32;

struct SmemF32 {
  float ar[CT_M][CT_K + 4];  // A[m][k]
  float ai[CT_M][CT_K + 4];
  float br[CT_N][CT_K + 4];  // B transposed: B[k][n] at [n][k]
  float bi[CT_N][CT_K + 4];
};

__device__ inline void stage_f32(SmemF32& s, const double2* a, const double2* b, int dl, int dm, int dr,
                                 int m0, int n0, int k0, int tid) {
  // A: 64 x 32, k contiguous in HBM (row-major dl x dm)
  for (int e = tid; e < CT_M * CT_K; e += 256) {
    const int k = e % CT_K, m = e / CT_K;
    double2 v = make_double2(0.0, 0.0);
    if (m0 + m < dl && k0 + k < dm) v = a[(int64_t)(m0 + m) * dm + k0 + k];
    s.ar[m][k] = (float)v.x;
    s.ai[m][k] = (float)v.y;
  }
  // B: 32 x 64, n contiguous in HBM (row-major dm x dr)
  for (int e = tid; e < CT_K * CT_N; e += 256) {
    const int n = e % CT_N, k = e / CT_N;
    double2 v = make_double2(0.0, 0.0);
    if (k0 + k < dm && n0 + n < dr) v = b[(int64_t)(k0 + k) * dr + n0 + n];
    s.br[n][k] = (float)v.x;
    s.bi[n][k] = (float)v.y;
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_two_site_lowp(const double2* A, const double2* B, double2* T, int dl,
                                                      int dm, int dr) {
  __shared__ SmemF32 sm;
  const int q = blockIdx.z, s1 = q >> 1, s2 = q & 1;
  const int m0 = blockIdx.y * CT_M, n0 = blockIdx.x * CT_N;
  const double2* a = A + (int64_t)s1 * dl * dm;
  const double2* b = B + (int64_t)s2 * dm * dr;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  float4_t cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = float4_t{0, 0, 0, 0};
      ci[i][j] = float4_t{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < dm; k0 += CT_K) {
    stage_f32(sm, a, b, dl, dm, dr, m0, n0, k0, tid);
    __syncthreads();
    if (PREC == RCS_PREC_C64) {
#pragma unroll
      for (int kk = 0; kk < CT_K; kk += 4) {
        const int k = kk + (lane >> 4);
        float ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          ar[t] = sm.ar[wm + t * 16 + (lane & 15)][k];
          ai[t] = sm.ai[wm + t * 16 + (lane & 15)][k];
          nai[t] = -ai[t];
          br[t] = sm.br[wn + t * 16 + (lane & 15)][k];
          bi[t] = sm.bi[wn + t * 16 + (lane & 15)][k];
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], br[nt], cr[mt][nt], 0, 0, 0);
            cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[mt], bi[nt], cr[mt][nt], 0, 0, 0);
            ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], bi[nt], ci[mt][nt], 0, 0, 0);
            ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mt], br[nt], ci[mt][nt], 0, 0, 0);
          }
      }
    } else {
      // one 16x16x32 step covers the whole 32-wide k stage
      const int kb = 8 * (lane >> 4);
      bf16x8_t arh[2], arl[2], aih[2], ail[2], naih[2], nail[2];
      bf16x8_t brh[2], brl[2], bih[2], bil[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int mr = wm + t * 16 + (lane & 15), nr = wn + t * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float x = sm.ar[mr][kb + j];
          __bf16 h = (__bf16)x;
          arh[t][j] = h;
          arl[t][j] = (__bf16)(x - (float)h);
          x = sm.ai[mr][kb + j];
          h = (__bf16)x;
          aih[t][j] = h;
          ail[t][j] = (__bf16)(x - (float)h);
          naih[t][j] = (__bf16)(-(float)aih[t][j]);
          nail[t][j] = (__bf16)(-(float)ail[t][j]);
          x = sm.br[nr][kb + j];
          h = (__bf16)x;
          brh[t][j] = h;
          brl[t][j] = (__bf16)(x - (float)h);
          x = sm.bi[nr][kb + j];
          h = (__bf16)x;
          bih[t][j] = h;
          bil[t][j] = (__bf16)(x - (float)h);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          // Re += Ar Br - Ai Bi
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[mt], brh[nt], cr[mt][nt], 0, 0, 0);
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[mt], brl[nt], cr[mt][nt], 0, 0, 0);
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[mt], brh[nt], cr[mt][nt], 0, 0, 0);
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih[mt], bih[nt], cr[mt][nt], 0, 0, 0);
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(naih[mt], bil[nt], cr[mt][nt], 0, 0, 0);
          cr[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nail[mt], bih[nt], cr[mt][nt], 0, 0, 0);
          // Im += Ar Bi + Ai Br
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[mt], bih[nt], ci[mt][nt], 0, 0, 0);
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[mt], bil[nt], ci[mt][nt], 0, 0, 0);
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[mt], bih[nt], ci[mt][nt], 0, 0, 0);
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[mt], brh[nt], ci[mt][nt], 0, 0, 0);
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[mt], brl[nt], ci[mt][nt], 0, 0, 0);
          ci[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail[mt], brh[nt], ci[mt][nt], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  double2* t = T + (int64_t)q * dl * dr;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + mt * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + nt * 16 + (lane & 15);
        if (m < dl && n < dr) t[(int64_t)m * dr + n] = make_double2((double)cr[mt][nt][r], (double)ci[mt][nt][r]);
      }
}

void contract_two_site_lowp(const double2* A, const double2* B, double2* T, int dl, int dm, int dr,
                            int precision, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  dim3 grid(ceil_div(dr, CT_N), ceil_div(dl, CT_M), 4);
  if (precision == RCS_PREC_C64)
    hipExtLaunchKernelGGL(k_two_site_lowp<RCS_PREC_C64>, grid, dim3(256), 0, s, start, stop, 0, A, B, T, dl, dm, dr);
  else
    hipExtLaunchKernelGGL(k_two_site_lowp<RCS_PREC_SPLIT_BF16>, grid, dim3(256), 0, s, start, stop, 0, A, B, T, dl,
                          dm, dr);
  HIP_LAUNCH_OK();
}

}  // namespace rcs
