// Rank-prediction network and its training kernels (fp32).
//
// Network: Linear(66,128) - ReLU - Linear(128,128) - ReLU - Linear(128,32),
// packed weights W1[128][66], b1[128], W2[128][128], b2[128], W3[32][128],
// b3[32].  Loss: mean over batch and outputs of (out - y)^2.  Every
// reduction has a fixed order (one thread per output element, sequential over
// the batch or the fan-in), so forward, backward and Adam are deterministic.
//
// Features (66): 64-bin histogram of log10(s^2 / sum s^2) of a bond's kept
// singular values (0.25-decade bins over [-16, 0), clamped at both ends,
// normalised to sum 1), then bond / (n - 2) and cycle / n_cycles.
#include "state.h"

namespace rcs {

constexpr int NI = 66, NH = 128, NO = 32;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH, N_PARAMS = OFF_B3 + NO;
static_assert(N_PARAMS == RCS_MLP_PARAMS, "parameter count");

// -------------------------------------------------------------- features
__global__ void k_spec_features(const double* s, int k, double bond_f, double cycle_f, float* feat) {
  __shared__ double red[256];
  __shared__ int hist[64];
  const int tid = threadIdx.x;
  if (tid < 64) hist[tid] = 0;
  double acc = 0.0;
  for (int i = tid; i < k; i += 256) acc += s[i] * s[i];
  red[tid] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double tot = red[0];
  for (int i = tid; i < k; i += 256) {
    const double v = s[i] * s[i];
    int b = 0;
    if (v > 0.0 && tot > 0.0) {
      const double x = log10(v / tot);
      const double fb = floor((x + 16.0) / 0.25);
      b = fb < 0.0 ? 0 : (fb > 63.0 ? 63 : (int)fb);
    }
    atomicAdd(&hist[b], 1);
  }
  __syncthreads();
  if (tid < 64) feat[tid] = k > 0 ? (float)((double)hist[tid] / (double)k) : 0.0f;
  if (tid == 64) feat[64] = (float)bond_f;
  if (tid == 65) feat[65] = (float)cycle_f;
}

void spectrum_features(const double* s_dev, int k, int bond, int n_sites, int cycle, int n_cycles,
                       float* feat_dev, hipStream_t st) {
  const double bf = (double)bond / (double)std::max(n_sites - 2, 1);
  const double cf = (double)cycle / (double)std::max(n_cycles, 1);
  hipLaunchKernelGGL(k_spec_features, dim3(1), dim3(256), 0, st, s_dev, k, bf, cf, feat_dev);
  HIP_LAUNCH_OK();
}

// Training targets (32): y_j = log10(max(tail(ceil(m j/32)) / w, 1e-20)),
// j = 1..32, tail(k) = sum_{r>=k} s_r^2 accumulated from the smallest upward
// with values s^2 <= 1e-24 w counted as zero, w = sum s^2.
__global__ void k_spec_targets(const double* s, int m, float* y) {
  if (threadIdx.x != 0) return;
  double w = 0.0;
  for (int i = m - 1; i >= 0; --i) w += s[i] * s[i];
  const double floor_ = 1e-24 * w;
  double tail = 0.0;
  int next = NO;   // fill targets from j = 32 downward while walking k down
  for (int kk = m; kk >= 0; --kk) {
    // tail == tail(kk)
    while (next >= 1) {
      int kj = (int)ceil((double)next / NO * m);
      if (kj > m) kj = m;
      if (kj != kk) break;
      const double v = w > 0.0 ? tail / w : 0.0;
      y[next - 1] = (float)log10(fmax(v, 1e-20));
      --next;
    }
    if (kk == 0) break;
    const double v2 = s[kk - 1] * s[kk - 1];
    tail += v2 <= floor_ ? 0.0 : v2;
  }
}

void spectrum_targets(const double* s_dev, int m, float* y_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_spec_targets, dim3(1), dim3(64), 0, st, s_dev, m, y_dev);
  HIP_LAUNCH_OK();
}

// ---------------------------------------------------------------- forward
// Per sample: one block of 128 threads; activations stay in LDS.  When
// `act` is non-null the pre-activations z1, z2 and activations h1, h2 are
// stored for the backward pass ([batch][4][128]).
__global__ __launch_bounds__(128) void k_mlp_fwd(const float* w, const float* x, int batch, float* out,
                                                 float* act) {
  __shared__ float xs[NI], h1[NH], h2[NH];
  const int b = blockIdx.x, t = threadIdx.x;
  if (b >= batch) return;
  if (t < NI) xs[t] = x[(int64_t)b * NI + t];
  __syncthreads();
  {
    float z = w[OFF_B1 + t];
    const float* wr = w + OFF_W1 + t * NI;
    for (int i = 0; i < NI; ++i) z += wr[i] * xs[i];
    h1[t] = z > 0.f ? z : 0.f;
    if (act) {
      act[((int64_t)b * 4 + 0) * NH + t] = z;
      act[((int64_t)b * 4 + 1) * NH + t] = h1[t];
    }
  }
  __syncthreads();
  {
    float z = w[OFF_B2 + t];
    const float* wr = w + OFF_W2 + t * NH;
    for (int i = 0; i < NH; ++i) z += wr[i] * h1[i];
    h2[t] = z > 0.f ? z : 0.f;
    if (act) {
      act[((int64_t)b * 4 + 2) * NH + t] = z;
      act[((int64_t)b * 4 + 3) * NH + t] = h2[t];
    }
  }
  __syncthreads();
  if (t < NO) {
    float z = w[OFF_B3 + t];
    const float* wr = w + OFF_W3 + t * NH;
    for (int i = 0; i < NH; ++i) z += wr[i] * h2[i];
    out[(int64_t)b * NO + t] = z;
  }
}

// --------------------------------------------------------------- backward
// Per-sample deltas: dout = 2 (out - y) / (batch * 32); dz2 = (dout W3) .
// [z2 > 0]; dz1 = (dz2 W2) . [z1 > 0].  Stored as [batch][3][128] (dout
// in the first 32 of slot 0, dz2 in slot 1, dz1 in slot 2).
__global__ __launch_bounds__(128) void k_mlp_delta(const float* w, const float* out, const float* y,
                                                   const float* act, int batch, float* dl) {
  __shared__ float dout[NO], dz2[NH];
  const int b = blockIdx.x, t = threadIdx.x;
  if (b >= batch) return;
  const float scale = 2.0f / ((float)batch * (float)NO);
  if (t < NO) {
    dout[t] = scale * (out[(int64_t)b * NO + t] - y[(int64_t)b * NO + t]);
    dl[((int64_t)b * 3 + 0) * NH + t] = dout[t];
  }
  __syncthreads();
  {
    float d = 0.f;
    for (int o = 0; o < NO; ++o) d += dout[o] * w[OFF_W3 + o * NH + t];
    const float z2 = act[((int64_t)b * 4 + 2) * NH + t];
    dz2[t] = z2 > 0.f ? d : 0.f;
    dl[((int64_t)b * 3 + 1) * NH + t] = dz2[t];
  }
  __syncthreads();
  {
    float d = 0.f;
    for (int o = 0; o < NH; ++o) d += dz2[o] * w[OFF_W2 + o * NH + t];
    const float z1 = act[((int64_t)b * 4 + 0) * NH + t];
    dl[((int64_t)b * 3 + 2) * NH + t] = z1 > 0.f ? d : 0.f;
  }
}

// Weight gradients: one thread per parameter, sequential sum over the batch.
__global__ void k_mlp_wgrad(const float* x, const float* act, const float* dl, int batch, float* g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N_PARAMS) return;
  float acc = 0.f;
  if (p < OFF_B1) {  // W1[o][i] = sum_b dz1[b][o] x[b][i]
    const int o = p / NI, i = p % NI;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 2) * NH + o] * x[(int64_t)b * NI + i];
  } else if (p < OFF_W2) {
    const int o = p - OFF_B1;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 2) * NH + o];
  } else if (p < OFF_B2) {  // W2[o][i] = sum_b dz2[b][o] h1[b][i]
    const int q = p - OFF_W2, o = q / NH, i = q % NH;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 1) * NH + o] * act[((int64_t)b * 4 + 1) * NH + i];
  } else if (p < OFF_W3) {
    const int o = p - OFF_B2;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 1) * NH + o];
  } else if (p < OFF_B3) {  // W3[o][i] = sum_b dout[b][o] h2[b][i]
    const int q = p - OFF_W3, o = q / NH, i = q % NH;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 0) * NH + o] * act[((int64_t)b * 4 + 3) * NH + i];
  } else {
    const int o = p - OFF_B3;
    for (int b = 0; b < batch; ++b) acc += dl[((int64_t)b * 3 + 0) * NH + o];
  }
  g[p] = acc;
}

// loss = mean (out - y)^2 over batch * 32 values, fixed-order tree.
__global__ void k_mlp_loss(const float* out, const float* y, int n, float* loss) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float d = out[i] - y[i];
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

// Adam (Kingma & Ba 2015) with bias correction.
__global__ void k_adam(float* w, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void mlp_forward(const float* w, const float* x, int batch, float* out, float* act, hipStream_t s) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(batch), dim3(128), 0, s, w, x, batch, out, act);
  HIP_LAUNCH_OK();
}

}  // namespace rcs

extern "C" {

#define RCS_API_BEGIN try {
#define RCS_API_END                  \
  }                                  \
  catch (const rcs::Error& e) {      \
    rcs::set_last_error(e.what());   \
    return e.status;                 \
  }                                  \
  catch (const std::exception& e) {  \
    rcs::set_last_error(e.what());   \
    return RCS_ERR_DEVICE;           \
  }                                  \
  return RCS_OK;

rcs_status rcs_spectrum_features(const double* s_dev, int32_t k, int32_t bond, int32_t n_sites,
                                 int32_t cycle, int32_t n_cycles, float* feat_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(feat_dev && (s_dev || k == 0) && k >= 0, "bad arguments");
  rcs::spectrum_features(s_dev, k, bond, n_sites, cycle, n_cycles, feat_dev, rcs::as_stream(stream));
  RCS_API_END
}

rcs_status rcs_spectrum_targets(const double* s_dev, int32_t m, float* y_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(s_dev && y_dev && m >= 1, "bad arguments");
  rcs::spectrum_targets(s_dev, m, y_dev, rcs::as_stream(stream));
  RCS_API_END
}

rcs_status rcs_mlp_forward(const float* w_dev, const float* x_dev, int32_t batch, float* out_dev,
                           void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(w_dev && x_dev && out_dev && batch >= 0, "bad arguments");
  rcs::mlp_forward(w_dev, x_dev, batch, out_dev, nullptr, rcs::as_stream(stream));
  RCS_API_END
}

rcs_status rcs_mlp_backward(const float* w_dev, const float* x_dev, const float* y_dev, int32_t batch,
                            float* grad_dev, float* loss_dev, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(w_dev && x_dev && y_dev && grad_dev && batch >= 1, "bad arguments");
  hipStream_t s = rcs::as_stream(stream);
  rcs::DevBuf out, act, dl;
  out.ensure((size_t)batch * rcs::NO * sizeof(float));
  act.ensure((size_t)batch * 4 * rcs::NH * sizeof(float));
  dl.ensure((size_t)batch * 3 * rcs::NH * sizeof(float));
  rcs::mlp_forward(w_dev, x_dev, batch, out.as<float>(), act.as<float>(), s);
  hipLaunchKernelGGL(rcs::k_mlp_delta, dim3(batch), dim3(128), 0, s, w_dev, out.as<float>(), y_dev,
                     act.as<float>(), batch, dl.as<float>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(rcs::k_mlp_wgrad, dim3(rcs::ceil_div(rcs::N_PARAMS, 256)), dim3(256), 0, s, x_dev,
                     act.as<float>(), dl.as<float>(), batch, grad_dev);
  HIP_LAUNCH_OK();
  if (loss_dev) {
    hipLaunchKernelGGL(rcs::k_mlp_loss, dim3(1), dim3(256), 0, s, out.as<float>(), y_dev, batch * rcs::NO,
                       loss_dev);
    HIP_LAUNCH_OK();
  }
  HIP_OK(hipStreamSynchronize(s));
  RCS_API_END
}

rcs_status rcs_mlp_adam(float* w_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t count,
                        int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(w_dev && grad_dev && m_dev && v_dev && count >= 0 && step >= 1, "bad arguments");
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  if (count > 0) {
    hipLaunchKernelGGL(rcs::k_adam, dim3(rcs::ceil_div(count, 256)), dim3(256), 0, rcs::as_stream(stream), w_dev,
                       grad_dev, m_dev, v_dev, count, lr, beta1, beta2, eps, c1, c2);
    HIP_LAUNCH_OK();
  }
  RCS_API_END
}

}  // extern "C"
