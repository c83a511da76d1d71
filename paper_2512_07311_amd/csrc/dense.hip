// Dense state vector of the random circuit on one GPU, the exact reference
// for true-fidelity XEB (Section 5.1 scores samples against exact output
// probabilities).  psi has 2^n complex128 amplitudes, index i = sum_q b_q 2^q
// (bit q = qubit q, the bitstring convention); 34 qubits take 256 GiB.
//
// Each layer is applied in passes over "windows" of WIN consecutive qubit
// bits: a workgroup stages the 2^(LOW + WIN) amplitudes whose indices vary
// in bits [0, LOW) and [w, w + WIN) (all other bits fixed) in LDS, applies
// every gate of the layer acting inside the window there, and writes them
// back.  Bits [0, LOW) are always part of the tile, so each global access
// moves 2^LOW consecutive amplitudes (256 B).  A single-qubit layer on n
// qubits is ceil(n / WIN) passes; a two-qubit layer groups its couplers into
// windows that contain both qubits (couplers span at most the grid width,
// which must stay below WIN).  Every pass reads and writes psi once, so a
// layer costs a few times 2 x 16 x 2^n bytes of HBM traffic.
#include <algorithm>
#include <vector>

#include "circuit.h"
#include "common.h"

namespace rcs {

constexpr int DW_WIN = 8;      // window bits
constexpr int DW_LOW = 4;      // always-staged low bits
constexpr int DW_THREADS = 256;
constexpr int DW_MAXOPS = 8;   // gates per pass: a window holds WIN single-qubit gates or WIN / 2 couplers

struct DenseOp {
  int kind;      // 1: single-qubit (g[0..3]); 2: two-qubit (g[0..15], index 2 s_a + s_b)
  int ta, tb;    // tile bits of qubit a (and b)
  double2 g[16];
};

struct DensePass {
  int w, win, low;   // window base bit, window width, staged low bits
  int nops;
  DenseOp ops[DW_MAXOPS];
};

__global__ void k_dense_init(double2* psi, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    psi[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
}

__device__ inline double2 cfma(double2 a, double2 b, double2 c) {   // c + a b
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}

// One workgroup per combination of the bits outside the tile.
__global__ __launch_bounds__(DW_THREADS) void k_dense_pass(double2* psi, int n, DensePass P) {
  extern __shared__ double2 tile[];
  const int tb = P.low + P.win;              // tile bits
  const int tsz = 1 << tb;
  const int mid_bits = P.w - P.low;          // bits [low, w) outside the tile
  const int64_t g = blockIdx.x;
  const int64_t mid = g & ((int64_t(1) << mid_bits) - 1);
  const int64_t hi = g >> mid_bits;
  const int64_t base = (mid << P.low) | (hi << (P.w + P.win));
  auto gidx = [&](int t) -> int64_t {
    const int64_t lo = t & ((1 << P.low) - 1);
    const int64_t wv = t >> P.low;
    return base | lo | (wv << P.w);
  };
  for (int t = threadIdx.x; t < tsz; t += DW_THREADS) tile[t] = psi[gidx(t)];
  __syncthreads();
  for (int o = 0; o < P.nops; ++o) {
    const DenseOp& op = P.ops[o];
    if (op.kind == 1) {
      const int b = op.ta, m = 1 << b;
      for (int p = threadIdx.x; p < (tsz >> 1); p += DW_THREADS) {
        const int t0 = ((p >> b) << (b + 1)) | (p & (m - 1));
        const int t1 = t0 | m;
        const double2 x0 = tile[t0], x1 = tile[t1];
        double2 y0 = make_double2(0.0, 0.0), y1 = make_double2(0.0, 0.0);
        y0 = cfma(op.g[0], x0, y0);
        y0 = cfma(op.g[1], x1, y0);
        y1 = cfma(op.g[2], x0, y1);
        y1 = cfma(op.g[3], x1, y1);
        tile[t0] = y0;
        tile[t1] = y1;
      }
    } else {
      const int ba = op.ta, bb = op.tb;
      const int lo = min(ba, bb), hb = max(ba, bb);
      for (int p = threadIdx.x; p < (tsz >> 2); p += DW_THREADS) {
        // insert zero bits at lo and hb
        int t = ((p >> lo) << (lo + 1)) | (p & ((1 << lo) - 1));
        t = ((t >> hb) << (hb + 1)) | (t & ((1 << hb) - 1));
        int idx[4];
        double2 x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {      // s = 2 s_a + s_b
          idx[s] = t | (((s >> 1) & 1) << ba) | ((s & 1) << bb);
          x[s] = tile[idx[s]];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double2 y = make_double2(0.0, 0.0);
#pragma unroll
          for (int s = 0; s < 4; ++s) y = cfma(op.g[r * 4 + s], x[s], y);
          tile[idx[r]] = y;
        }
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < tsz; t += DW_THREADS) psi[gidx(t)] = tile[t];
}

static void launch_pass(double2* psi, int n, DensePass& P, hipStream_t s) {
  if (P.nops == 0) return;
  const int tb = P.low + P.win;
  const int64_t groups = int64_t(1) << (n - tb);
  RCS_REQUIRE(groups <= (int64_t(1) << 31) - 1, "state vector too large for the grid");
  hipLaunchKernelGGL(k_dense_pass, dim3((unsigned)groups), dim3(DW_THREADS), (size_t(1) << tb) * sizeof(double2), s,
                     psi, n, P);
  HIP_LAUNCH_OK();
}

// Window [w, w + win) and the staged low bits [0, low) for n qubits.
static DensePass make_pass(int n, int w) {
  DensePass P{};
  P.win = std::min(DW_WIN, n);
  P.w = std::min(w, n - P.win);
  P.low = std::min(DW_LOW, P.w);
  P.nops = 0;
  return P;
}

static void add_1q(DensePass& P, int q, const std::array<cplx, 4>& u) {
  RCS_REQUIRE(P.nops < DW_MAXOPS, "too many gates in one dense pass");
  DenseOp& op = P.ops[P.nops++];
  op.kind = 1;
  op.ta = P.low + (q - P.w);
  op.tb = 0;
  for (int e = 0; e < 4; ++e) op.g[e] = make_double2(u[e].real(), u[e].imag());
}

static void add_2q(DensePass& P, int qa, int qb, const std::array<cplx, 16>& G) {
  RCS_REQUIRE(P.nops < DW_MAXOPS, "too many gates in one dense pass");
  DenseOp& op = P.ops[P.nops++];
  op.kind = 2;
  op.ta = P.low + (qa - P.w);
  op.tb = P.low + (qb - P.w);
  for (int e = 0; e < 16; ++e) op.g[e] = make_double2(G[e].real(), G[e].imag());
}

void dense_simulate(const rcs_circuit_s& c, double2* psi, hipStream_t s) {
  const int n = c.n;
  const int64_t len = int64_t(1) << n;
  hipLaunchKernelGGL(k_dense_init, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 1 << 20)), dim3(256), 0, s,
                     psi, len);
  HIP_LAUNCH_OK();
  auto layer_1q = [&](const std::vector<int>& g) {
    for (int w0 = 0; w0 < n; w0 += DW_WIN) {
      DensePass P = make_pass(n, w0);
      for (int q = std::max(w0, P.w); q < std::min(n, w0 + DW_WIN); ++q) add_1q(P, q, one_qubit_gate(g[q]));
      // qubits the clamped window covers but an earlier pass already did
      // are not repeated (the loop starts at w0)
      launch_pass(psi, n, P, s);
    }
  };
  const size_t n1 = c.layers_1q.size();
  for (int t = 0; t < c.n_cycles; ++t) {
    layer_1q(c.layers_1q[t]);
    std::vector<std::pair<int, int>> cp;
    for (auto& e : c.layers_2q[t]) cp.emplace_back(std::min(e.first, e.second), std::max(e.first, e.second));
    std::sort(cp.begin(), cp.end());
    size_t i = 0;
    std::vector<char> done(cp.size(), 0);
    while (i < cp.size()) {
      if (done[i]) {
        ++i;
        continue;
      }
      RCS_REQUIRE(cp[i].second - cp[i].first < std::min(DW_WIN, n), "coupler wider than the dense window");
      DensePass P = make_pass(n, cp[i].first);
      for (size_t j = i; j < cp.size(); ++j)
        if (!done[j] && cp[j].first >= P.w && cp[j].second < P.w + P.win && P.nops < DW_MAXOPS) {
          add_2q(P, cp[j].first, cp[j].second, c.fsim);
          done[j] = 1;
        }
      launch_pass(psi, n, P, s);
    }
  }
  if (c.final_layer && n1 > (size_t)c.n_cycles) layer_1q(c.layers_1q[c.n_cycles]);
}

// out[i] = psi[bits[i]] (mode 0: amplitude, complex) or |psi[bits[i]]|^2
// (mode 1: probability, real).
__global__ void k_dense_gather(const double2* psi, int n, const uint64_t* bits, uint64_t m, int mode, void* out) {
  const uint64_t mask = n == 64 ? ~0ull : ((1ull << n) - 1);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
    const double2 a = psi[bits[i] & mask];
    if (mode == 0)
      static_cast<double2*>(out)[i] = a;
    else
      static_cast<double*>(out)[i] = a.x * a.x + a.y * a.y;
  }
}

void dense_gather(const double2* psi, int n, const uint64_t* bits, uint64_t m, int mode, void* out, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_dense_gather, dim3((unsigned)std::min<uint64_t>((m + 255) / 256, 65535)), dim3(256), 0, s, psi,
                     n, bits, m, mode, out);
  HIP_LAUNCH_OK();
}

}  // namespace rcs

extern "C" {

rcs_status rcs_dense_simulate(rcs_circuit c, double* psi_dev, int64_t n_amps, void* stream) {
  try {
    RCS_REQUIRE(c && psi_dev, "null argument");
    RCS_REQUIRE(c->n <= 36, "dense state vector limited to 36 qubits");
    RCS_REQUIRE(n_amps == (int64_t(1) << c->n), "psi must hold exactly 2^n amplitudes");
    rcs::dense_simulate(*c, reinterpret_cast<double2*>(psi_dev), rcs::as_stream(stream));
  } catch (const rcs::Error& e) {
    rcs::set_last_error(e.what());
    return e.status;
  }
  return RCS_OK;
}

rcs_status rcs_dense_gather(const double* psi_dev, int32_t n_qubits, const uint64_t* bits_dev, uint64_t m,
                            int32_t probabilities, double* out_dev, void* stream) {
  try {
    RCS_REQUIRE(psi_dev && (bits_dev || m == 0) && (out_dev || m == 0), "null device pointer");
    RCS_REQUIRE(n_qubits >= 1 && n_qubits <= 36, "n_qubits out of range");
    rcs::dense_gather(reinterpret_cast<const double2*>(psi_dev), n_qubits, bits_dev, m, probabilities ? 1 : 0,
                      out_dev, rcs::as_stream(stream));
  } catch (const rcs::Error& e) {
    rcs::set_last_error(e.what());
    return e.status;
  }
  return RCS_OK;
}

}  // extern "C"
