// Shot sampler, amplitude evaluator and linear-XEB reduction.
//
// Sampling (Section 3.2, stage 3) from a right-canonical MPS: for a batch of
// S shots the partial amplitude vectors v (one row per shot) advance site by
// site:  W^s = V A_k^s  (s = 0, 1), a complex GEMM with the shots as the M
// dimension so that every site tensor is streamed once per batch and reused
// by all S shots on the matrix cores.  The GEMM epilogue reduces |W^s|^2 per
// shot over its 64 columns (fixed-order tree), and a per-shot decision step
// sums the column-tile partials in fixed order, draws u from Philox, picks
// the branch and records the bit.  The next site reads its V rows straight
// out of W at the chosen half (no copy).  The last site has a single column,
// whose |w|^2 is p(b).
//
// Because the tensors right of the current site are right-canonical, the two
// branch probabilities of a shot add up to the squared norm of its row
// vector, p0 + p1 = ||v||^2, which the previous site already produced (the
// partial norms of the chosen half).  At the sites past the first whose
// GEMM is large, sampling therefore computes W^0 for every shot, decides
// with u ||v||^2 >= p0, and computes W^1 = v A^1 only for the shots that
// chose 1 (compacted row list): 1.5 instead of 2 shot GEMMs per site on
// average.  Both W halves keep the values the two-branch GEMM gives, and the
// decision differs from u (p0 + p1) >= p0 only where the two sides lie
// within the state's canonical residual of each other.
#include <mutex>

#include "gemm_f64.h"
#include "prof.h"
#include "state.h"

namespace rcs {

struct ChainArgs {
  const double2* wprev = nullptr;  // S x 2*dl from the previous site (null at site 0)
  const int8_t* sel = nullptr;     // per-shot chosen half at the previous site
  const double2* site = nullptr;   // A_k, [s][a][b], dl x dr
  double2* wout = nullptr;         // S x 2*dr
  double* part = nullptr;          // [2][S][ntiles] partial |w|^2
  int S = 0, dl = 0, dr = 0, ntiles = 0;
  int s_fixed = -1;                // >= 0: only this half (grid z = 1); else half = blockIdx.z
  const int* rows = nullptr;       // compacted shot list (logical row -> shot), or null
  const int* nrows = nullptr;      // its length (device), when rows is set
  int* reset = nullptr;            // zeroed by the first thread of the launch, or null
};

__device__ inline void chain_gemm_tile(const ChainArgs& a, int tn, int tm, int s, SmemC64& sm,
                                       double (*rowsum)[GT_M]) {
  const int m0 = tm * GT_M, n0 = tn * GT_N;
  const int M = a.rows ? *a.nrows : a.S;       // logical rows
  if (m0 >= M) return;                         // whole workgroup: nothing to do
  const int dl = a.dl, dr = a.dr;
  auto shot = [&](int m) -> int { return a.rows ? a.rows[m] : m; };
  auto fa = [&](int m, int k) -> double2 {
    if (a.wprev == nullptr) return (k == 0) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
    const int sm_ = shot(m);
    return a.wprev[(int64_t)sm_ * 2 * dl + (int64_t)a.sel[sm_] * dl + k];
  };
  const double2* bs = a.site + (int64_t)s * dl * dr;
  auto fb = [&](int k, int n) -> double2 { return bs[(int64_t)k * dr + n]; };
  LoadA<decltype(fa), true> la{fa, m0, M, dl};
  LoadB<decltype(fb), true> lb{fb, n0, dl, dr};
  AccC64 acc;
  acc_zero(acc);
  cgemm_mainloop(la, lb, dl, sm, acc);

  // store W and reduce |w|^2 per row over this tile's columns
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  double rs[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[mt][r] = 0.0;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = m0 + wm + mt * 16 + f64_row(lane, r);
        int n = n0 + wn + nt * 16 + (lane & 15);
        double re = acc.re[mt][nt][r], im = acc.im[mt][nt][r];
        if (m < M && n < dr) {
          a.wout[(int64_t)shot(m) * 2 * dr + (int64_t)s * dr + n] = make_double2(re, im);
          rs[mt][r] += re * re + im * im;
        }
      }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = rs[mt][r];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if ((lane & 15) == 0) rowsum[w >> 1][wm + mt * 16 + f64_row(lane, r)] = v;
    }
  __syncthreads();
  if (tid < GT_M) {
    int m = m0 + tid;
    if (m < M) a.part[((int64_t)s * a.S + shot(m)) * a.ntiles + tn] = rowsum[0][tid] + rowsum[1][tid];
  }
}

__global__ __launch_bounds__(GT_THREADS) void k_chain_gemm(ChainArgs a) {
  __shared__ SmemC64 sm;
  __shared__ double rowsum[2][GT_M];
  if (a.reset && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *a.reset = 0;
  chain_gemm_tile(a, blockIdx.x, blockIdx.y, a.s_fixed >= 0 ? a.s_fixed : (int)blockIdx.z, sm, rowsum);
}

// Grouped form for a batch of states: group g owns tiles [tile0[g],
// tile0[g+1]) of the launch (ntiles x mtiles of its own GEMM).
struct ChainGroup {
  ChainArgs a;
  int tile0, mtiles;
};

__global__ __launch_bounds__(GT_THREADS) void k_chain_gemm_grouped(const ChainGroup* groups, int ng) {
  __shared__ SmemC64 sm;
  __shared__ double rowsum[2][GT_M];
  const int t = blockIdx.x;
  int g = 0;
  while (g + 1 < ng && groups[g + 1].tile0 <= t) ++g;
  const ChainGroup& G = groups[g];
  const int local = t - G.tile0;
  chain_gemm_tile(G.a, local % G.a.ntiles, local / G.a.ntiles, blockIdx.z, sm, rowsum);
}

struct DecideArgs {
  const double* part = nullptr;
  int S = 0, ntiles = 0, site = 0, qubit = 0, last = 0, mode = 0;
  uint64_t seed = 0, shot0 = 0;
  int8_t* sel = nullptr;
  uint64_t* bits = nullptr;          // mode 0 output
  double* log2p = nullptr;           // mode 0 output (nullable)
  const uint64_t* inbits = nullptr;  // mode 1 input
  const double2* wlast = nullptr;    // S x 2 at the last site
  double2* amps = nullptr;           // mode 1 output
  double* vnorm = nullptr;           // mode 0: ||v||^2 of each shot's next row (nullable)
  int split = 0;                     // only W^0 was computed: decide with u ||v||^2 >= p0
  int* n1 = nullptr;                 // split: length of the list of shots that chose 1
  int* idx1 = nullptr;               // split: that list
};

__device__ inline void decide_one(const DecideArgs& a, int m) {
  if (a.mode == 0 && a.split) {
    double p0 = 0.0;
    const double* q0 = a.part + (int64_t)m * a.ntiles;
    for (int t = 0; t < a.ntiles; ++t) p0 += q0[t];
    const double u = shot_uniform(a.seed, a.shot0 + (uint64_t)m, a.site);
    const int b = (u * a.vnorm[m] >= p0) ? 1 : 0;
    a.bits[m] |= (uint64_t)b << a.qubit;
    a.sel[m] = (int8_t)b;
    if (b == 0)
      a.vnorm[m] = p0;
    else
      a.idx1[atomicAdd(a.n1, 1)] = m;
  } else if (a.mode == 0) {
    double p0 = 0.0, p1 = 0.0;
    const double* q0 = a.part + (int64_t)m * a.ntiles;
    const double* q1 = a.part + ((int64_t)a.S + m) * a.ntiles;
    for (int t = 0; t < a.ntiles; ++t) {
      p0 += q0[t];
      p1 += q1[t];
    }
    const double u = shot_uniform(a.seed, a.shot0 + (uint64_t)m, a.site);
    const int b = (u * (p0 + p1) >= p0) ? 1 : 0;
    const uint64_t bit = (uint64_t)b << a.qubit;
    a.bits[m] = (a.site == 0) ? bit : (a.bits[m] | bit);
    a.sel[m] = (int8_t)b;
    if (a.vnorm) a.vnorm[m] = b ? p1 : p0;
    if (a.last && a.log2p) a.log2p[m] = log2(b ? p1 : p0);
  } else {
    const int b = (int)((a.inbits[m] >> a.qubit) & 1ull);
    a.sel[m] = (int8_t)b;
    if (a.last) a.amps[m] = a.wlast[(int64_t)m * 2 + b];
  }
}

__global__ void k_decide(DecideArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < a.S) decide_one(a, m);
}

// ||v||^2 of the shots that chose 1 at a split site: their W^1 partial
// norms, summed in the same order as the two-branch decision sums p1.
__global__ void k_vnorm1(const double* part, int S, int ntiles, const int* idx1, const int* n1, double* vnorm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n1) return;
  const int m = idx1[i];
  const double* q1 = part + ((int64_t)S + m) * ntiles;
  double p1 = 0.0;
  for (int t = 0; t < ntiles; ++t) p1 += q1[t];
  vnorm[m] = p1;
}

__global__ void k_decide_grouped(const DecideArgs* groups) {
  const DecideArgs& a = groups[blockIdx.y];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < a.S) decide_one(a, m);
}

int state_max_bond(const rcs_state_s& st) {
  int maxd = 1;
  for (int d : st.dims) maxd = std::max(maxd, d);
  return maxd;
}

// Bytes of sampler workspace for S shots per pass at maximum bond maxd:
// two ping-pong W buffers (S x 2 maxd complex), the per-shot partial norms
// of every column tile of both branches, the chosen branch per shot, the
// per-shot ||v||^2, the list of shots that chose 1 and its length.  The
// chosen branch is double-buffered by site parity: a split site's W^1 GEMM
// runs after its decision and still reads the previous site's choice.
size_t chain_work_bytes(int64_t S, int maxd) {
  const int ntiles = ceil_div(maxd, GT_N);
  return 2 * round_up((size_t)S * 2 * maxd * sizeof(double2), 256) +
         round_up((size_t)2 * S * ntiles * sizeof(double), 256) + 2 * round_up((size_t)S, 256) +
         round_up((size_t)S * sizeof(double), 256) + round_up((size_t)S * sizeof(int), 256) + 256;
}

ChainBuffers chain_buffers_in(char* base, int64_t S, int maxd) {
  const int ntiles = ceil_div(maxd, GT_N);
  ChainBuffers b;
  b.S0 = S;
  size_t off = 0;
  const size_t wb = round_up((size_t)S * 2 * maxd * sizeof(double2), 256);
  b.w[0] = reinterpret_cast<double2*>(base);
  b.w[1] = reinterpret_cast<double2*>(base + wb);
  off = 2 * wb;
  b.part = reinterpret_cast<double*>(base + off);
  off += round_up((size_t)2 * S * ntiles * sizeof(double), 256);
  b.sel = reinterpret_cast<int8_t*>(base + off);
  off += round_up((size_t)S, 256);
  b.sel2 = reinterpret_cast<int8_t*>(base + off);
  off += round_up((size_t)S, 256);
  b.vnorm = reinterpret_cast<double*>(base + off);
  off += round_up((size_t)S * sizeof(double), 256);
  b.idx1 = reinterpret_cast<int*>(base + off);
  off += round_up((size_t)S * sizeof(int), 256);
  b.n1 = reinterpret_cast<int*>(base + off);
  return b;
}

void run_chain(rcs_state_s& st, uint64_t first_shot, uint64_t n_shots, uint64_t seed, int mode,
               uint64_t* bits_dev, double* log2p_dev, const uint64_t* in_bits_dev,
               double* amps_dev) {
  if (n_shots == 0) return;
  const int maxd = state_max_bond(st);
  int64_t smax = (int64_t(1) << 30) / (2 * (int64_t)maxd * 16);
  smax = std::max<int64_t>(64, std::min<int64_t>(65536, smax / 64 * 64));
  const int64_t S0 = std::min<int64_t>(smax, (int64_t)round_up((int64_t)n_shots, 64));
  const int ntiles_max = ceil_div(maxd, GT_N);
  st.wbuf[0].ensure((size_t)S0 * 2 * maxd * sizeof(double2));
  st.wbuf[1].ensure((size_t)S0 * 2 * maxd * sizeof(double2));
  st.part.ensure((size_t)2 * S0 * ntiles_max * sizeof(double));
  st.sel.ensure((size_t)2 * S0);
  st.vnorm.ensure((size_t)S0 * sizeof(double));
  st.idx1.ensure((size_t)S0 * sizeof(int) + 256);
  ChainBuffers b;
  b.S0 = S0;
  b.w[0] = st.wbuf[0].as<double2>();
  b.w[1] = st.wbuf[1].as<double2>();
  b.part = st.part.as<double>();
  b.sel = st.sel.as<int8_t>();
  b.sel2 = st.sel.as<int8_t>() + S0;
  b.vnorm = st.vnorm.as<double>();
  b.idx1 = st.idx1.as<int>();
  b.n1 = reinterpret_cast<int*>(st.idx1.as<char>() + round_up((size_t)S0 * sizeof(int), 256));
  run_chain_with(st, b, first_shot, n_shots, seed, mode, bits_dev, log2p_dev, in_bits_dev, amps_dev);
}

void run_chain_with(rcs_state_s& st, const ChainBuffers& buf, uint64_t first_shot, uint64_t n_shots,
                    uint64_t seed, int mode, uint64_t* bits_dev, double* log2p_dev,
                    const uint64_t* in_bits_dev, double* amps_dev, bool probe) {
  if (n_shots == 0) return;
  const int64_t S0 = buf.S0;
  for (uint64_t b0 = 0; b0 < n_shots; b0 += (uint64_t)S0) {
    const int S = (int)std::min<uint64_t>((uint64_t)S0, n_shots - b0);
    for (int k = 0; k < st.n; ++k) {
      int8_t* sel_prev = (k & 1) ? buf.sel : buf.sel2;   // written by site k - 1
      int8_t* sel_cur = (k & 1) ? buf.sel2 : buf.sel;
      ChainArgs ca;
      ca.wprev = (k == 0) ? nullptr : buf.w[(k - 1) & 1];
      ca.sel = sel_prev;
      ca.site = st.site[k];
      ca.wout = buf.w[k & 1];
      ca.part = buf.part;
      ca.S = S;
      ca.dl = st.dims[k];
      ca.dr = st.dims[k + 1];
      ca.ntiles = ceil_div(ca.dr, GT_N);
      // split sites: past the first, not the last, GEMM large enough
      const bool split = mode == 0 && k > 0 && k < st.n - 1 && (int64_t)ca.dl * ca.dr >= 1024 &&
                         buf.vnorm && buf.idx1 && buf.n1;
      if (split) {
        ca.s_fixed = 0;
        ca.reset = buf.n1;
      }
      dim3 grid(ca.ntiles, ceil_div(S, GT_M), split ? 1 : 2);
      {
        // algorithmic: complex GEMMs S x dl x dr per half (8 real flops per
        // complex multiply-add); HBM: site tensor + V rows read + W written
        const double halves = split ? 1.0 : 2.0;
        const double fl = 8.0 * halves * S * (double)ca.dl * ca.dr;
        const double by = 16.0 * (halves * ca.dl * ca.dr + (double)S * ca.dl + halves * S * ca.dr);
        Probe pr(probe ? kKcChainGemm : -1, st.stream, fl, by);
        hipExtLaunchKernelGGL(k_chain_gemm, grid, dim3(GT_THREADS), 0, st.stream, pr.start(), pr.stop(), 0, ca);
      }
      HIP_LAUNCH_OK();
      DecideArgs da;
      da.part = ca.part;
      da.S = S;
      da.ntiles = ca.ntiles;
      da.site = k;
      da.qubit = st.pi[k];
      da.last = (k == st.n - 1);
      da.mode = mode;
      da.seed = seed;
      da.shot0 = first_shot + b0;
      da.sel = sel_cur;
      da.bits = bits_dev ? bits_dev + b0 : nullptr;
      da.log2p = log2p_dev ? log2p_dev + b0 : nullptr;
      da.inbits = in_bits_dev ? in_bits_dev + b0 : nullptr;
      da.wlast = ca.wout;
      da.amps = amps_dev ? reinterpret_cast<double2*>(amps_dev) + b0 : nullptr;
      da.vnorm = mode == 0 ? buf.vnorm : nullptr;
      da.split = split ? 1 : 0;
      da.n1 = buf.n1;
      da.idx1 = buf.idx1;
      hipLaunchKernelGGL(k_decide, dim3(ceil_div(S, 256)), dim3(256), 0, st.stream, da);
      HIP_LAUNCH_OK();
      if (split) {
        // W^1 for the shots that chose 1 (work about half the W^0 GEMM's)
        ChainArgs cb = ca;
        cb.s_fixed = 1;
        cb.reset = nullptr;
        cb.rows = buf.idx1;
        cb.nrows = buf.n1;
        {
          const double fl = 8.0 * 0.5 * S * (double)ca.dl * ca.dr;
          const double by = 16.0 * (ca.dl * ca.dr + 0.5 * S * ca.dl + 0.5 * S * ca.dr);
          Probe pr(probe ? kKcChainGemm : -1, st.stream, fl, by);
          hipExtLaunchKernelGGL(k_chain_gemm, grid, dim3(GT_THREADS), 0, st.stream, pr.start(), pr.stop(), 0, cb);
        }
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_vnorm1, dim3(ceil_div(S, 256)), dim3(256), 0, st.stream, ca.part, S, ca.ntiles,
                           buf.idx1, buf.n1, buf.vnorm);
        HIP_LAUNCH_OK();
      }
    }
  }
}

// ------------------------------------------------ allocation-free sampling
// Workspace for callers that cannot allocate device memory: one statically
// sized device array, of which every GPU the library runs on holds its own
// copy until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name is
// not a device address in host code).  Nothing in it has to start at zero:
// every pass writes the partial norms, the chosen branches and the W rows it
// later reads.  All calls on one GPU share the array, so calls that overlap
// on one GPU (two streams, two threads) race.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device
// with that device current.
static char* scratch_on(int dev) {
  RCS_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIP_OK(hipGetDevice(&cur));
    if (cur != dev) HIP_OK(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIP_OK(hipSetDevice(cur));
    HIP_OK(e);
    RCS_REQUIRE(ptr != nullptr, "no device address for the sampler scratch");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Largest shot pass (a multiple of 64, at most 65,536) whose workspace fits
// the scratch array at maximum bond maxd; 0 when not even 64 shots fit.
int64_t noalloc_pass_shots(int maxd) {
  int64_t S = 65536;
  while (S >= 64 && chain_work_bytes(S, maxd) > kNoAllocScratchBytes) S -= 64;
  return S >= 64 ? S : 0;
}

void run_chain_noalloc(rcs_state_s& st, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                       uint64_t* bits_dev, double* log2p_dev) {
  const int maxd = state_max_bond(st);
  const int64_t smax = noalloc_pass_shots(maxd);
  if (smax == 0)
    fail(RCS_ERR_INVALID_ARG, "state's bond dimension too large for the allocation-free sampler's scratch");
  char* base = scratch_on(st.device);
  if (n_shots == 0) return;
  const int64_t S0 = std::min<int64_t>(smax, (int64_t)round_up((int64_t)n_shots, 64));
  const ChainBuffers b = chain_buffers_in(base, S0, maxd);
  run_chain_with(st, b, first_shot, n_shots, seed, 0, bits_dev, log2p_dev, nullptr, nullptr, false);
}

// Batched sampling: for every shot pass and site index, one grouped GEMM
// launch over all states that have that site and one grouped decision
// launch.  All launch descriptors are built on the host up front and
// uploaded once, so the whole sequence is captured into a HIP graph (on a
// private stream) and replayed.
void run_chain_batch(rcs_state_s** states, int n, uint64_t n_shots, uint64_t seed, uint64_t* bits_dev,
                     double* log2p_dev, hipStream_t user_stream) {
  if (n == 0 || n_shots == 0) return;
  int maxd = 1, maxn = 0;
  for (int i = 0; i < n; ++i) {
    for (int d : states[i]->dims) maxd = std::max(maxd, d);
    maxn = std::max(maxn, states[i]->n);
  }
  // shots per state per pass, so that all W buffers together stay <= 4 GiB
  int64_t S0 = ((int64_t)1 << 32) / ((int64_t)n * 2 * 2 * maxd * 16);
  S0 = std::max<int64_t>(64, std::min<int64_t>(16384, S0 / 64 * 64));
  S0 = std::min<int64_t>(S0, round_up((int64_t)n_shots, 64));
  const int ntiles_max = ceil_div(maxd, GT_N);
  DevBuf w0, w1, part, sel;
  w0.ensure((size_t)n * S0 * 2 * maxd * sizeof(double2));
  w1.ensure((size_t)n * S0 * 2 * maxd * sizeof(double2));
  part.ensure((size_t)n * 2 * S0 * ntiles_max * sizeof(double));
  sel.ensure((size_t)n * S0);
  const int passes = (int)((n_shots + S0 - 1) / S0);
  // descriptors: per (pass, site): groups of states with site k
  std::vector<ChainGroup> cg;
  std::vector<DecideArgs> dg;
  struct Launch {
    size_t c0, d0;
    int ng, tiles, S;
  };
  std::vector<Launch> launches;
  for (int pass = 0; pass < passes; ++pass) {
    const uint64_t b0 = (uint64_t)pass * S0;
    const int S = (int)std::min<uint64_t>((uint64_t)S0, n_shots - b0);
    for (int k = 0; k < maxn; ++k) {
      Launch L{cg.size(), dg.size(), 0, 0, S};
      for (int i = 0; i < n; ++i) {
        rcs_state_s& st = *states[i];
        if (k >= st.n) continue;
        double2* wb0 = w0.as<double2>() + (size_t)i * S0 * 2 * maxd;
        double2* wb1 = w1.as<double2>() + (size_t)i * S0 * 2 * maxd;
        ChainGroup g;
        g.a.wprev = (k == 0) ? nullptr : ((k - 1) & 1 ? wb1 : wb0);
        g.a.sel = sel.as<int8_t>() + (size_t)i * S0;
        g.a.site = st.site[k];
        g.a.wout = (k & 1) ? wb1 : wb0;
        g.a.part = part.as<double>() + (size_t)i * 2 * S0 * ntiles_max;
        g.a.S = S;
        g.a.dl = st.dims[k];
        g.a.dr = st.dims[k + 1];
        g.a.ntiles = ceil_div(g.a.dr, GT_N);
        g.mtiles = ceil_div(S, GT_M);
        g.tile0 = L.tiles;
        L.tiles += g.a.ntiles * g.mtiles;
        cg.push_back(g);
        DecideArgs d;
        d.part = g.a.part;
        d.S = S;
        d.ntiles = g.a.ntiles;
        d.site = k;
        d.qubit = st.pi[k];
        d.last = (k == st.n - 1);
        d.mode = 0;
        d.seed = seed;
        d.shot0 = b0;
        d.sel = sel.as<int8_t>() + (size_t)i * S0;
        d.bits = bits_dev + (uint64_t)i * n_shots + b0;
        d.log2p = log2p_dev ? log2p_dev + (uint64_t)i * n_shots + b0 : nullptr;
        d.inbits = nullptr;
        d.wlast = g.a.wout;
        d.amps = nullptr;
        dg.push_back(d);
        L.ng += 1;
      }
      if (L.ng) launches.push_back(L);
    }
  }
  DevBuf dcg, ddg;
  dcg.ensure(cg.size() * sizeof(ChainGroup));
  ddg.ensure(dg.size() * sizeof(DecideArgs));
  HIP_OK(hipMemcpyAsync(dcg.p, cg.data(), cg.size() * sizeof(ChainGroup), hipMemcpyHostToDevice, user_stream));
  HIP_OK(hipMemcpyAsync(ddg.p, dg.data(), dg.size() * sizeof(DecideArgs), hipMemcpyHostToDevice, user_stream));
  HIP_OK(hipStreamSynchronize(user_stream));
  hipStream_t cs;
  HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (const Launch& L : launches) {
    hipLaunchKernelGGL(k_chain_gemm_grouped, dim3(L.tiles, 1, 2), dim3(GT_THREADS), 0, cs,
                       dcg.as<ChainGroup>() + L.c0, L.ng);
    hipLaunchKernelGGL(k_decide_grouped, dim3(ceil_div(L.S, 256), L.ng), dim3(256), 0, cs,
                       ddg.as<DecideArgs>() + L.d0);
  }
  hipError_t ce = hipStreamEndCapture(cs, &graph);
  if (ce == hipSuccess) ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ce == hipSuccess) ce = hipGraphLaunch(exec, cs);
  if (ce == hipSuccess) ce = hipStreamSynchronize(cs);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  HIP_OK(ce);
}

__global__ void k_abs2(const double2* z, uint64_t m, double* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = z[i].x * z[i].x + z[i].y * z[i].y;
}

void abs2_to(const double2* z, uint64_t m, double* out, hipStream_t stream) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_abs2, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, z, m, out);
  HIP_LAUNCH_OK();
}

// ------------------------------------------------------------------- XEB
// Section 5.1: F = 2^n mean(p) - 1.  Two fixed-order passes (mean, then
// squared deviations) over per-block partial sums; the host adds the block
// partials in index order.
constexpr int XEB_BLOCK = 256;
constexpr int XEB_PER_THREAD = 16;

__device__ inline double xeb_term(const double* v, uint64_t i, int nq, int is_log2) {
  return is_log2 ? exp2(v[i] + (double)nq) : ldexp(v[i], nq);
}

__global__ void k_xeb_partial(const double* vals, uint64_t m, int nq, int is_log2, int pass,
                              double mean, double* out) {
  __shared__ double red[XEB_BLOCK];
  const uint64_t base = (uint64_t)blockIdx.x * XEB_BLOCK * XEB_PER_THREAD;
  double acc = 0.0;
  for (int j = 0; j < XEB_PER_THREAD; ++j) {
    uint64_t i = base + (uint64_t)j * XEB_BLOCK + threadIdx.x;
    if (i < m) {
      double x = xeb_term(vals, i, nq, is_log2);
      acc += pass == 0 ? x : (x - mean) * (x - mean);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = XEB_BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

void xeb_reduce(int n_qubits, const double* vals_dev, uint64_t m, bool is_log2, double* xeb,
                double* se, hipStream_t stream) {
  RCS_REQUIRE(m >= 2, "need at least two samples");
  RCS_REQUIRE(n_qubits >= 1 && n_qubits <= 64, "n_qubits out of range");
  const uint64_t per = (uint64_t)XEB_BLOCK * XEB_PER_THREAD;
  const int nb = (int)((m + per - 1) / per);
  DevBuf part;
  part.ensure((size_t)nb * sizeof(double));
  std::vector<double> h(nb);
  double sums[2] = {0.0, 0.0};
  double mean = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_xeb_partial, dim3(nb), dim3(XEB_BLOCK), 0, stream, vals_dev, m, n_qubits,
                       is_log2 ? 1 : 0, pass, mean, part.as<double>());
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(h.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += h[i];
    sums[pass] = s;
    if (pass == 0) mean = s / (double)m;
  }
  *xeb = mean - 1.0;
  *se = std::sqrt(sums[1] / (double)(m - 1)) / std::sqrt((double)m);
}

}  // namespace rcs

