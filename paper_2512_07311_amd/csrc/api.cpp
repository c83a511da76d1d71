// C ABI entry points: circuits, state access, sampling, amplitudes, XEB.
#include <memory>
#include <string>
#include <cstring>
#include <cstdio>
#include <algorithm>
#include <cmath>
#include <mutex>

#include "circuit.h"
#include "state.h"

namespace rcs {
static thread_local std::string g_last_error;
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }
}  // namespace rcs

#define RCS_API_BEGIN try {
#define RCS_API_END                                      \
  }                                                      \
  catch (const rcs::Error& e) {                          \
    rcs::set_last_error(e.what());                       \
    return e.status;                                     \
  }                                                      \
  catch (const std::bad_alloc&) {                        \
    rcs::set_last_error("host allocation failed");       \
    return RCS_ERR_OUT_OF_MEMORY;                        \
  }                                                      \
  catch (const std::exception& e) {                      \
    rcs::set_last_error(e.what());                       \
    return RCS_ERR_DEVICE;                               \
  }                                                      \
  return RCS_OK;

extern "C" {

const char* rcs_last_error(void) { return rcs::g_last_error.c_str(); }
const char* rcs_version(void) { return "librcs 0.1 gfx950"; }

// ---------------------------------------------------------------- circuits
rcs_status rcs_circuit_create(const rcs_circuit_desc* desc, rcs_circuit* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(desc && out, "null argument");
  *out = nullptr;
  auto c = std::make_unique<rcs_circuit_s>();
  rcs::generate_circuit(*desc, *c);
  *out = c.release();
  RCS_API_END
}

void rcs_circuit_destroy(rcs_circuit c) { delete c; }

rcs_status rcs_circuit_info(rcs_circuit c, int32_t* n_qubits, int32_t* n_layers_1q,
                            int32_t* n_ops, int32_t* n_updates) {
  RCS_API_BEGIN
  RCS_REQUIRE(c, "null circuit");
  if (n_qubits) *n_qubits = c->n;
  if (n_layers_1q) *n_layers_1q = (int32_t)c->layers_1q.size();
  if (n_ops) *n_ops = (int32_t)c->ops.size();
  if (n_updates) *n_updates = c->n_updates;
  RCS_API_END
}

rcs_status rcs_circuit_one_qubit_gates(rcs_circuit c, int32_t* gates_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(c && gates_host, "null argument");
  for (size_t l = 0; l < c->layers_1q.size(); ++l)
    for (int q = 0; q < c->n; ++q) gates_host[l * c->n + q] = c->layers_1q[l][q];
  RCS_API_END
}

rcs_status rcs_circuit_schedule(rcs_circuit c, int32_t* snake_host, int32_t* ops_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(c, "null circuit");
  if (snake_host)
    for (int p = 0; p < c->n; ++p) snake_host[p] = c->snake[p];
  if (ops_host)
    for (size_t o = 0; o < c->ops.size(); ++o) {
      ops_host[4 * o + 0] = c->ops[o].kind;
      ops_host[4 * o + 1] = c->ops[o].arg;
      ops_host[4 * o + 2] = c->ops[o].gate;
      ops_host[4 * o + 3] = c->ops[o].cycle;
    }
  RCS_API_END
}

// ------------------------------------------------------------ state access
rcs_status rcs_state_info_get(rcs_state s, rcs_state_info* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(s && out, "null argument");
  rcs_state_info inf{};
  inf.n_qubits = s->n;
  inf.max_bond = *std::max_element(s->dims.begin(), s->dims.end());
  inf.center = s->center;
  inf.canonical = s->canonical ? 1 : 0;
  inf.n_truncations = s->n_trunc;
  inf.n_fallbacks = s->n_fallback;
  inf.n_rsvd_accepted = s->n_rsvd_ok;
  inf.jacobi_sweeps_max = s->jacobi_sweeps_max;
  inf.log_fidelity_est = s->log_fest;
  inf.sum_eps = s->sum_eps;
  inf.build_seconds = s->build_seconds;
  inf.svd_seconds = s->svd_seconds;
  inf.device_bytes = (int64_t)(s->slab.bytes + s->spare.bytes);
  inf.n_center_moves = s->n_moves;
  inf.nominal_svd_flops = s->nominal_svd_flops;
  inf.nominal_qr_flops = s->nominal_qr_flops;
  inf.n_precond = s->n_precond;
  inf.n_precond_fallback = s->n_precond_fallback;
  inf.n_center_moves_cholqr = s->n_moves_cholqr;
  inf.n_svd_f32 = s->n_svd_f32;
  inf.n_svd_f32_redone = s->n_svd_f32_redone;
  *out = inf;
  RCS_API_END
}

rcs_status rcs_state_layout(rcs_state s, int32_t* bond_dims_host, int32_t* snake_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  if (bond_dims_host)
    for (int k = 0; k < s->n - 1; ++k) bond_dims_host[k] = s->dims[k + 1];
  if (snake_host)
    for (int k = 0; k < s->n; ++k) snake_host[k] = s->pi[k];
  RCS_API_END
}

rcs_status rcs_state_set_stream(rcs_state s, void* stream) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  s->stream = rcs::as_stream(stream);
  RCS_API_END
}

rcs_status rcs_state_export(rcs_state s, double* tensors_host, int64_t count_doubles,
                            int64_t* needed_doubles) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  int64_t need = 0;
  for (int k = 0; k < s->n; ++k) need += (int64_t)s->dims[k] * 2 * s->dims[k + 1] * 2;
  if (needed_doubles) *needed_doubles = need;
  if (!tensors_host) return RCS_OK;
  RCS_REQUIRE(count_doubles >= need, "output buffer too small");
  std::vector<double2> tmp;
  int64_t off = 0;
  for (int k = 0; k < s->n; ++k) {
    const int dl = s->dims[k], dr = s->dims[k + 1];
    tmp.resize((size_t)dl * 2 * dr);
    HIP_OK(hipMemcpyAsync(tmp.data(), s->site[k], tmp.size() * sizeof(double2),
                          hipMemcpyDeviceToHost, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    // device [s][a][b] -> host (a, s, b)
    for (int a = 0; a < dl; ++a)
      for (int ph = 0; ph < 2; ++ph)
        for (int b = 0; b < dr; ++b) {
          const double2 v = tmp[((size_t)ph * dl + a) * dr + b];
          const int64_t o = off + (((int64_t)a * 2 + ph) * dr + b) * 2;
          tensors_host[o] = v.x;
          tensors_host[o + 1] = v.y;
        }
    off += (int64_t)dl * 2 * dr * 2;
  }
  RCS_API_END
}

rcs_status rcs_state_import(int32_t n, const int32_t* dims_host, const int32_t* snake_host,
                            const double* tensors_host, int32_t canonical, void* stream,
                            rcs_state* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(out && dims_host && snake_host && tensors_host, "null argument");
  *out = nullptr;
  RCS_REQUIRE(n >= 1 && n <= 64, "n must be in [1, 64]");
  RCS_REQUIRE(dims_host[0] == 1 && dims_host[n] == 1, "boundary bond dimensions must be 1");
  std::vector<char> seen(n, 0);
  for (int k = 0; k < n; ++k) {
    RCS_REQUIRE(snake_host[k] >= 0 && snake_host[k] < n && !seen[snake_host[k]],
                "snake must be a permutation of 0..n-1");
    seen[snake_host[k]] = 1;
  }
  int chi = 1;
  for (int k = 0; k <= n; ++k) {
    RCS_REQUIRE(dims_host[k] >= 1 && dims_host[k] <= 8192, "bond dimension out of range");
    chi = std::max(chi, (int)dims_host[k]);
  }
  auto st = std::make_unique<rcs_state_s>();
  st->stream = rcs::as_stream(stream);
  HIP_OK(hipGetDevice(&st->device));
  rcs::state_alloc(*st, n, chi);
  for (int k = 0; k <= n; ++k)
    RCS_REQUIRE(dims_host[k] <= st->cap[k], "bond dimension exceeds 2^min(k, n-k)");
  st->dims.assign(dims_host, dims_host + n + 1);
  st->pi.assign(snake_host, snake_host + n);
  std::vector<double2> tmp;
  int64_t off = 0;
  for (int k = 0; k < n; ++k) {
    const int dl = st->dims[k], dr = st->dims[k + 1];
    tmp.resize((size_t)dl * 2 * dr);
    for (int a = 0; a < dl; ++a)
      for (int ph = 0; ph < 2; ++ph)
        for (int b = 0; b < dr; ++b) {
          const int64_t o = off + (((int64_t)a * 2 + ph) * dr + b) * 2;
          tmp[((size_t)ph * dl + a) * dr + b] = make_double2(tensors_host[o], tensors_host[o + 1]);
        }
    HIP_OK(hipMemcpyAsync(st->site[k], tmp.data(), tmp.size() * sizeof(double2),
                          hipMemcpyHostToDevice, st->stream));
    HIP_OK(hipStreamSynchronize(st->stream));
    off += (int64_t)dl * 2 * dr * 2;
  }
  st->canonical = canonical != 0;
  st->center = 0;
  *out = st.release();
  RCS_API_END
}

// ------------------------------------------------------------ persistence
// File layout (little-endian): 8-byte magic "RCSMPS1\n"; int32 version (1),
// n, canonical, reserved (0); float64 log_fidelity_est; int32 dims[n+1];
// int32 snake[n]; the site tensors as rcs_state_export writes them (A_k of
// shape (dims[k], 2, dims[k+1]), row-major complex128); uint64 checksum =
// FNV-1a over the preceding bytes taken as 64-bit words.
namespace {
constexpr char kMagic[8] = {'R', 'C', 'S', 'M', 'P', 'S', '1', '\n'};

// FNV-1a over a byte stream taken as little-endian 64-bit words, the last
// (length mod 8) bytes one at a time; add() may be called with any split
// of the stream.
struct Fnv64 {
  uint64_t h = 1469598103934665603ull;
  unsigned char pend[8];
  int np = 0;
  void word(uint64_t w) { h = (h ^ w) * 1099511628211ull; }
  void add(const void* p, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    size_t i = 0;
    while (np > 0 && i < bytes) {
      pend[np++] = c[i++];
      if (np == 8) {
        uint64_t w;
        std::memcpy(&w, pend, 8);
        word(w);
        np = 0;
      }
    }
    for (; i + 8 <= bytes; i += 8) {
      uint64_t w;
      std::memcpy(&w, c + i, 8);
      word(w);
    }
    for (; i < bytes; ++i) pend[np++] = c[i];
  }
  uint64_t finish() {
    for (int i = 0; i < np; ++i) h = (h ^ pend[i]) * 1099511628211ull;
    np = 0;
    return h;
  }
};

struct FileCloser {
  void operator()(std::FILE* f) const {
    if (f) std::fclose(f);
  }
};
using FilePtr = std::unique_ptr<std::FILE, FileCloser>;
}  // namespace

rcs_status rcs_state_save(rcs_state s, const char* path) {
  RCS_API_BEGIN
  RCS_REQUIRE(s && path, "null argument");
  int64_t need = 0;
  rcs_status e = rcs_state_export(s, nullptr, 0, &need);
  if (e != RCS_OK) return e;
  std::vector<double> t((size_t)need);
  e = rcs_state_export(s, t.data(), need, nullptr);
  if (e != RCS_OK) return e;
  const int32_t hdr[4] = {1, s->n, s->canonical ? 1 : 0, 0};
  std::vector<int32_t> dims(s->dims.begin(), s->dims.end()), snake(s->pi.begin(), s->pi.end());
  const std::string tmp_path = std::string(path) + ".tmp";
  Fnv64 h;
  {
    FilePtr f(std::fopen(tmp_path.c_str(), "wb"));
    if (!f) rcs::fail(RCS_ERR_INVALID_ARG, std::string("cannot open for writing: ") + path);
    auto put = [&](const void* p, size_t bytes) {
      h.add(p, bytes);
      if (std::fwrite(p, 1, bytes, f.get()) != bytes) rcs::fail(RCS_ERR_DEVICE, "write failed");
    };
    put(kMagic, 8);
    put(hdr, sizeof(hdr));
    put(&s->log_fest, sizeof(double));
    put(dims.data(), dims.size() * sizeof(int32_t));
    put(snake.data(), snake.size() * sizeof(int32_t));
    put(t.data(), t.size() * sizeof(double));
    const uint64_t sum = h.finish();
    if (std::fwrite(&sum, 1, 8, f.get()) != 8) rcs::fail(RCS_ERR_DEVICE, "write failed");
    if (std::fflush(f.get()) != 0) rcs::fail(RCS_ERR_DEVICE, "write failed");
  }
  // the file appears complete or not at all
  if (std::rename(tmp_path.c_str(), path) != 0) rcs::fail(RCS_ERR_DEVICE, "rename failed");
  RCS_API_END
}

rcs_status rcs_state_load(const char* path, void* stream, rcs_state* out) {
  RCS_API_BEGIN
  RCS_REQUIRE(path && out, "null argument");
  *out = nullptr;
  FilePtr f(std::fopen(path, "rb"));
  if (!f) rcs::fail(RCS_ERR_INVALID_ARG, std::string("cannot open: ") + path);
  Fnv64 h;
  auto get = [&](void* p, size_t bytes) {
    if (std::fread(p, 1, bytes, f.get()) != bytes) rcs::fail(RCS_ERR_INVALID_ARG, "truncated state file");
    h.add(p, bytes);
  };
  char magic[8];
  get(magic, 8);
  RCS_REQUIRE(std::memcmp(magic, kMagic, 8) == 0, "not a state file (bad magic)");
  int32_t hdr[4];
  get(hdr, sizeof(hdr));
  RCS_REQUIRE(hdr[0] == 1, "unsupported state file version");
  const int n = hdr[1];
  RCS_REQUIRE(n >= 1 && n <= 64, "bad qubit count in state file");
  double log_fest = 0.0;
  get(&log_fest, sizeof(double));
  std::vector<int32_t> dims(n + 1), snake(n);
  get(dims.data(), dims.size() * sizeof(int32_t));
  get(snake.data(), snake.size() * sizeof(int32_t));
  int64_t need = 0;
  for (int k = 0; k < n; ++k) {
    RCS_REQUIRE(dims[k] >= 1 && dims[k] <= 8192 && dims[k + 1] >= 1 && dims[k + 1] <= 8192,
                "bond dimension out of range in state file");
    need += (int64_t)dims[k] * 2 * dims[k + 1] * 2;
  }
  std::vector<double> t((size_t)need);
  get(t.data(), t.size() * sizeof(double));
  uint64_t sum = 0;
  if (std::fread(&sum, 1, 8, f.get()) != 8) rcs::fail(RCS_ERR_INVALID_ARG, "truncated state file");
  RCS_REQUIRE(sum == h.finish(), "state file checksum mismatch");
  rcs_state st = nullptr;
  const rcs_status e = rcs_state_import(n, dims.data(), snake.data(), t.data(), hdr[2], stream, &st);
  if (e != RCS_OK) return e;
  st->log_fest = log_fest;
  *out = st;
  RCS_API_END
}

void rcs_state_destroy(rcs_state s) {
  if (s && s->stream) (void)hipStreamSynchronize(s->stream);
  delete s;
}

rcs_status rcs_state_spectra(rcs_state s, int32_t* n_records, int64_t* n_values,
                             int32_t* meta_host, double* values_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  int64_t nv = 0;
  for (auto& r : s->spectra) nv += (int64_t)r.values.size();
  if (n_records) *n_records = (int32_t)s->spectra.size();
  if (n_values) *n_values = nv;
  int64_t o = 0;
  for (size_t i = 0; i < s->spectra.size(); ++i) {
    const auto& r = s->spectra[i];
    if (meta_host) {
      int32_t* m = meta_host + 6 * i;
      m[0] = r.pos;
      m[1] = r.cycle;
      m[2] = r.m;
      m[3] = r.kept;
      m[4] = r.chi_l;
      m[5] = r.chi_r;
    }
    if (values_host) std::copy(r.values.begin(), r.values.end(), values_host + o);
    o += (int64_t)r.values.size();
  }
  RCS_API_END
}

rcs_status rcs_state_updates(rcs_state s, int32_t* n_updates, int32_t* records_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  if (n_updates) *n_updates = (int32_t)s->updates.size();
  if (records_host)
    for (size_t i = 0; i < s->updates.size(); ++i) {
      const auto& u = s->updates[i];
      int32_t* r = records_host + 7 * i;
      r[0] = u.pos;
      r[1] = u.cycle;
      r[2] = u.chi_l;
      r[3] = u.chi_m;
      r[4] = u.chi_r;
      r[5] = u.kept;
      r[6] = u.path;
    }
  RCS_API_END
}

rcs_status rcs_state_rsvd_log(rcs_state s, int32_t* n_records, int64_t* n_values, int32_t* ints_host,
                              double* doubles_host, float* net_host, double* values_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  int64_t nv = 0;
  for (const auto& r : s->rsvd_log) nv += (int64_t)r.values.size();
  if (n_records) *n_records = (int32_t)s->rsvd_log.size();
  if (n_values) *n_values = nv;
  int64_t o = 0;
  for (size_t i = 0; i < s->rsvd_log.size(); ++i) {
    const auto& r = s->rsvd_log[i];
    if (ints_host) {
      int32_t* q = ints_host + 10 * i;
      q[0] = r.update;
      q[1] = r.pos;
      q[2] = r.cycle;
      q[3] = r.m;
      q[4] = r.k_hat;
      q[5] = r.l;
      q[6] = r.k;
      q[7] = r.accepted;
      q[8] = r.early;
      q[9] = (int32_t)r.values.size();
    }
    if (doubles_host) {
      double* d = doubles_host + 4 * i;
      d[0] = r.eps_pred;
      d[1] = r.eps_rand;
      d[2] = r.outside;
      d[3] = r.total;
    }
    if (net_host) {
      std::copy(r.feat, r.feat + 66, net_host + 98 * i);
      std::copy(r.y, r.y + 32, net_host + 98 * i + 66);
    }
    if (values_host) std::copy(r.values.begin(), r.values.end(), values_host + o);
    o += (int64_t)r.values.size();
  }
  RCS_API_END
}

// ------------------------------------------------------------- sampling
rcs_status rcs_sample_range(rcs_state s, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                            uint64_t* bits_dev, double* log2p_dev) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  RCS_REQUIRE(bits_dev || n_shots == 0, "null bits_dev");
  if (!s->canonical) rcs::fail(RCS_ERR_STATE, "rcs_sample: state is not right-canonical");
  rcs::run_chain(*s, first_shot, n_shots, seed, 0, bits_dev, log2p_dev, nullptr, nullptr);
  RCS_API_END
}

rcs_status rcs_sample_range_noalloc(rcs_state s, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                                    uint64_t* bits_dev, double* log2p_dev) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  RCS_REQUIRE(bits_dev || n_shots == 0, "null bits_dev");
  if (!s->canonical) rcs::fail(RCS_ERR_STATE, "rcs_sample_range_noalloc: state is not right-canonical");
  rcs::run_chain_noalloc(*s, first_shot, n_shots, seed, bits_dev, log2p_dev);
  RCS_API_END
}

rcs_status rcs_sample(rcs_state s, uint64_t n_shots, uint64_t seed, uint64_t* bits_dev,
                      double* log2p_dev) {
  return rcs_sample_range(s, 0, n_shots, seed, bits_dev, log2p_dev);
}

rcs_status rcs_sample_batch(const rcs_state* states, int32_t n, uint64_t n_shots, uint64_t seed,
                            uint64_t* bits_dev, double* log2p_dev) {
  RCS_API_BEGIN
  RCS_REQUIRE(states && n >= 0, "bad arguments");
  RCS_REQUIRE(bits_dev || n_shots == 0, "null bits_dev");
  for (int i = 0; i < n; ++i) {
    RCS_REQUIRE(states[i], "null state in batch");
    if (!states[i]->canonical) rcs::fail(RCS_ERR_STATE, "state in batch is not right-canonical");
  }
  std::vector<rcs_state_s*> v(states, states + n);
  rcs::run_chain_batch(v.data(), n, n_shots, seed, bits_dev, log2p_dev, n ? states[0]->stream : nullptr);
  RCS_API_END
}

rcs_status rcs_amplitudes(rcs_state s, const uint64_t* bits_dev, uint64_t m, double* amps_dev) {
  RCS_API_BEGIN
  RCS_REQUIRE(s, "null state");
  RCS_REQUIRE((bits_dev && amps_dev) || m == 0, "null device pointer");
  rcs::run_chain(*s, 0, m, 0, 1, nullptr, nullptr, bits_dev, amps_dev);
  RCS_API_END
}

rcs_status rcs_xeb(int32_t n_qubits, const double* p_ref_dev, uint64_t m, double* xeb_host,
                   double* stderr_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(p_ref_dev && xeb_host && stderr_host, "null argument");
  rcs::xeb_reduce(n_qubits, p_ref_dev, m, false, xeb_host, stderr_host, nullptr);
  RCS_API_END
}

rcs_status rcs_xeb_log2(int32_t n_qubits, const double* log2p_dev, uint64_t m, double* xeb_host,
                        double* stderr_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(log2p_dev && xeb_host && stderr_host, "null argument");
  rcs::xeb_reduce(n_qubits, log2p_dev, m, true, xeb_host, stderr_host, nullptr);
  RCS_API_END
}

}  // extern "C"

extern "C" rcs_status rcs_xeb_state(rcs_state ref, const uint64_t* bits_dev, uint64_t m,
                                    double* xeb_host, double* stderr_host) {
  RCS_API_BEGIN
  RCS_REQUIRE(ref && bits_dev && xeb_host && stderr_host, "null argument");
  rcs::DevBuf amps, p;
  amps.ensure((size_t)m * sizeof(double2));
  p.ensure((size_t)m * sizeof(double));
  rcs::run_chain(*ref, 0, m, 0, 1, nullptr, nullptr, bits_dev, amps.as<double>());
  rcs::abs2_to(amps.as<double2>(), m, p.as<double>(), ref->stream);
  rcs::xeb_reduce(ref->n, p.as<double>(), m, false, xeb_host, stderr_host, ref->stream);
  RCS_API_END
}
