// Circuit generator and schedule compiler (host C++).
//
// Circuit family of the paper's Section 3.1 (Sycamore random circuits: random
// single-qubit gates from {sqrt X, sqrt Y, sqrt W}, fSim on coupler patterns
// in the sequence ABCDCDAB) on a rectangular grid, generated from a seed:
//   * W = min(rows, cols) columns, H = max rows; qubits = present sites in
//     row-major order; one optional seed-chosen absent site: word x of
//     Philox(seed; (0, 0, 0, 1)) mod (H W);
//   * A: (r,c)-(r,c+1), c even; B: c odd; C: (r,c)-(r+1,c), r even; D: r odd;
//   * gate draw for qubit q at layer t: x = word x of Philox(seed; (q,t,0,0));
//     t = 0: floor(3x / 2^32); t > 0: the two gates other than the previous
//     one, in increasing order, indexed by x >> 31.
// Schedule (snake-ordered MPS): positions follow rows, even rows left to
// right, odd rows right to left; a gate on positions i < j becomes SWAP
// updates at j-1..i+1, the gate update at i, SWAP updates at i+1..j-1.
#include "circuit.h"

#include <algorithm>
#include <cmath>

namespace rcs {

const std::array<cplx, 4>& one_qubit_gate(int g) {
  static const double r2 = std::sqrt(2.0);
  static const std::array<cplx, 4> gates[3] = {
      // principal square roots ((1+i) I + (1-i) P) / 2
      {cplx(0.5, 0.5), cplx(0.5, -0.5), cplx(0.5, -0.5), cplx(0.5, 0.5)},      // sqrt X
      {cplx(0.5, 0.5), cplx(-0.5, -0.5), cplx(0.5, 0.5), cplx(0.5, 0.5)},      // sqrt Y
      {cplx(0.5, 0.5), cplx(0.0, -0.5 * r2), cplx(0.5 * r2, 0.0), cplx(0.5, 0.5)}  // sqrt W
  };
  return gates[g];
}

std::array<cplx, 16> swap_gate() {
  std::array<cplx, 16> s{};
  s[0] = s[6] = s[9] = s[15] = 1.0;
  return s;
}

static std::array<cplx, 16> fsim_gate(double theta, double phi) {
  std::array<cplx, 16> g{};
  g[0] = 1.0;
  g[5] = std::cos(theta);
  g[6] = cplx(0.0, -std::sin(theta));
  g[9] = cplx(0.0, -std::sin(theta));
  g[10] = std::cos(theta);
  g[15] = std::polar(1.0, -phi);
  return g;
}

static std::vector<int> draw_layer(uint64_t seed, int n, int t, const std::vector<int>* prev) {
  std::vector<int> out(n);
  for (int q = 0; q < n; ++q) {
    U4 r = philox4x32_10(U4{(uint32_t)q, (uint32_t)t, 0u, kStreamCircuit}, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
    if (!prev) {
      out[q] = (int)(((uint64_t)r.x * 3u) >> 32);
    } else {
      int p = (*prev)[q];
      int pick = (int)(r.x >> 31);
      int choices[2], m = 0;
      for (int g = 0; g < 3; ++g)
        if (g != p) choices[m++] = g;
      out[q] = choices[pick];
    }
  }
  return out;
}

void generate_circuit(const rcs_circuit_desc& d, rcs_circuit_s& c) {
  RCS_REQUIRE(d.rows >= 2 && d.cols >= 2, "grid must be at least 2x2");
  RCS_REQUIRE((int64_t)d.rows * d.cols <= 4096, "grid too large");
  RCS_REQUIRE(d.n_cycles >= 0, "n_cycles must be >= 0");
  RCS_REQUIRE(d.n_removed >= 0 && (d.n_removed == 0 || d.removed_sites), "bad removed sites");
  RCS_REQUIRE(d.n_removed_random == 0 || d.n_removed_random == 1,
              "n_removed_random must be 0 or 1");
  c.rows = d.rows;
  c.cols = d.cols;
  c.W = std::min(d.rows, d.cols);
  c.H = std::max(d.rows, d.cols);
  c.n_cycles = d.n_cycles;
  c.seed = d.seed;
  c.pattern = d.pattern ? std::string(d.pattern) : std::string("ABCDCDAB");
  RCS_REQUIRE(!c.pattern.empty(), "empty pattern");
  for (char ch : c.pattern) RCS_REQUIRE(ch >= 'A' && ch <= 'D', "pattern letters must be A-D");
  c.theta = d.theta;
  c.phi = d.phi;
  c.final_layer = d.final_1q_layer != 0;
  const int nsite = c.W * c.H;
  std::vector<char> absent(nsite, 0);
  for (int i = 0; i < d.n_removed; ++i) {
    int s = d.removed_sites[i];
    RCS_REQUIRE(s >= 0 && s < nsite, "removed site out of range");
    absent[s] = 1;
  }
  if (d.n_removed_random) {
    U4 r = philox4x32_10(U4{0u, 0u, 0u, kStreamLayout}, (uint32_t)c.seed, (uint32_t)(c.seed >> 32));
    absent[r.x % (uint32_t)nsite] = 1;
  }
  c.removed.clear();
  c.qubit_of_site.assign(nsite, -1);
  int n = 0;
  for (int s = 0; s < nsite; ++s) {
    if (absent[s])
      c.removed.push_back(s);
    else
      c.qubit_of_site[s] = n++;
  }
  RCS_REQUIRE(n >= 2 && n <= 64, "number of qubits must be in [2, 64]");
  c.n = n;
  c.fsim = fsim_gate(c.theta, c.phi);

  auto couplers = [&](char letter) {
    std::vector<std::pair<int, int>> out;
    for (int r = 0; r < c.H; ++r)
      for (int col = 0; col < c.W; ++col) {
        int a, b;
        if (letter == 'A' || letter == 'B') {
          if (col + 1 >= c.W || (col & 1) != (letter == 'A' ? 0 : 1)) continue;
          a = r * c.W + col;
          b = r * c.W + col + 1;
        } else {
          if (r + 1 >= c.H || (r & 1) != (letter == 'C' ? 0 : 1)) continue;
          a = r * c.W + col;
          b = (r + 1) * c.W + col;
        }
        if (c.qubit_of_site[a] >= 0 && c.qubit_of_site[b] >= 0)
          out.emplace_back(c.qubit_of_site[a], c.qubit_of_site[b]);
      }
    return out;
  };

  c.layers_1q.clear();
  c.layers_2q.clear();
  const std::vector<int>* prev = nullptr;
  for (int t = 0; t < c.n_cycles; ++t) {
    c.layers_1q.push_back(draw_layer(c.seed, n, t, prev));
    prev = &c.layers_1q.back();
    c.layers_2q.push_back(couplers(c.pattern[t % c.pattern.size()]));
  }
  if (c.final_layer) c.layers_1q.push_back(draw_layer(c.seed, n, c.n_cycles, prev));

  // snake order and schedule
  c.snake.clear();
  for (int r = 0; r < c.H; ++r)
    for (int k = 0; k < c.W; ++k) {
      int col = (r % 2 == 0) ? k : c.W - 1 - k;
      int q = c.qubit_of_site[r * c.W + col];
      if (q >= 0) c.snake.push_back(q);
    }
  std::vector<int> pos(n);
  for (int p = 0; p < n; ++p) pos[c.snake[p]] = p;
  c.ops.clear();
  c.n_updates = 0;
  for (int t = 0; t < c.n_cycles; ++t) {
    c.ops.push_back(Op{0, t, 0, t});
    std::vector<std::pair<int, int>> pr;
    for (auto& e : c.layers_2q[t]) {
      int i = std::min(pos[e.first], pos[e.second]);
      int j = std::max(pos[e.first], pos[e.second]);
      pr.emplace_back(i, j);
    }
    std::sort(pr.begin(), pr.end());
    for (auto& e : pr) {
      int i = e.first, j = e.second;
      for (int k = j - 1; k > i; --k) c.ops.push_back(Op{1, k, 1, t});
      c.ops.push_back(Op{1, i, 0, t});
      for (int k = i + 1; k < j; ++k) c.ops.push_back(Op{1, k, 1, t});
    }
  }
  if (c.final_layer) c.ops.push_back(Op{0, c.n_cycles, 0, c.n_cycles});
  for (auto& o : c.ops) c.n_updates += (o.kind == 1);
}

}  // namespace rcs
