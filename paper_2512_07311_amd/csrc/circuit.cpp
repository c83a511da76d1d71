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
// Schedules:
//  * snake (network 0): positions follow rows, even rows left to right, odd
//    rows right to left; a gate on positions i < j becomes SWAP updates at
//    j-1..i+1, the gate update at i, SWAP updates at i+1..j-1;
//  * interleaved (network 1): positions follow rows, every row left to
//    right, so position = qubit number between layers.  A horizontal gate
//    is one update.  A vertical layer handles its row pairs (r, r+1) one at
//    a time: the pair's block (row r then row r+1) is put in the order of
//    the key 2c (top, column c) / 2c+1 (bottom) by insertion, a column's
//    fSim update following as soon as the walking qubit stops beside its
//    partner, and the walk's SWAPs are then replayed last-first to restore
//    the row-major order.  Even cycles run left to right (gates and row
//    pairs in increasing position; bottom qubits, in column order, walk
//    left while the left neighbour's key is larger); odd cycles run right to
//    left (decreasing position; top qubits, in reverse column order, walk
//    right while the right neighbour's key is smaller), so each layer
//    starts where the orthogonality centre was left.  A full row pair is
//    W^2 updates instead of the snake's 2W(W-1) + W.
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

// Interleaved network (see the file header).  `order` tracks which qubit
// sits at each position while a row pair is being sorted.
static void compile_interleaved(rcs_circuit_s& c) {
  const int n = c.n;
  std::vector<int> order(n);
  for (int p = 0; p < n; ++p) order[p] = p;      // row-major numbering
  c.snake = order;
  // column and row of every qubit
  std::vector<int> col_of(n), row_of(n);
  for (int s = 0; s < c.W * c.H; ++s)
    if (c.qubit_of_site[s] >= 0) {
      col_of[c.qubit_of_site[s]] = s % c.W;
      row_of[c.qubit_of_site[s]] = s / c.W;
    }
  for (int t = 0; t < c.n_cycles; ++t) {
    c.ops.push_back(Op{0, t, 0, t});
    const char letter = c.pattern[t % c.pattern.size()];
    const bool leftward = (t % 2) == 1;     // odd cycles run right to left
    const auto& cp = c.layers_2q[t];
    if (c.lattice == 0 && (letter == 'A' || letter == 'B')) {
      std::vector<int> left;
      for (auto& e : cp) {
        const int a = std::min(e.first, e.second), b = std::max(e.first, e.second);
        RCS_REQUIRE(b == a + 1, "horizontal coupler not on neighbouring positions");
        left.push_back(a);
      }
      std::sort(left.begin(), left.end());
      if (leftward) std::reverse(left.begin(), left.end());
      for (int a : left) c.ops.push_back(Op{1, a, 0, t});
      continue;
    }
    // vertical: top qubit -> bottom partner of this layer's couplers
    std::vector<int> partner_above(n, -1);
    for (auto& e : cp) {
      const int a = std::min(e.first, e.second), b = std::max(e.first, e.second);
      partner_above[b] = a;
    }
    std::vector<int> row_pairs;
    if (c.lattice == 0) {
      for (int r = (letter == 'C' ? 0 : 1); r + 1 < c.H; r += 2) row_pairs.push_back(r);
    } else {
      // the rows holding the layer's couplers (as top rows), ascending
      for (auto& e : cp) row_pairs.push_back(row_of[std::min(e.first, e.second)]);
      std::sort(row_pairs.begin(), row_pairs.end());
      row_pairs.erase(std::unique(row_pairs.begin(), row_pairs.end()), row_pairs.end());
    }
    if (leftward) std::reverse(row_pairs.begin(), row_pairs.end());
    for (int r : row_pairs) {
      // column offset (bottom minus top) of this row pair's couplers
      int delta = 0;
      bool have = false;
      for (auto& e : cp) {
        const int a = std::min(e.first, e.second), b = std::max(e.first, e.second);
        if (row_of[a] != r) continue;
        const int dlt = col_of[b] - col_of[a];
        RCS_REQUIRE(!have || dlt == delta, "row pair with mixed coupler offsets");
        delta = dlt;
        have = true;
      }
      // block [lo, hi): the present qubits of rows r and r+1 (contiguous)
      int lo = n, hi = 0;
      for (int q = 0; q < n; ++q)
        if (row_of[q] == r || row_of[q] == r + 1) {
          lo = std::min(lo, q);
          hi = std::max(hi, q + 1);
        }
      if (lo >= hi) continue;
      auto key = [&](int q) { return row_of[q] == r + 1 ? 2 * (col_of[q] - delta) + 1 : 2 * col_of[q]; };
      std::vector<int> walk;                      // SWAP positions, in order
      auto where = [&](int q) { return (int)(std::find(order.begin() + lo, order.begin() + hi, q) - order.begin()); };
      if (!leftward) {
        for (int q = lo; q < hi; ++q) {
          if (row_of[q] != r + 1) continue;       // bottom qubits, column order
          int p = where(q);
          while (p > lo && key(order[p - 1]) > key(q)) {
            c.ops.push_back(Op{1, p - 1, 1, t});
            walk.push_back(p - 1);
            std::swap(order[p - 1], order[p]);
            --p;
          }
          if (p > lo && partner_above[q] >= 0 && order[p - 1] == partner_above[q])
            c.ops.push_back(Op{1, p - 1, 0, t});
        }
      } else {
        for (int q = hi - 1; q >= lo; --q) {
          if (row_of[q] != r) continue;           // top qubits, reverse column order
          int p = where(q);
          while (p + 1 < hi && key(order[p + 1]) < key(q)) {
            c.ops.push_back(Op{1, p, 1, t});
            walk.push_back(p);
            std::swap(order[p], order[p + 1]);
            ++p;
          }
          if (p + 1 < hi && partner_above[order[p + 1]] == q) c.ops.push_back(Op{1, p, 0, t});
        }
      }
      for (auto it = walk.rbegin(); it != walk.rend(); ++it) {
        c.ops.push_back(Op{1, *it, 1, t});
        std::swap(order[*it], order[*it + 1]);
      }
    }
    for (int p = 0; p < n; ++p) RCS_REQUIRE(order[p] == p, "interleaved network did not restore the order");
  }
  if (c.final_layer) c.ops.push_back(Op{0, c.n_cycles, 0, c.n_cycles});
}

void generate_circuit(const rcs_circuit_desc& d, rcs_circuit_s& c) {
  RCS_REQUIRE(d.rows >= 2 && d.cols >= 2, "grid must be at least 2x2");
  RCS_REQUIRE((int64_t)d.rows * d.cols <= 4096, "grid too large");
  RCS_REQUIRE(d.n_cycles >= 0, "n_cycles must be >= 0");
  RCS_REQUIRE(d.n_removed >= 0 && (d.n_removed == 0 || d.removed_sites), "bad removed sites");
  RCS_REQUIRE(d.n_removed_random == 0 || d.n_removed_random == 1,
              "n_removed_random must be 0 or 1");
  RCS_REQUIRE(d.swap_network == 0 || d.swap_network == 1, "swap_network must be 0 or 1");
  c.rows = d.rows;
  c.cols = d.cols;
  c.W = std::min(d.rows, d.cols);
  c.H = std::max(d.rows, d.cols);
  c.n_cycles = d.n_cycles;
  c.seed = d.seed;
  c.pattern = d.pattern ? std::string(d.pattern) : std::string("ABCDCDAB");
  RCS_REQUIRE(!c.pattern.empty(), "empty pattern");
  RCS_REQUIRE(d.lattice == 0 || d.lattice == 1, "lattice must be 0 (rectangular) or 1 (rotated)");
  c.lattice = d.lattice;
  for (char ch : c.pattern)
    RCS_REQUIRE(ch >= 'A' && ch <= (c.lattice == 1 ? 'H' : 'D'),
                c.lattice == 1 ? "pattern letters must be A-H" : "pattern letters must be A-D");
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
    if (c.lattice == 1) {
      // rotated lattice: down-left (r,c)-(r+1,c) for A, B, E, F and
      // down-right (r,c)-(r+1,c+s), s = +1 on even rows, -1 on odd rows, for
      // C, D, G, H; A-D select by row parity, E-H by r minus the coupler
      // chain's column (c, or c-1 for down-right couplers from odd rows)
      const bool down_left = letter == 'A' || letter == 'B' || letter == 'E' || letter == 'F';
      const bool stripes = letter <= 'D';
      const int want = (letter == 'A' || letter == 'C' || letter == 'E' || letter == 'G') ? 0 : 1;
      for (int r = 0; r + 1 < c.H; ++r)
        for (int col = 0; col < c.W; ++col) {
          const int shift = down_left ? 0 : (r % 2 == 0 ? 1 : -1);
          const int col2 = col + shift;
          if (col2 < 0 || col2 >= c.W) continue;
          const int chain = (down_left || r % 2 == 0) ? col : col - 1;
          const int parity = stripes ? (r % 2) : (((r - chain) % 2) + 2) % 2;
          if (parity != want) continue;
          const int a = r * c.W + col, b = (r + 1) * c.W + col2;
          if (c.qubit_of_site[a] >= 0 && c.qubit_of_site[b] >= 0)
            out.emplace_back(c.qubit_of_site[a], c.qubit_of_site[b]);
        }
      return out;
    }
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

  c.ops.clear();
  c.n_updates = 0;
  c.network = d.swap_network;
  if (c.network == 1) {
    compile_interleaved(c);
    for (auto& o : c.ops) c.n_updates += (o.kind == 1);
    return;
  }
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
