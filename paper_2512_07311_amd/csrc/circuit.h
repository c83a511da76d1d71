// Host-side circuit generation and MPS schedule compilation.
#pragma once

#include <array>
#include <complex>
#include <string>
#include <vector>

#include "common.h"

using cplx = std::complex<double>;

struct Op {
  int32_t kind;   // 0 = single-qubit layer, 1 = two-site update
  int32_t arg;    // layer index (kind 0) or left position (kind 1)
  int32_t gate;   // kind 1: 0 = fSim, 1 = SWAP
  int32_t cycle;  // cycle index of the op
};

struct rcs_circuit_s {
  int rows = 0, cols = 0, W = 0, H = 0, n_cycles = 0;
  uint64_t seed = 0;
  std::string pattern;
  double theta = 0, phi = 0;
  bool final_layer = true;
  std::vector<int> removed;            // absent site indices
  std::vector<int> qubit_of_site;      // -1 when absent
  int n = 0;
  std::vector<std::vector<int>> layers_1q;               // gate index per qubit
  std::vector<std::vector<std::pair<int, int>>> layers_2q; // couplers (qubit ids)
  int network = 0;                     // 0 snake, 1 interleaved row pairs
  int lattice = 0;                     // 0 rectangular, 1 rotated (couplers between adjacent rows)
  std::vector<int> snake;              // position -> qubit at the start
  std::vector<Op> ops;
  int n_updates = 0;
  std::array<cplx, 16> fsim;           // row-major 4x4 in |s1 s2>, index 2 s1 + s2
};

namespace rcs {
// Generates geometry, gate draws and the schedule; throws rcs::Error.
void generate_circuit(const rcs_circuit_desc& d, rcs_circuit_s& c);
// 2x2 single-qubit gate matrices, row-major: 0 sqrtX, 1 sqrtY, 2 sqrtW.
const std::array<cplx, 4>& one_qubit_gate(int g);
std::array<cplx, 16> swap_gate();
}  // namespace rcs
