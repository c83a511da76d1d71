"""Sycamore-style random circuits on a rectangular grid (oracle side).

The paper (Section 3.1) runs Google's 53-qubit random circuits: cycles of
random single-qubit gates from {sqrt(X), sqrt(Y), sqrt(W)} followed by fSim
two-qubit gates on one of four coupler patterns, in the sequence ABCDCDAB.
Those circuit files are not available, so circuits are generated here from
a seed under these readings:

* grid: W = min(rows, cols) columns, H = max(rows, cols) rows; site (r, c);
  qubits are the present sites numbered in row-major order;
* a seed-chosen removed site (53 = 6x9 - 1): index x0 mod (H*W) of
  Philox(seed; (0, 0, 0, stream 1)); couplers touching it are dropped;
* patterns: A horizontal (r,c)-(r,c+1) with c even, B the same with c odd,
  C vertical (r,c)-(r+1,c) with r even, D the same with r odd;
* single-qubit gates are principal square roots ((1+i)I + (1-i)P)/2 of
  P in {X, Y, W=(X+Y)/sqrt2}; fSim(theta, phi) with theta=pi/2, phi=pi/6;
* gate draws: x = word 0 of Philox(seed; (q, t, 0, stream 0)); at t = 0 the
  gate is floor(3x / 2^32); later the two gates different from the previous
  one on that qubit, in increasing order, indexed by x >> 31;
* cycle t: single-qubit layer on every qubit, then fSim on every coupler of
  pattern[t mod len(pattern)]; after the last cycle one more single-qubit
  layer (drawn at t = n_cycles) when final_layer is set.

A second lattice ("rotated") stands in for Sycamore's rotated square
lattice, where every qubit couples to up to four diagonal neighbours, two in
the row above and two in the row below, and the coupler patterns are
labelled A-H (Section 3.1 runs ABCDCDAB and EFGH).  Google's layout files
are not available, so the lattice and the patterns are a reading:
* couplers join adjacent rows only: "down-left" (r,c)-(r+1,c) and
  "down-right" (r,c)-(r+1,c+s) with s = +1 on even rows and -1 on odd rows,
  so each site has two neighbours below and two above;
* A, B: down-left couplers with r even / odd; C, D: down-right couplers
  with r even / odd (row-parity stripes);
* E, F: down-left couplers with r - c even / odd; G, H: down-right
  couplers with r - ch even / odd, ch = c on even rows and c - 1 on odd
  rows (the column of the coupler's chain: down-right couplers chain
  (r, c) -> (r+1, c+s) -> (r+2, c)), a staggered split;
* every pattern is a matching, A-D and E-H each cover every coupler once.
"""
import math
import numpy as np

from .philox import philox4x32_10, key_of, STREAM_CIRCUIT, STREAM_LAYOUT

_S2 = math.sqrt(2.0)
SQRT_X = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
SQRT_Y = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
SQRT_W = 0.5 * np.array([[1 + 1j, -1j * _S2], [_S2, 1 + 1j]], dtype=np.complex128)
ONE_QUBIT_GATES = (SQRT_X, SQRT_Y, SQRT_W)

SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def fsim(theta, phi):
    """fSim(theta, phi) in the basis |s_a s_b>, index 2*s_a + s_b."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


class Circuit:
    """A generated circuit: grid geometry plus the list of layers.

    layers: list of ('1q', gate_index_per_qubit ndarray[int]) and
            ('2q', list of (qa, qb) couplers).
    """

    def __init__(self, rows, cols, n_cycles, seed, pattern="ABCDCDAB",
                 removed=None, n_removed_random=0, theta=math.pi / 2,
                 phi=math.pi / 6, final_layer=True, lattice="rect"):
        if lattice not in ("rect", "rotated"):
            raise ValueError("lattice is 'rect' or 'rotated'")
        self.lattice = lattice
        self.rows, self.cols = int(rows), int(cols)
        self.W = min(self.rows, self.cols)
        self.H = max(self.rows, self.cols)
        self.n_cycles = int(n_cycles)
        self.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.pattern = pattern
        self.theta, self.phi = float(theta), float(phi)
        self.final_layer = bool(final_layer)
        nsite = self.W * self.H
        removed = set(int(r) for r in (removed or ()))
        if n_removed_random:
            if n_removed_random != 1:
                raise ValueError("only one seed-chosen removed site is defined")
            k0, k1 = key_of(self.seed)
            x0, _, _, _ = philox4x32_10(0, 0, 0, STREAM_LAYOUT, k0, k1)
            removed.add(int(x0) % nsite)
        self.removed = sorted(removed)
        self.present = [s for s in range(nsite) if s not in removed]
        self.qubit_of_site = {s: q for q, s in enumerate(self.present)}
        self.n = len(self.present)
        self.gate2 = fsim(self.theta, self.phi)
        self.layers = self._generate()

    # geometry -----------------------------------------------------------
    def site(self, r, c):
        return r * self.W + c

    def couplers(self, letter):
        """Couplers (qa, qb) of pattern letter, qa < qb as qubit ids."""
        if self.lattice == "rotated":
            return self._rotated_couplers(letter)
        out = []
        for r in range(self.H):
            for c in range(self.W):
                if letter in "AB":
                    if c + 1 >= self.W or (c % 2) != (0 if letter == "A" else 1):
                        continue
                    a, b = self.site(r, c), self.site(r, c + 1)
                elif letter in "CD":
                    if r + 1 >= self.H or (r % 2) != (0 if letter == "C" else 1):
                        continue
                    a, b = self.site(r, c), self.site(r + 1, c)
                else:
                    raise ValueError("pattern letters are A, B, C, D")
                if a in self.qubit_of_site and b in self.qubit_of_site:
                    out.append((self.qubit_of_site[a], self.qubit_of_site[b]))
        return out

    def _rotated_couplers(self, letter):
        if letter not in "ABCDEFGH":
            raise ValueError("rotated-lattice pattern letters are A-H")
        down_left = letter in "ABEF"
        out = []
        for r in range(self.H - 1):
            for c in range(self.W):
                shift = 0 if down_left else (1 if r % 2 == 0 else -1)
                c2 = c + shift
                if not 0 <= c2 < self.W:
                    continue
                if letter in "ABCD":
                    parity = r % 2
                else:
                    chain = c if (down_left or r % 2 == 0) else c - 1
                    parity = (r - chain) % 2
                if parity != (0 if letter in "ACEG" else 1):
                    continue
                a, b = self.site(r, c), self.site(r + 1, c2)
                if a in self.qubit_of_site and b in self.qubit_of_site:
                    out.append((self.qubit_of_site[a], self.qubit_of_site[b]))
        return out

    # gate draws -----------------------------------------------------------
    def _draw_layer(self, t, prev):
        k0, k1 = key_of(self.seed)
        q = np.arange(self.n, dtype=np.uint64)
        x0, _, _, _ = philox4x32_10(q, t, 0, STREAM_CIRCUIT, k0, k1)
        x0 = x0.astype(np.uint64)
        if prev is None:
            return ((x0 * np.uint64(3)) >> np.uint64(32)).astype(np.int64)
        pick = (x0 >> np.uint64(31)).astype(np.int64)       # 0 or 1
        out = np.empty(self.n, dtype=np.int64)
        for i in range(self.n):
            choices = [g for g in range(3) if g != prev[i]]
            out[i] = choices[pick[i]]
        return out

    def _generate(self):
        layers = []
        prev = None
        for t in range(self.n_cycles):
            g = self._draw_layer(t, prev)
            layers.append(("1q", g))
            prev = g
            letter = self.pattern[t % len(self.pattern)]
            layers.append(("2q", self.couplers(letter)))
        if self.final_layer:
            layers.append(("1q", self._draw_layer(self.n_cycles, prev)))
        return layers

    def one_qubit_draws(self):
        """Array [n_layers_1q, n] of gate indices (0 sqrtX, 1 sqrtY, 2 sqrtW)."""
        return np.array([g for kind, g in self.layers if kind == "1q"])


def near_square_grid(n):
    """Grid for a ragged qubit count: R = floor(sqrt n), C = ceil(n / R);
    the last R*C - n sites of the last row (row-major) are absent."""
    R = int(math.isqrt(n))
    C = -(-n // R)
    removed = list(range(n, R * C))
    return R, C, removed
