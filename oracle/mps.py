"""Plain CPU matrix-product state along the snake ordering of the grid.

The paper does not describe its engine's state representation (Section 3.2
only says the state is built once and then sampled).  The representation
fixed for this work is an MPS along a boustrophedon ("snake") ordering of
the grid, with the bond dimension capped at chi and SVD truncation.  Every
step below is the plain textbook operation, in complex128 with numpy/LAPACK:

* snake order: row r runs c = 0..W-1 if r is even, W-1..0 if r is odd,
  absent sites skipped; pi[pos] = qubit;
* site tensors A[pos] with shape (chi_left, 2, chi_right), |0...0> initially;
* one-qubit gate: A[pos] <- U on the physical index;
* two-qubit gate on qubits at positions i < j: if j = i+1 one update(i, G);
  otherwise SWAP updates at k = j-1 .. i+1 bring the far qubit next to the
  near one, update(i, G) applies the gate, SWAP updates at k = i+1 .. j-1
  restore the order (the base swap network);
* interleaved network (a second schedule): row-major order with every row
  in the same direction, so each qubit's position is its qubit number.
  Horizontal couplers join neighbouring positions.  For a vertical layer,
  each row pair (r, r+1) of the pattern sits in one contiguous block (row r,
  then row r+1).  The block is sorted by the key 2c for the top qubit of
  column c and 2c+1 for the bottom one, by insertion, and the fSim update of
  a column follows as soon as the moving qubit stops next to its partner.
  The recorded SWAPs are then replayed in reverse order, which restores the
  row-major order.  Cycles alternate direction so that each layer starts
  where the previous one left the orthogonality centre: even cycles take
  their gates and row pairs left to right and sort by moving bottom qubits
  left (in column order); odd cycles go right to left and move top qubits
  right (in reverse column order).  A full row pair costs W^2 updates
  (W(W-1)/2 SWAPs each way plus W gates) against 2W(W-1) + W for the base
  network on the snake order.  On the rotated lattice every layer is made of
  row pairs (the rows holding the layer's couplers), and a bottom qubit's
  key uses its column minus the pair's coupler offset (0, or +-1 for
  down-right couplers), so that it sorts just after its partner;
* update(i, G): move the orthogonality centre into {i, i+1} with exact QR/LQ
  steps; theta = A_i A_{i+1}; theta' = G on (s1, s2); M = theta' as a
  (2 chi_l) x (2 chi_r) matrix with rows (s1, a) and columns (s2, c); SVD;
  rank rule; A_i <- U_k, A_{i+1} <- S_k Vh_k / ||S_k||; centre at i+1;
* rank rule: w = sum s^2; values with s^2 <= 1e-24 w count as exact zeros;
  tail(k) = sum_{r >= k} s_r^2 accumulated from the smallest upward;
  k_eps = min{k >= 1 : tail(k) <= eps w}; k = min(k_eps, chi);
  eps_step = tail(k) / w; log F_est += log(1 - eps_step);
* final: move the centre to position 0 with LQ steps and normalise A[0], so
  the state is right-canonical with unit norm (the form the sampler needs).
"""
import numpy as np

from .circuit import ONE_QUBIT_GATES, SWAP

ZERO_FLOOR = 1e-24


def snake_order(circ):
    order = []
    for r in range(circ.H):
        cols = range(circ.W) if r % 2 == 0 else range(circ.W - 1, -1, -1)
        for c in cols:
            s = r * circ.W + c
            if s in circ.qubit_of_site:
                order.append(circ.qubit_of_site[s])
    return order


NETWORKS = ("snake", "interleaved")


def row_major_order(circ):
    """Every row left to right; qubits are numbered in this order, so the
    position of a qubit is its qubit number."""
    return [q for q in range(circ.n)]


def schedule(circ, network="snake"):
    """(pi, ops): ops are ('1q', gate_idx_per_qubit, t) and
    ('u', i, 'fsim'|'swap', t), t = cycle index of the op."""
    if network == "interleaved":
        return _schedule_interleaved(circ)
    if network != "snake":
        raise ValueError("network is 'snake' or 'interleaved'")
    pi = snake_order(circ)
    pos = {q: p for p, q in enumerate(pi)}
    ops = []
    t = 0
    for kind, data in circ.layers:
        if kind == "1q":
            ops.append(("1q", data, t))
        else:
            pairs = sorted((min(pos[a], pos[b]), max(pos[a], pos[b])) for a, b in data)
            for i, j in pairs:
                for k in range(j - 1, i, -1):
                    ops.append(("u", k, "swap", t))
                ops.append(("u", i, "fsim", t))
                for k in range(i + 1, j):
                    ops.append(("u", k, "swap", t))
            t += 1
    return pi, ops


def _schedule_interleaved(circ):
    pi = row_major_order(circ)
    ops = []
    t = 0
    for kind, data in circ.layers:
        if kind == "1q":
            ops.append(("1q", data, t))
            continue
        letter = circ.pattern[t % len(circ.pattern)]
        right_to_left = (t % 2 == 1)
        if circ.lattice == "rect" and letter in "AB":
            # horizontal neighbours are neighbouring positions
            for a, b in sorted(data, reverse=right_to_left):
                i, j = sorted((pi.index(a), pi.index(b)))
                assert j == i + 1
                ops.append(("u", i, "fsim", t))
        else:
            coupled = set(data)
            if circ.lattice == "rect":
                first_row = 0 if letter == "C" else 1
                row_pairs = list(range(first_row, circ.H - 1, 2))
            else:
                row_pairs = sorted({circ.present[a] // circ.W for a, _ in data})
            if right_to_left:
                row_pairs.reverse()
            for r in row_pairs:
                top = [circ.qubit_of_site[circ.site(r, c)] for c in range(circ.W)
                       if circ.site(r, c) in circ.qubit_of_site]
                bot = [circ.qubit_of_site[circ.site(r + 1, c)] for c in range(circ.W)
                       if circ.site(r + 1, c) in circ.qubit_of_site]
                # column offset of this row pair's couplers (bottom minus top):
                # 0 for vertical couplers, +-1 for the rotated lattice's
                # down-right ones; a bottom qubit sorts just after its partner
                offsets = {circ.present[b] % circ.W - circ.present[a] % circ.W
                           for a, b in data if circ.present[a] // circ.W == r}
                assert len(offsets) <= 1
                delta = offsets.pop() if offsets else 0
                key = {}
                for q in top:
                    key[q] = 2 * (circ.present[q] % circ.W)
                for q in bot:
                    key[q] = 2 * (circ.present[q] % circ.W - delta) + 1
                block = [pi.index(q) for q in top + bot]
                start, end = min(block), max(block)
                swaps = []
                if not right_to_left:
                    for q in bot:                        # column order
                        p = pi.index(q)
                        while p > start and key[pi[p - 1]] > key[q]:
                            ops.append(("u", p - 1, "swap", t))
                            swaps.append(p - 1)
                            pi[p - 1], pi[p] = pi[p], pi[p - 1]
                            p -= 1
                        if p > start and (pi[p - 1], q) in coupled:
                            ops.append(("u", p - 1, "fsim", t))
                else:
                    for q in reversed(top):              # reverse column order
                        p = pi.index(q)
                        while p < end and key[pi[p + 1]] < key[q]:
                            ops.append(("u", p, "swap", t))
                            swaps.append(p)
                            pi[p], pi[p + 1] = pi[p + 1], pi[p]
                            p += 1
                        if p < end and (q, pi[p + 1]) in coupled:
                            ops.append(("u", p, "fsim", t))
                for k in reversed(swaps):
                    ops.append(("u", k, "swap", t))
                    pi[k], pi[k + 1] = pi[k + 1], pi[k]
        t += 1
    return row_major_order(circ), ops


def rank_rule(s, chi, eps, floor=ZERO_FLOOR):
    """Return (k, eps_step, w, tail) for singular values s (descending)."""
    s2 = np.asarray(s, dtype=np.float64) ** 2
    w = float(np.sum(s2))
    s2z = np.where(s2 <= floor * w, 0.0, s2)
    m = len(s2z)
    tail = np.zeros(m + 1)
    tail[:m] = np.cumsum(s2z[::-1])[::-1]          # tail[k] = sum_{r>=k}
    k_eps = m
    for k in range(1, m + 1):
        if tail[k] <= eps * w:
            k_eps = k
            break
    k = min(k_eps, int(chi))
    return k, float(tail[k] / w), w, tail


class MPS:
    def __init__(self, n, pi):
        self.n = n
        self.pi = list(pi)
        self.A = []
        for _ in range(n):
            a = np.zeros((1, 2, 1), dtype=np.complex128)
            a[0, 0, 0] = 1.0
            self.A.append(a)
        self.center = 0
        self.log_fest = 0.0
        self.sum_eps = 0.0
        self.records = []      # one dict per truncating update

    # ---------------------------------------------------------------- gauge
    def _shift_right(self):
        c = self.center
        a = self.A[c]
        cl, _, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl * 2, cr))
        self.A[c] = q.reshape(cl, 2, q.shape[1])
        self.A[c + 1] = np.einsum("xr,rsc->xsc", r, self.A[c + 1])
        self.center = c + 1

    def _shift_left(self):
        c = self.center
        a = self.A[c]
        cl, _, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl, 2 * cr).conj().T)   # a = r^H q^H
        self.A[c] = q.conj().T.reshape(q.shape[1], 2, cr)
        self.A[c - 1] = np.einsum("asb,bx->asx", self.A[c - 1], r.conj().T)
        self.center = c - 1

    def move_center(self, lo, hi):
        while self.center < lo:
            self._shift_right()
        while self.center > hi:
            self._shift_left()

    # ----------------------------------------------------------------- gates
    def apply_1q(self, pos, U):
        self.A[pos] = np.einsum("st,atb->asb", U, self.A[pos])

    def two_site_matrix(self, i, G):
        a, b = self.A[i], self.A[i + 1]
        theta = np.einsum("asb,btc->astc", a, b)
        thetap = np.einsum("xyst,astc->axyc", G.reshape(2, 2, 2, 2), theta)
        cl, cr = a.shape[0], b.shape[2]
        return thetap.transpose(1, 0, 2, 3).reshape(2 * cl, 2 * cr), cl, cr

    def update(self, i, G, chi, eps, tag=None, perturb=None):
        """perturb: None for every reference value; otherwise a function
        applied to the two-site matrix before its SVD, used only to measure
        how strongly a schedule amplifies a small per-step error."""
        self.move_center(i, i + 1)
        M, cl, cr = self.two_site_matrix(i, G)
        if perturb is not None:
            M = perturb(M)
        U, s, Vh = np.linalg.svd(M, full_matrices=False)
        k, eps_step, w, _ = rank_rule(s, chi, eps)
        nk = np.sqrt(np.sum(s[:k] ** 2))
        self.A[i] = U[:, :k].reshape(2, cl, k).transpose(1, 0, 2).copy()
        self.A[i + 1] = ((s[:k, None] * Vh[:k, :]) / nk).reshape(k, 2, cr)
        self.center = i + 1
        self.log_fest += np.log1p(-eps_step)
        self.sum_eps += eps_step
        self.records.append(dict(pos=i, k=k, eps=eps_step, spectrum=s.copy(),
                                 chi_l=cl, chi_r=cr, tag=tag))
        return k, eps_step

    def swap_positions(self, i):
        self.pi[i], self.pi[i + 1] = self.pi[i + 1], self.pi[i]

    def right_canonicalize(self):
        self.move_center(0, 0)
        nrm = np.linalg.norm(self.A[0])
        self.A[0] = self.A[0] / nrm
        return nrm

    # ------------------------------------------------------------- readout
    def bond_dims(self):
        return [a.shape[2] for a in self.A[:-1]]

    def amplitudes(self, bits):
        """psi(b) for uint64 bitstrings (bit q = outcome of qubit q)."""
        bits = np.asarray(bits, dtype=np.uint64)
        v = np.ones((len(bits), 1), dtype=np.complex128)
        for k in range(self.n):
            sel = ((bits >> np.uint64(self.pi[k])) & np.uint64(1)).astype(bool)
            w0 = v @ self.A[k][:, 0, :]
            w1 = v @ self.A[k][:, 1, :]
            v = np.where(sel[:, None], w1, w0)
        return v[:, 0]

    def to_dense(self):
        if self.n > 24:
            raise ValueError("to_dense is for small states")
        t = self.A[0][0]                      # (2, chi)
        for k in range(1, self.n):
            t = np.tensordot(t, self.A[k], axes=([-1], [0]))
        t = t[..., 0]                         # axes: positions 0..n-1
        pos = {q: p for p, q in enumerate(self.pi)}
        perm = [pos[q] for q in range(self.n - 1, -1, -1)]
        return np.transpose(t, perm).reshape(-1)

    def canonical_residual(self):
        """max over sites 1..n-1 of ||sum_s A^s A^s^H - I|| (right-canonical)."""
        worst = 0.0
        for k in range(1, self.n):
            a = self.A[k]
            g = np.einsum("asb,csb->ac", a, a.conj())
            worst = max(worst, float(np.abs(g - np.eye(a.shape[0])).max()))
        return worst


def build(circ, chi, eps, max_ops=None, perturb=None, network="snake"):
    """Run the whole schedule; returns the right-canonical MPS.  `perturb`
    is passed to every truncating update (None: the plain method)."""
    pi, ops = schedule(circ, network)
    st = MPS(circ.n, pi)
    for oi, op in enumerate(ops):
        if max_ops is not None and oi >= max_ops:
            break
        if op[0] == "1q":
            gates = op[1]
            for p in range(st.n):
                st.apply_1q(p, ONE_QUBIT_GATES[int(gates[st.pi[p]])])
        else:
            _, i, kind, t = op
            G = circ.gate2 if kind == "fsim" else SWAP
            st.update(i, G, chi, eps, tag=(oi, t), perturb=perturb)
            if kind == "swap":
                st.swap_positions(i)
    st.right_canonicalize()
    return st
