"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test anchors one oracle function to something other than itself: a
published known-answer vector, a closed form, an independent brute-force
construction, an exact invariant or a library routine it reduces to.
"""
import math
import os

import numpy as np
import pytest

from oracle import philox, circuit, dense, mps, sample, precision, mlp, rsvd
from oracle.circuit import Circuit, SQRT_X, SQRT_Y, SQRT_W, SWAP, fsim
from tests import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
WP = (X + Y) / math.sqrt(2)


# ------------------------------------------------------------------ Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:4], v[4], v[5])
        assert [int(o) for o in out] == v[6:]


def test_u53_range_and_resolution():
    assert philox.u53(0, 0) == 0.0
    assert philox.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # the low 11 bits of the 64-bit word are dropped
    assert philox.u53(0x7FF, 0) == 0.0 and philox.u53(0x800, 0) == 2.0 ** -53


def test_shot_uniform_word_selection():
    k0, k1 = philox.key_of(1234)
    x = philox.philox4x32_10(7, 0, 2, philox.STREAM_SHOTS, k0, k1)
    assert philox.shot_uniform(1234, 7, 4) == philox.u53(x[0], x[1])
    assert philox.shot_uniform(1234, 7, 5) == philox.u53(x[2], x[3])


# ------------------------------------------------------------------- gates
@pytest.mark.parametrize("U,P", [(SQRT_X, X), (SQRT_Y, Y), (SQRT_W, WP)])
def test_sqrt_gates(U, P):
    assert np.abs(U.conj().T @ U - np.eye(2)).max() < 1e-15
    assert np.abs(U @ U - P).max() < 1e-15          # principal square root
    assert abs(abs(U[0, 0]) ** 2 - 0.5) < 1e-15


def test_fsim_identities():
    phi = math.pi / 6
    G = fsim(math.pi / 2, phi)
    assert np.abs(G.conj().T @ G - np.eye(4)).max() < 1e-15
    D = np.diag([1, -1j, -1j, np.exp(-1j * phi)])
    assert np.abs(G @ SWAP - D).max() < 1e-15
    assert np.abs(SWAP @ G - D).max() < 1e-15

    def op_schmidt_rank(g):
        t = g.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
        return int(np.sum(np.linalg.svd(t, compute_uv=False) > 1e-12))
    assert op_schmidt_rank(G) == 4
    assert op_schmidt_rank(SWAP @ G) == 2
    assert op_schmidt_rank(SWAP) == 4
    # fSim is symmetric under exchanging the qubits
    assert np.abs(SWAP @ G @ SWAP - G).max() < 1e-15


# ---------------------------------------------------------------- circuits
def test_generator_rules():
    c = Circuit(6, 9, 20, seed=99, n_removed_random=1)
    assert c.n == 53 and c.W == 6 and c.H == 9 and len(c.removed) == 1
    draws = c.one_qubit_draws()
    assert draws.shape == (21, 53)
    assert np.all(draws[1:] != draws[:-1])            # never repeats
    assert set(np.unique(draws)) == {0, 1, 2}
    for letter in "ABCD":
        cp = c.couplers(letter)
        qs = [q for e in cp for q in e]
        assert len(qs) == len(set(qs))                # a matching
    full = Circuit(6, 9, 1, seed=1)
    assert [len(full.couplers(l)) for l in "ABCD"] == [27, 18, 24, 24]
    # pattern order ABCDCDAB
    seq = [len(d) for k, d in Circuit(3, 4, 8, seed=3).layers if k == "2q"]
    ref = Circuit(3, 4, 1, seed=3)
    assert seq == [len(ref.couplers(l)) for l in "ABCDCDAB"]


def test_removed_site_follows_layout_stream():
    c = Circuit(6, 9, 2, seed=5, n_removed_random=1)
    x0 = philox.philox4x32_10(0, 0, 0, 1, 5, 0)[0]
    assert c.removed == [int(x0) % 54]


def test_first_draw_is_uniform_over_three():
    c = Circuit(20, 20, 1, seed=11)
    g = c.one_qubit_draws()[0]
    counts = np.bincount(g, minlength=3)
    assert counts.min() > 400 / 3 - 4 * math.sqrt(400 * 2 / 9)


# ------------------------------------------------------------------- dense
def _kron_unitary(circ):
    """Brute force: the full 2^n x 2^n unitary as a product of Kronecker
    products (qubit q is the 2^q place value, so it is the q-th factor from
    the right)."""
    n = circ.n
    total = np.eye(1 << n, dtype=complex)
    gates = circuit.ONE_QUBIT_GATES

    def embed1(U, q):
        mats = [np.eye(2)] * n
        mats[n - 1 - q] = U
        out = np.array([[1.0 + 0j]])
        for m_ in mats:
            out = np.kron(out, m_)
        return out

    def embed2(G, qa, qb):
        dim = 1 << n
        out = np.zeros((dim, dim), dtype=complex)
        for i in range(dim):
            sa, sb = (i >> qa) & 1, (i >> qb) & 1
            for ta in range(2):
                for tb in range(2):
                    j = i & ~(1 << qa) & ~(1 << qb) | (ta << qa) | (tb << qb)
                    out[j, i] += G[2 * ta + tb, 2 * sa + sb]
        return out

    for kind, data in circ.layers:
        if kind == "1q":
            for q in range(n):
                total = embed1(gates[int(data[q])], q) @ total
        else:
            for qa, qb in data:
                total = embed2(circ.gate2, qa, qb) @ total
    return total


@pytest.mark.parametrize("rows,cols,cyc,seed", [(2, 3, 4, 1), (2, 2, 8, 7), (3, 2, 5, 3)])
def test_dense_equals_kronecker_brute_force(rows, cols, cyc, seed):
    c = Circuit(rows, cols, cyc, seed=seed)
    psi = dense.simulate(c)
    ref = _kron_unitary(c)[:, 0]
    assert np.abs(psi - ref).max() < 1e-13


def test_first_layer_is_uniform_and_norm_kept():
    c = Circuit(3, 4, 8, seed=2)
    p = dense.probabilities(dense.simulate(c, max_layers=1))
    assert np.abs(p - 2.0 ** -12).max() < 1e-15
    psi = dense.simulate(c)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12


def test_product_distribution_without_two_qubit_layers():
    c = Circuit(2, 3, 3, seed=4, pattern="A")
    c.layers = [l for l in c.layers if l[0] == "1q"]
    p = dense.probabilities(dense.simulate(c))
    per_q = []
    for q in range(c.n):
        v = np.array([1, 0], dtype=complex)
        for kind, g in c.layers:
            v = circuit.ONE_QUBIT_GATES[int(g[q])] @ v
        per_q.append(np.abs(v) ** 2)
    for i in range(1 << c.n):
        ref = np.prod([per_q[q][(i >> q) & 1] for q in range(c.n)])
        assert abs(p[i] - ref) < 1e-15


def test_porter_thomas_n12():
    m2 = []
    for seed in range(1, 17):
        p = dense.probabilities(dense.simulate(Circuit(3, 4, 8, seed=seed)))
        x = (2 ** 12) * p
        assert abs(x.mean() - 1) < 1e-12
        m2.append(np.mean(x * x))
        assert 1.7 <= m2[-1] <= 2.5
        xs = np.sort(x)
        ks = np.max(np.abs(np.arange(1, len(xs) + 1) / len(xs) - (1 - np.exp(-xs))))
        assert ks <= 0.05
    assert 1.9 <= np.mean(m2) <= 2.2


def test_porter_thomas_n20():
    p = dense.probabilities(dense.simulate(Circuit(4, 5, 14, seed=1)))
    x = (2 ** 20) * p
    assert abs(np.mean(x * x) - 2.0) <= 0.02


# --------------------------------------------------------------------- MPS
@pytest.mark.parametrize("rows,cols,cyc,seed,chi", [(3, 4, 8, 1, 64), (3, 4, 8, 5, 64),
                                                    (4, 4, 6, 2, 256), (3, 5, 10, 3, 128)])
def test_exact_mps_equals_dense(rows, cols, cyc, seed, chi):
    c = Circuit(rows, cols, cyc, seed=seed)
    st = mps.build(c, chi, 0.0)
    psi = dense.simulate(c)
    assert np.abs(st.to_dense() - psi).max() <= 1e-12 * 2.0 ** (-c.n / 2)
    assert st.canonical_residual() <= 1e-12
    assert st.log_fest == 0.0
    bits = np.arange(1 << c.n, dtype=np.uint64)
    assert np.abs(st.amplitudes(bits) - psi).max() < 1e-13


def test_removed_site_mps_equals_dense():
    c = Circuit(3, 4, 6, seed=8, n_removed_random=1)
    assert c.n == 11
    st = mps.build(c, 64, 0.0)
    assert np.abs(st.to_dense() - dense.simulate(c)).max() < 1e-13


@pytest.mark.parametrize("rows,cols,cyc,seed,removed", [(3, 4, 8, 1, None), (3, 5, 8, 2, None),
                                                        (4, 4, 9, 3, [6]), (4, 5, 10, 4, [0, 13, 19]),
                                                        (4, 4, 8, 5, [15])])
def test_interleaved_network_exact_mps_equals_dense(rows, cols, cyc, seed, removed):
    """The interleaved swap network builds the same exact state as the
    dense simulator (which knows nothing of MPS positions): a misplaced SWAP
    or gate, or an order left unrestored, would change the amplitudes."""
    c = Circuit(rows, cols, cyc, seed=seed, removed=removed)
    st = mps.build(c, 1 << (c.n // 2), 0.0, network="interleaved")
    psi = dense.simulate(c)
    assert st.pi == list(range(c.n))
    assert np.abs(st.to_dense() - psi).max() <= 1e-12 * 2.0 ** (-c.n / 2)
    assert st.canonical_residual() <= 1e-12


def test_branch_probabilities_add_to_the_prefix_norm():
    """On a right-canonical MPS the two branch probabilities at a site add up
    to the squared norm of the prefix vector, p0 + p1 = ||v||^2, and that
    norm is the marginal probability of the prefix computed from the dense
    state: the identity the GPU sampler uses to decide from W^0 alone.
    Checked on a truncated build along random prefixes; a left-canonical
    site breaks it."""
    c = Circuit(4, 4, 10, seed=6)
    st = mps.build(c, 8, 1e-12)
    assert st.canonical_residual() <= 1e-12
    psi = st.to_dense()
    g = np.random.default_rng(3)
    for _ in range(20):
        v = np.ones(1, dtype=np.complex128)
        prefix = []
        for k in range(st.n):
            w = [v @ st.A[k][:, s, :] for s in (0, 1)]
            p = [float(np.vdot(x, x).real) for x in w]
            assert abs(p[0] + p[1] - float(np.vdot(v, v).real)) <= 1e-12 * max(1.0, float(np.vdot(v, v).real))
            b = int(g.random() < p[1] / (p[0] + p[1]))
            prefix.append(b)
            v = w[b]
            # marginal of the prefix from the dense state (bit q = qubit q)
            idx = np.arange(1 << st.n)
            mask = np.ones(1 << st.n, dtype=bool)
            for kk, bb in enumerate(prefix):
                mask &= ((idx >> st.pi[kk]) & 1) == bb
            marg = float(np.sum(np.abs(psi[mask]) ** 2))
            assert abs(marg - float(np.vdot(v, v).real)) <= 1e-12
    # the same state with its centre moved to the last site: the first
    # sites are then left-canonical (sum_s A^s^H A^s = I), and at site 0 the
    # branch probabilities add up to the bond dimension, not to ||v||^2 = 1
    bad = mps.build(c, 8, 1e-12)
    bad.move_center(bad.n - 1, bad.n - 1)
    w0 = [bad.A[0][:, s, :].ravel() for s in (0, 1)]
    assert abs(sum(float(np.vdot(x, x).real) for x in w0) - bad.A[0].shape[2]) < 1e-12
    assert bad.A[0].shape[2] > 1


def _replay_labels(circ, ops, pi0):
    """Follow the qubit labels through a schedule: the qubit pairs every
    fSim update acts on, per cycle, and the order at each layer's end."""
    pi = list(pi0)
    gates, orders = {}, {}
    for op in ops:
        if op[0] == "1q":
            orders[op[2]] = list(pi)
            continue
        _, i, kind, t = op
        if kind == "fsim":
            gates.setdefault(t, []).append(tuple(sorted((pi[i], pi[i + 1]))))
        else:
            pi[i], pi[i + 1] = pi[i + 1], pi[i]
        orders[t + 1] = list(pi)
    return gates, orders


@pytest.mark.parametrize("rows,cols,cyc,removed", [(6, 9, 14, None), (5, 6, 14, None), (4, 7, 8, [9]),
                                                   (6, 9, 20, [40])])
def test_interleaved_network_gates_counts_and_order(rows, cols, cyc, removed):
    """Each cycle's fSim updates act on exactly that cycle's couplers, once
    each; the row-major order holds at every layer boundary; on a full grid
    the update count is the closed form: per cycle, the horizontal couplers
    of an A/B layer, or W^2 per row pair of a C/D layer."""
    c = Circuit(rows, cols, cyc, seed=11, removed=removed)
    pi, ops = mps.schedule(c, "interleaved")
    gates, orders = _replay_labels(c, ops, pi)
    for t in range(cyc):
        layer = sorted(tuple(sorted(e)) for e in c.layers[2 * t + 1][1])
        assert sorted(gates.get(t, [])) == layer
        assert orders[t + 1] == list(range(c.n))
        # layers alternate direction: the first update of an odd cycle lies
        # right of its last one, the reverse for an even cycle
        pos = [o[1] for o in ops if o[0] == "u" and o[3] == t]
        if len(pos) > 1:
            assert (pos[0] > pos[-1]) if t % 2 else (pos[0] < pos[-1])
    n_upd = sum(1 for o in ops if o[0] == "u")
    if removed is None:
        W, H = c.W, c.H
        expect = 0
        for t in range(cyc):
            letter = c.pattern[t % len(c.pattern)]
            if letter == "A":
                expect += H * (W // 2)
            elif letter == "B":
                expect += H * ((W - 1) // 2)
            else:
                pairs = len(range(0 if letter == "C" else 1, H - 1, 2))
                expect += pairs * W * W
        assert n_upd == expect
    # the base network on the snake order, for comparison: 2W(W-1)+W per row pair
    _, base_ops = mps.schedule(c, "snake")
    assert n_upd < sum(1 for o in base_ops if o[0] == "u")


def test_interleaved_network_53_qubit_counts():
    """The 53-qubit, 14- and 20-cycle circuits (seed 1, one seed-chosen site
    removed): 1,233 and 1,595 updates against 2,113 and 2,695 on the snake."""
    for cyc, n_int, n_snake in ((14, 1233, 2113), (20, 1595, 2695)):
        c = Circuit(6, 9, cyc, seed=1, n_removed_random=1)
        for net, want in (("interleaved", n_int), ("snake", n_snake)):
            assert sum(1 for o in mps.schedule(c, net)[1] if o[0] == "u") == want


def test_rotated_lattice_patterns():
    """Rotated lattice (the Sycamore stand-in): every pattern A-H is a
    matching; A-D and E-H each cover the same couplers, every one once;
    interior sites have two neighbours in the row above and two below, and
    every coupler joins adjacent rows."""
    c = Circuit(6, 9, 1, 1, lattice="rotated")
    nbrs = {q: set() for q in range(c.n)}
    covers = []
    for group in ("ABCD", "EFGH"):
        seen = []
        for letter in group:
            cp = c.couplers(letter)
            qs = [q for e in cp for q in e]
            assert len(qs) == len(set(qs)), letter
            seen += [tuple(sorted(e)) for e in cp]
        assert len(seen) == len(set(seen))
        covers.append(set(seen))
    assert covers[0] == covers[1] and len(covers[0]) == 6 * 8 + 5 * 8
    for a, b in covers[0]:
        ra, rb = c.present[a] // c.W, c.present[b] // c.W
        assert rb == ra + 1 and abs(c.present[b] % c.W - c.present[a] % c.W) <= 1
        nbrs[a].add(b)
        nbrs[b].add(a)
    for r in range(1, c.H - 1):
        for col in range(1, c.W - 1):
            q = c.qubit_of_site[c.site(r, col)]
            rows = sorted(c.present[x] // c.W for x in nbrs[q])
            assert rows == [r - 1, r - 1, r + 1, r + 1]


@pytest.mark.parametrize("network", ["snake", "interleaved"])
@pytest.mark.parametrize("rows,cols,cyc,pattern,removed", [(3, 4, 8, "ABCDCDAB", None), (4, 4, 8, "EFGH", None),
                                                           (4, 4, 10, "ABCDCDAB", [6]), (3, 5, 8, "GHEF", None)])
def test_rotated_lattice_exact_mps_equals_dense(network, rows, cols, cyc, pattern, removed):
    c = Circuit(rows, cols, cyc, seed=3, pattern=pattern, removed=removed, lattice="rotated")
    st = mps.build(c, 1 << (c.n // 2), 0.0, network=network)
    assert np.abs(st.to_dense() - dense.simulate(c)).max() <= 1e-12 * 2.0 ** (-c.n / 2)


@pytest.mark.parametrize("pattern", ["ABCDCDAB", "EFGH"])
def test_rotated_lattice_interleaved_gates_and_order(pattern):
    """Each cycle's fSim updates act on exactly that cycle's couplers, and
    the row-major order holds at every layer boundary (rotated lattice,
    53 qubits)."""
    c = Circuit(6, 9, 14, seed=1, pattern=pattern, n_removed_random=1, lattice="rotated")
    pi, ops = mps.schedule(c, "interleaved")
    gates, orders = _replay_labels(c, ops, pi)
    for t in range(c.n_cycles):
        assert sorted(gates.get(t, [])) == sorted(tuple(sorted(e)) for e in c.layers[2 * t + 1][1])
        assert orders[t + 1] == list(range(c.n))


def test_single_truncation_fidelity_is_one_minus_eps():
    c = Circuit(3, 4, 8, seed=3)
    psi = dense.simulate(c)
    pi, ops = mps.schedule(c)
    # build exactly, then truncate one central bond with a tight cap
    st = mps.build(c, 64, 0.0)
    st.move_center(5, 6)
    M, cl, cr = st.two_site_matrix(5, np.eye(4))
    s = np.linalg.svd(M, compute_uv=False)
    k_cap = 10
    k, eps_step = st.update(5, np.eye(4), k_cap, 0.0)
    assert k == k_cap
    st.right_canonicalize()
    ov = abs(np.vdot(psi, st.to_dense())) ** 2
    assert abs(ov - (1 - eps_step)) < 1e-12
    # Eckart-Young: the discarded weight is the squared tail
    assert abs(eps_step - np.sum(s[k:] ** 2) / np.sum(s ** 2)) < 1e-14


def test_rank_rule_cases():
    s = np.array([3.0, 2.0, 1.0, 1e-3, 1e-13])
    w = np.sum(s ** 2)
    k, e, _, _ = mps.rank_rule(s, 10, 0.0)
    assert k == 4 and e == 0.0               # 1e-26 <= 1e-24 w counts as zero
    k, e, _, _ = mps.rank_rule(s, 10, 1e-7)
    assert k == 3 and abs(e - 1e-6 / w) < 1e-20
    k, e, _, _ = mps.rank_rule(s, 2, 0.0)
    assert k == 2 and abs(e - (1.0 + 1e-6) / w) < 1e-16
    k, e, _, _ = mps.rank_rule(s, 10, 0.5)
    assert k == 1


def test_truncated_fest_tracks_true_fidelity():
    c = Circuit(4, 4, 10, seed=6)
    psi = dense.simulate(c)
    for chi in (8, 16):
        st = mps.build(c, chi, 1e-10)
        f_true = abs(np.vdot(psi, st.to_dense())) ** 2
        f_est = sample.fidelity_estimate(st.log_fest)
        assert f_est < 1.0 and f_true < 1.0
        assert abs(f_true - f_est) / f_est < 0.5


# ----------------------------------------------------------------- sampler
def _dense_sequential_sampler(psi, n, order, seed, n_shots):
    """Independent sampler: marginals summed from the dense distribution."""
    p = dense.probabilities(psi)
    idx = np.arange(1 << n)
    out = []
    for i in range(n_shots):
        mask = np.ones(1 << n, dtype=bool)
        b = 0
        for k, q in enumerate(order):
            sel0 = mask & (((idx >> q) & 1) == 0)
            sel1 = mask & (((idx >> q) & 1) == 1)
            p0, p1 = p[sel0].sum(), p[sel1].sum()
            u = philox.shot_uniform(seed, i, k)
            s = 0 if u * (p0 + p1) < p0 else 1
            mask = sel1 if s else sel0
            b |= s << q
        out.append(b)
    return np.array(out, dtype=np.uint64)


def test_sampler_matches_dense_marginal_sampler():
    c = Circuit(3, 3, 6, seed=12)
    st = mps.build(c, 64, 0.0)
    bits, log2p, tight = sample.sample(st, 200, seed=77)
    ref = _dense_sequential_sampler(dense.simulate(c), c.n, st.pi, 77, 200)
    assert np.all((bits == ref) | (tight >= 0))
    assert np.sum(tight >= 0) == 0
    p = dense.probabilities(dense.simulate(c))[bits.astype(np.int64)]
    assert np.abs(log2p - np.log2(p)).max() < 1e-12


def test_sampler_ghz():
    n = 6
    A = []
    for k in range(n):
        if k == 0:
            a = np.zeros((1, 2, 2), dtype=complex); a[0, 0, 0] = a[0, 1, 1] = 1 / math.sqrt(2)
        elif k == n - 1:
            a = np.zeros((2, 2, 1), dtype=complex); a[0, 0, 0] = a[1, 1, 0] = 1
        else:
            a = np.zeros((2, 2, 2), dtype=complex); a[0, 0, 0] = a[1, 1, 1] = 1
        A.append(a)
    st = mps.MPS(n, list(range(n)))
    st.A = A
    bits, log2p, _ = sample.sample(st, 500, seed=5)
    u0 = philox.shot_uniform(5, np.arange(500, dtype=np.uint64), 0)
    assert np.all(bits == np.where(u0 < 0.5, 0, (1 << n) - 1).astype(np.uint64))
    assert np.abs(log2p + 1).max() < 1e-14


def test_sampler_product_state_bernoulli():
    n = 5
    probs1 = np.array([0.1, 0.3, 0.5, 0.7, 0.9])
    st = mps.MPS(n, [4, 0, 3, 1, 2])
    for k in range(n):
        q = st.pi[k]
        a = np.zeros((1, 2, 1), dtype=complex)
        a[0, 0, 0] = math.sqrt(1 - probs1[q]); a[0, 1, 0] = 1j * math.sqrt(probs1[q])
        st.A[k] = a
    bits, _, _ = sample.sample(st, 20000, seed=9)
    for q in range(n):
        f = np.mean((bits >> np.uint64(q)) & np.uint64(1))
        assert abs(f - probs1[q]) < 4 * math.sqrt(probs1[q] * (1 - probs1[q]) / 20000)


def test_sampler_goodness_of_fit_c1():
    c = Circuit(3, 4, 8, seed=1)
    st = mps.build(c, 64, 0.0)
    p = dense.probabilities(dense.simulate(c))
    bits, _, _ = sample.sample(st, 10000, seed=1001)
    # 20 bins equiprobable under p: sort outcomes by p, cut cumulative mass
    order = np.argsort(p)
    cum = np.cumsum(p[order])
    bin_of = np.empty(len(p), dtype=int)
    bin_of[order] = np.minimum((cum * 20).astype(int), 19)
    expect = np.array([p[bin_of == b].sum() for b in range(20)]) * 10000
    obs = np.bincount(bin_of[bits.astype(np.int64)], minlength=20)
    chi2 = np.sum((obs - expect) ** 2 / expect)
    assert chi2 < 43.8          # chi-square, 19 dof, p = 0.001


# --------------------------------------------------------------------- XEB
def test_xeb_exact_samples_and_uniform():
    c = Circuit(3, 4, 8, seed=4)
    st = mps.build(c, 64, 0.0)
    p = dense.probabilities(dense.simulate(c))
    bits, _, _ = sample.sample(st, 20000, seed=3)
    f, se = sample.linear_xeb(c.n, p[bits.astype(np.int64)])
    assert abs(f - ((2 ** c.n) * np.sum(p * p) - 1)) < 4 * se
    ub = inputs.random_bitstrings(c.n, 20000, seed=8)
    f0, se0 = sample.linear_xeb(c.n, p[ub.astype(np.int64)])
    assert abs(f0) < 4 * se0
    # closed form of the estimator on a fixed sample
    x = (2 ** c.n) * p[bits.astype(np.int64)]
    assert f == pytest.approx(x.sum() / len(x) - 1, abs=1e-12)


# --------------------------------------------------------------- precision
def test_bf16_emulation_matches_torch_rounding():
    torch = pytest.importorskip("torch")
    x = np.concatenate([inputs.random_complex(4096, 3).real.astype(np.float32),
                        np.array([1.0, 1.00390625, 1.01171875, -3.0, 1e-30, 65504.0],
                                 dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(precision.bf16_rne(x), ref)


def test_split_bf16_product_error_bound():
    a = inputs.random_complex((64, 96), 1)
    b = inputs.random_complex((96, 80), 2)
    exact = a.astype(np.complex64).astype(complex) @ b.astype(np.complex64).astype(complex)
    got = precision.matmul_split_bf16_complex(a, b)
    rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    assert rel < 2.0 ** -14
    # dropping the cross terms (plain bf16) is far worse: the split matters
    ah, bh = precision.bf16_rne(a.real.astype(np.float32)), precision.bf16_rne(b.real.astype(np.float32))
    rel_plain = np.linalg.norm(ah.astype(float) @ bh.astype(float) - a.real.astype(np.float32).astype(float) @ b.real.astype(np.float32).astype(float)) \
        / np.linalg.norm(a.real @ b.real)
    assert rel_plain > 50 * rel


# --------------------------------------------------------------------- MLP
def test_mlp_backward_matches_finite_differences():
    flat = inputs.mlp_init(3)
    g = inputs.rng(4)
    x = g.standard_normal((7, 66))
    y = g.standard_normal((7, 32))
    p = mlp.unpack(flat)
    grad = mlp.pack(mlp.backward(p, x, y))
    h = 1e-6
    idx = np.concatenate([np.arange(0, 20), g.integers(0, len(flat), 60),
                          np.arange(len(flat) - 40, len(flat))])
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h; fm[i] -= h
        fd = (mlp.loss(mlp.unpack(fp), x, y) - mlp.loss(mlp.unpack(fm), x, y)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(fd))
    assert mlp.n_params() == 66 * 128 + 128 + 128 * 128 + 128 + 128 * 32 + 32


def test_adam_first_step_closed_form():
    g = inputs.rng(5).standard_normal(100)
    th = inputs.rng(6).standard_normal(100)
    new, m, v = mlp.adam_step(th, g, np.zeros(100), np.zeros(100), 1)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_features_and_targets():
    s = np.array([1.0, 0.1, 0.01, 0.0])
    h = mlp.spectrum_histogram(s[:3])
    # log10 of normalised squares: -0.0043, -2.0043, -4.0043 -> bins 63, 55, 47
    assert h[63] == h[55] == h[47] == pytest.approx(1 / 3) and h.sum() == pytest.approx(1)
    y = mlp.targets(s)
    w = 1.0101
    assert y[7] == pytest.approx(math.log10((0.01 + 1e-4) / w))     # f = 8/32 -> k = 1
    assert y[-1] == -20.0
    assert mlp.predict_rank(y, 4, 64, 1e-3) >= 2


# -------------------------------------------------------------------- RSVD
def test_rsvd_exact_when_sketch_covers_rank():
    M = inputs.planted_matrix(40, 30, np.linspace(2, 0.5, 12), seed=1)
    U, s, Vh = rsvd.rsvd(M, 16, 1, seed=3, step=0)
    s_full = np.linalg.svd(M, compute_uv=False)
    assert np.abs(s[:12] - s_full[:12]).max() < 1e-12
    assert np.linalg.norm(U[:, :12] * s[:12] @ Vh[:12] - M) < 1e-12


def test_rsvd_interlacing_and_hmt_bound():
    spec = 0.9 ** np.arange(60)
    M = inputs.planted_matrix(80, 70, spec, seed=2)
    k, p, q = 10, 6, 1
    U, s, Vh = rsvd.rsvd(M, k + p, q, seed=4, step=1)
    s_full = np.linalg.svd(M, compute_uv=False)
    assert np.all(s <= s_full[:len(s)] + 1e-12)
    fro2 = np.sum(s_full ** 2)
    _, e_rand = rsvd.rsvd_rank(s, fro2, k, 0.0)
    e_full = np.sum(s_full[k:] ** 2) / fro2
    assert e_rand >= e_full - 1e-15
    # HMT (Thm 10.5 / 10.6 style) expected-error bound, generous constant
    err = np.linalg.norm(M - (U[:, :k] * s[:k]) @ Vh[:k], 2)
    bound = (1 + 9 * math.sqrt(k + p) * math.sqrt(min(M.shape))) ** (1 / (2 * q + 1)) * s_full[k]
    assert err <= bound


def test_rsvd_rank_counts_weight_outside_the_sketch():
    """A sketch narrower than the rank leaves weight outside span(Q).  When
    even keeping every sketched direction leaves more than eps of the total,
    no rank meets eps: the rule keeps all l directions (or the cap), and
    the discarded fraction is exactly the weight outside the sketch, never
    zero."""
    s_full = 0.8 ** np.arange(40)
    fro2 = float(np.sum(s_full ** 2))
    s = s_full[:6]                               # an exact 6-column sketch
    outside = float(np.sum(s_full[6:] ** 2)) / fro2
    k, e = rsvd.rsvd_rank(s, fro2, 32, 1e-9)     # cap above the sketch width
    assert k == 6 and abs(e - outside) < 1e-15 and e > 1e-9
    k, e = rsvd.rsvd_rank(s, fro2, 4, 1e-9)      # cap below it
    assert k == 4 and abs(e - float(np.sum(s_full[4:] ** 2)) / fro2) < 1e-15
    # when the sketch holds nearly all the weight, the usual eps rank applies
    k, e = rsvd.rsvd_rank(s_full[:30], fro2, 32, 1e-4)
    assert e <= 1e-4 and k == int(np.argmax(1.0 - np.cumsum(s_full ** 2) / fro2 <= 1e-4)) + 1


def test_sketch_entries_are_unit_phases():
    om = rsvd.sketch(50, 20, seed=9, step=3)
    assert np.all(np.isin(np.round(om, 12), [1, 1j, -1, -1j]))
    k0, k1 = philox.key_of(9)
    x0 = philox.philox4x32_10(17, 5, 3, 4, k0, k1)[0]
    assert om[17, 5] == [1, 1j, -1, -1j][int(x0) & 3]


# ------------------------------------------------- learned-rank decisions
# A prediction that falls by 1/4 decade per knot: y(f) = -8 f exactly
# (knots at f = j/32 with y(0) = 0), so every crossing and every
# interpolated value below is known in closed form.
_Y_LINEAR = np.array([-j / 4.0 for j in range(1, 33)])


def test_predict_rank_hand_worked_cases():
    # crossing exactly on a knot: log10(1e-3) = -3 at f = 12/32, k = 64 * 3/8
    assert mlp.predict_rank(_Y_LINEAR, 64, 64, 1e-3) == 24
    # crossing between knots: -2.9 is 0.6 of the way from y_11 = -2.75 to
    # y_12 = -3, f* = 11.6/32 = 0.3625, k = ceil(100 f*) = ceil(36.25)
    assert mlp.predict_rank(_Y_LINEAR, 100, 100, 10 ** -2.9) == 37
    # the cap clamps, and so does m
    assert mlp.predict_rank(_Y_LINEAR, 100, 20, 10 ** -2.9) == 20
    assert mlp.predict_rank(_Y_LINEAR, 7, 100, 1e-9) == 7
    # first segment interpolates from y(0) = 0: y = -4 at f = 1/32 reaches
    # -2 half-way, f* = 1/64; k = ceil(640 / 64) = 10, and never below 1
    flat4 = np.full(32, -4.0)
    assert mlp.predict_rank(flat4, 640, 640, 1e-2) == 10
    assert mlp.predict_rank(flat4, 64, 64, 1e-2) == 1
    # a prediction that never reaches eps keeps min(cap, m)
    assert mlp.predict_rank(np.full(32, -1.0), 300, 128, 1e-8) == 128
    # eps = 0 aims at 1e-20: not reached by y >= -8, so full rank
    assert mlp.predict_rank(_Y_LINEAR, 50, 64, 0.0) == 50
    # an exact product m f* = integer is not pushed up by rounding
    assert mlp.predict_rank(_Y_LINEAR, 32, 32, 1e-4) == 16


def test_predicted_eps_hand_worked_cases():
    # on the linear prediction 10^y(k/m) = 10^(-8 k/m)
    assert mlp.predicted_eps(_Y_LINEAR, 32, 64) == pytest.approx(1e-4, rel=1e-12)
    assert mlp.predicted_eps(_Y_LINEAR, 64, 64) == pytest.approx(1e-8, rel=1e-12)
    assert mlp.predicted_eps(_Y_LINEAR, 37, 100) == pytest.approx(10 ** -2.96, rel=1e-12)
    # between knots of a non-linear prediction: plain linear interpolation
    y = np.zeros(32)
    y[2], y[3] = -1.0, -5.0                   # knots f = 3/32 and 4/32
    assert mlp.predicted_eps(y, 7, 64) == pytest.approx(10 ** -3.0, rel=1e-12)   # f = 3.5/32
    # first segment from y(0) = 0
    assert mlp.predicted_eps(flat := np.full(32, -4.0), 1, 64) == pytest.approx(10 ** -2.0, rel=1e-12)
    assert flat.shape == (32,)


def test_judge_accepts_threshold_cases():
    tau = 1e-6
    # the threshold is max(eps, eps_pred) + tau, inclusive
    assert rsvd.judge_accepts(1e-8 + tau, 1e-8, 0.0, tau)
    assert not rsvd.judge_accepts(1e-8 + tau + 1e-12, 1e-8, 0.0, tau)
    # a larger prediction raises the bar
    assert rsvd.judge_accepts(1e-3 + tau, 1e-8, 1e-3, tau)
    assert not rsvd.judge_accepts(1e-3 + 2 * tau, 1e-8, 1e-3, tau)
    # tau < 0 rejects everything at or below eps as well
    assert not rsvd.judge_accepts(0.0, 1e-8, 0.0, -1.0)


def test_rsvd_rank_against_brute_force_search():
    """The randomized rank rule is a minimum over k of a monotone condition:
    checked against an exhaustive scan written from the definition."""
    g = inputs.rng(21)
    for trial in range(20):
        l = int(g.integers(1, 40))
        s = np.sort(np.abs(g.standard_normal(l)) * 10.0 ** g.uniform(-6, 0, l))[::-1]
        outside = float(10.0 ** g.uniform(-12, -1))
        fro2 = float(np.sum(s ** 2)) + outside
        eps = float(10.0 ** g.uniform(-9, -1))
        cap = int(g.integers(1, 50))
        ok = [k for k in range(1, l + 1) if fro2 - sum(float(x) ** 2 for x in s[:k]) <= eps * fro2]
        k_ref = min(ok[0] if ok else l, cap)
        e_ref = (fro2 - sum(float(x) ** 2 for x in s[:k_ref])) / fro2
        k, e = rsvd.rsvd_rank(s, fro2, cap, eps)
        assert k == k_ref and e == pytest.approx(e_ref, rel=1e-9, abs=1e-15)


def test_matmul_c64_rounds_inputs_per_element():
    """complex64 emulation: inputs rounded to float32 element by element
    (checked against Python's own IEEE single rounding through struct) and
    products summed exactly; exact when the inputs are float32 numbers."""
    import struct
    g = inputs.rng(22)
    a = g.standard_normal((5, 7)) + 1j * g.standard_normal((5, 7))
    b = g.standard_normal((7, 4)) + 1j * g.standard_normal((7, 4))
    f32 = lambda x: struct.unpack("f", struct.pack("f", x))[0]
    r32 = lambda z: complex(f32(z.real), f32(z.imag))
    ref = np.zeros((5, 4), dtype=np.complex128)
    for i in range(5):
        for j in range(4):
            ref[i, j] = sum(r32(a[i, k]) * r32(b[k, j]) for k in range(7))
    assert np.abs(precision.matmul_c64(a, b) - ref).max() < 1e-14
    # inputs already float32: no rounding at all
    a2 = (g.integers(-64, 64, (6, 3)) + 0.5j * g.integers(-64, 64, (6, 3))).astype(np.complex128)
    b2 = (g.integers(-64, 64, (3, 2)) * 0.25 + 1j * g.integers(-64, 64, (3, 2))).astype(np.complex128)
    assert np.array_equal(precision.matmul_c64(a2, b2), a2 @ b2)
    # and the rounding is visible for values that are not float32 numbers
    assert np.abs(precision.matmul_c64(a, b) - a @ b).max() > 0
