"""GPU parity: state construction through the C-ABI against the dense state
(exact builds) and the oracle MPS on the same schedule (truncated builds)."""
import numpy as np
import pytest

from oracle import circuit as oc, dense, mps, sample
from tests import inputs
from tests.gpu_util import truncated_tolerance, get_rcs, to_complex, normwise_rel, oracle_state_from, compare_shots

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _amps(torch, g, b):
    bits = torch.from_numpy(np.asarray(b).astype(np.int64)).cuda()
    amps = torch.zeros(len(b), 2, dtype=torch.float64, device="cuda")
    g.amplitudes(bits, amps)
    return to_complex(amps)


@pytest.mark.parametrize("rows,cols,cyc,seed", [(3, 4, 8, 1), (3, 4, 8, 7), (4, 4, 8, 2),
                                                (2, 5, 6, 3)])
def test_exact_build_equals_dense(env, rows, cols, cyc, seed):
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed)
    g = rcs.State.build(c, 256, 0.0)
    psi = dense.simulate(oc.Circuit(rows, cols, cyc, seed))
    got = _amps(torch, g, np.arange(1 << c.n))
    # fp64 bar: amplitudes within 1e-10 of the exact state (normwise and
    # elementwise at the typical amplitude size 2^(-n/2))
    assert np.abs(got - psi).max() <= 1e-10 * 2.0 ** (-c.n / 2)
    assert normwise_rel(got, psi) < 1e-10
    inf = g.info()
    assert inf.canonical == 1 and inf.log_fidelity_est == 0.0
    o = oracle_state_from(g.to_host())
    assert o.canonical_residual() < 1e-12
    om = mps.build(oc.Circuit(rows, cols, cyc, seed), 256, 0.0)
    assert list(g.layout()[0]) == om.bond_dims()


@pytest.mark.parametrize("rows,cols,cyc,seed,chi,eps", [(4, 5, 10, 3, 16, 1e-10),
                                                        (3, 6, 12, 4, 12, 0.0),
                                                        (4, 4, 10, 6, 8, 1e-6),
                                                        (3, 7, 14, 8, 33, 1e-9)])
def test_truncated_build_matches_oracle(env, rows, cols, cyc, seed, chi, eps):
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed)
    g = rcs.State.build(c, chi, eps)
    om = mps.build(oc.Circuit(rows, cols, cyc, seed), chi, eps)
    b = inputs.random_bitstrings(c.n, 1000, seed=21)
    got = _amps(torch, g, b)
    ref = om.amplitudes(b)
    assert normwise_rel(got, ref) < truncated_tolerance(om)
    inf = g.info()
    assert abs(inf.log_fidelity_est - om.log_fest) <= 1e-6 * max(1e-300, abs(om.log_fest)) + 1e-14
    assert list(g.layout()[0]) == om.bond_dims()
    assert inf.n_truncations == c.n_updates


@pytest.mark.parametrize("rows,cols,cyc,seed,removed", [(3, 4, 8, 1, ()), (4, 4, 8, 2, ()),
                                                        (4, 5, 9, 3, (7,)), (5, 4, 10, 4, (0, 13))])
def test_interleaved_exact_build_equals_dense(env, rows, cols, cyc, seed, removed):
    """The interleaved swap network on the GPU: exact builds equal the dense
    state to 1e-10 2^(-n/2) elementwise, with the oracle's bond dimensions."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed, removed=removed, network="interleaved")
    oc1 = oc.Circuit(rows, cols, cyc, seed, removed=list(removed) or None)
    g = rcs.State.build(c, 1024, 0.0)
    psi = dense.simulate(oc1)
    got = _amps(torch, g, np.arange(1 << c.n))
    assert np.abs(got - psi).max() <= 1e-10 * 2.0 ** (-c.n / 2)
    om = mps.build(oc1, 1024, 0.0, network="interleaved")
    assert list(g.layout()[0]) == om.bond_dims()
    assert list(g.to_host()[1]) == list(range(c.n))


@pytest.mark.parametrize("rows,cols,cyc,seed,removed,chi,eps", [(4, 5, 10, 3, (), 16, 1e-10),
                                                                (3, 7, 14, 8, (), 33, 1e-9),
                                                                (5, 4, 12, 4, (0,), 12, 1e-8)])
def test_interleaved_truncated_build_matches_oracle(env, rows, cols, cyc, seed, removed, chi, eps):
    """Truncated builds on the interleaved network against the oracle on the
    same schedule: amplitudes within the cut-conditioning bar, equal bond
    dimensions, estimated fidelity to 1e-6 relative."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed, removed=removed, network="interleaved")
    om = mps.build(oc.Circuit(rows, cols, cyc, seed, removed=list(removed) or None), chi, eps,
                   network="interleaved")
    g = rcs.State.build(c, chi, eps)
    b = inputs.random_bitstrings(c.n, 1000, seed=25)
    assert normwise_rel(_amps(torch, g, b), om.amplitudes(b)) < truncated_tolerance(om)
    inf = g.info()
    assert abs(inf.log_fidelity_est - om.log_fest) <= 1e-6 * max(1e-300, abs(om.log_fest)) + 1e-14
    assert list(g.layout()[0]) == om.bond_dims()
    assert inf.n_truncations == c.n_updates


@pytest.mark.parametrize("network", ["snake", "interleaved"])
@pytest.mark.parametrize("rows,cols,cyc,pattern,removed", [(3, 4, 8, "ABCDCDAB", ()), (4, 4, 8, "EFGH", ()),
                                                           (4, 5, 9, "GHEF", (6,))])
def test_rotated_lattice_exact_build_equals_dense(env, network, rows, cols, cyc, pattern, removed):
    """Rotated lattice (patterns A-H): exact GPU builds on both networks equal
    the oracle's dense state to 1e-10 2^(-n/2)."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, 3, pattern=pattern, removed=removed, network=network, lattice="rotated")
    g = rcs.State.build(c, 1024, 0.0)
    psi = dense.simulate(oc.Circuit(rows, cols, cyc, 3, pattern=pattern, removed=list(removed) or None,
                                    lattice="rotated"))
    assert np.abs(_amps(torch, g, np.arange(1 << c.n)) - psi).max() <= 1e-10 * 2.0 ** (-c.n / 2)


@pytest.mark.parametrize("network", ["snake", "interleaved"])
def test_rotated_lattice_truncated_build_matches_oracle(env, network):
    """A truncated rotated-lattice build (EFGH, chi 20) against the oracle
    on the same schedule.  The case is chosen with every cut well separated
    (smallest relative gap at a cut 5.8e-4 on the snake schedule): where a
    cut falls inside an exactly degenerate pair of singular values the
    truncation is not unique and two correct builds part ways."""
    rcs, torch = env
    c = rcs.Circuit(4, 5, 12, 5, pattern="EFGH", network=network, lattice="rotated")
    om = mps.build(oc.Circuit(4, 5, 12, 5, pattern="EFGH", lattice="rotated"), 20, 1e-9, network=network)
    g = rcs.State.build(c, 20, 1e-9)
    b = inputs.random_bitstrings(c.n, 1000, seed=27)
    assert normwise_rel(_amps(torch, g, b), om.amplitudes(b)) < truncated_tolerance(om)
    assert list(g.layout()[0]) == om.bond_dims()
    assert abs(g.info().log_fidelity_est - om.log_fest) <= 1e-6 * abs(om.log_fest) + 1e-14


def test_shots_from_built_state(env):
    rcs, torch = env
    c = rcs.Circuit(4, 5, 10, 11)
    g = rcs.State.build(c, 32, 1e-10)
    o = oracle_state_from(g.to_host())
    bits = torch.zeros(5000, dtype=torch.int64, device="cuda")
    g.sample(bits, seed=4)
    ob, _, tight = sample.sample(o, 5000, 4)
    ok, n_exempt, n_diff = compare_shots(bits.cpu().numpy(), ob, tight)
    assert ok and n_exempt == 0


def test_build_is_deterministic(env):
    rcs, torch = env
    c = rcs.Circuit(4, 5, 8, 13)
    a = rcs.State.build(c, 24, 1e-9).to_host()
    b = rcs.State.build(c, 24, 1e-9).to_host()
    assert all(np.array_equal(x, y) for x, y in zip(a[2], b[2]))


def test_invalid_build_arguments(env):
    rcs, torch = env
    c = rcs.Circuit(3, 3, 2, 1)
    for chi, eps in [(0, 0.0), (64, -1.0), (64, 1.0), (5000, 0.0)]:
        with pytest.raises(rcs.RcsError) as ei:
            rcs.State.build(c, chi, eps)
        assert ei.value.status == 1


@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
@pytest.mark.parametrize("rows,cols,cyc,seed,chi,eps", [(3, 4, 8, 1, 64, 0.0), (4, 5, 10, 3, 16, 1e-10)])
def test_reduced_precision_build_error_budget(env, precision, rows, cols, cyc, seed, chi, eps):
    """complex64 / split-bf16 contractions with fp64 SVD against the fp64
    oracle on the same schedule: 2e-4 (normwise relative) for exact builds;
    truncated builds amplify the contraction error like fp64 round-off, so
    their bar is the per-contraction error times the summed cut
    conditioning.  Per-contraction error: fp32 inner products of length K
    carry about sqrt(K) u32 relative error (probabilistic rounding model),
    K = 4 chi for the two-site contraction, so 2^-24 sqrt(4 chi) for
    complex64; 2^-15 for the three-product bf16 split, whose dropped lo*lo
    term dominates."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed)
    g = rcs.State.build(c, chi, eps, contraction=precision)
    om = mps.build(oc.Circuit(rows, cols, cyc, seed), chi, eps)
    b = inputs.random_bitstrings(c.n, 1000, seed=23)
    err = normwise_rel(_amps(torch, g, b), om.amplitudes(b))
    u = 2.0 ** -24 * np.sqrt(4.0 * chi) if precision == "c64" else 2.0 ** -15
    bar = 2e-4 if eps == 0.0 else max(2e-4, u * truncated_tolerance(om) / 1e-13)
    assert err < bar, (err, bar)
    assert g.info().canonical == 1


@pytest.mark.parametrize("rows,cols,cyc,chi,eps", [
    (8, 8, 2, 2, 0.0),      # 64 qubits: every bit of the uint64 bitstring is used
    (3, 3, 6, 1, 0.0),      # bond cap 1: every cut truncated to a product state
    (2, 3, 0, 8, 0.0),      # no cycles: the final single-qubit layer only
])
def test_build_edge_cases(env, rows, cols, cyc, chi, eps):
    """Degenerate and maximal builds against the oracle MPS: amplitudes on
    random bitstrings, estimated fidelity, and bit-exact shots from the
    built state (high bit included at 64 qubits)."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, 5)
    g = rcs.State.build(c, chi, eps)
    om = mps.build(oc.Circuit(rows, cols, cyc, 5), chi, eps)
    b = inputs.random_bitstrings(c.n, 500, seed=31)
    err = normwise_rel(_amps(torch, g, b), om.amplitudes(b))
    assert err < truncated_tolerance(om), err
    assert abs(g.info().log_fidelity_est - om.log_fest) < 1e-10
    o = oracle_state_from(g.to_host())
    bits = torch.zeros(2000, dtype=torch.int64, device="cuda")
    g.sample(bits, seed=17)
    ob, _, tight = sample.sample(o, 2000, 17)
    ok, n_exempt, _ = compare_shots(bits.cpu().numpy().view(np.uint64), ob, tight)
    assert ok and n_exempt == 0
