"""GPU parity: sampler, amplitudes and XEB through the C-ABI on MPS states
imported from the oracle (same tensors on both sides)."""
import numpy as np
import pytest

from oracle import circuit as oc, dense, mps, sample
from tests import inputs
from tests.gpu_util import get_rcs, to_complex, normwise_rel, oracle_state_from, compare_shots

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _import(rcs, st):
    dims = [1] + st.bond_dims() + [1]
    return rcs.State.from_host(dims, st.pi, st.A)


CASES = {
    "c1_exact": (dict(rows=3, cols=4, n_cycles=8, seed=1), 64, 0.0),
    "4x5_trunc": (dict(rows=4, cols=5, n_cycles=10, seed=3), 16, 1e-10),
    "3x7_trunc": (dict(rows=3, cols=7, n_cycles=12, seed=5), 40, 1e-9),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, env):
    rcs, torch = env
    kw, chi, eps = CASES[request.param]
    c = oc.Circuit(kw["rows"], kw["cols"], kw["n_cycles"], kw["seed"])
    st = mps.build(c, chi, eps)
    return request.param, c, st, _import(rcs, st)


def test_shots_bit_exact(env, case):
    rcs, torch = env
    name, c, st, g = case
    n = 10_000 if name == "c1_exact" else 3_000 + 37     # ragged tails
    bits = torch.zeros(n, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    g.sample(bits, l2, seed=1001)
    ob, ol2, tight = sample.sample(st, n, 1001)
    ok, n_exempt, n_diff = compare_shots(bits.cpu().numpy(), ob, tight)
    assert ok, "%d shots differ" % n_diff
    assert n_exempt == 0
    assert np.abs(l2.cpu().numpy() - ol2).max() < 1e-10


def test_shot_ranges_concatenate(env, case):
    rcs, torch = env
    name, c, st, g = case
    full = torch.zeros(700, dtype=torch.int64, device="cuda")
    g.sample(full, seed=77)
    parts = []
    for a, b in [(0, 1), (1, 64), (64, 333), (333, 700)]:
        t = torch.zeros(b - a, dtype=torch.int64, device="cuda")
        g.sample(t, seed=77, first_shot=a)
        parts.append(t)
    assert torch.equal(torch.cat(parts), full)


def test_amplitudes(env, case):
    rcs, torch = env
    name, c, st, g = case
    m = 1000 + 13
    b = inputs.random_bitstrings(c.n, m, seed=11)
    bits = torch.from_numpy(b.astype(np.int64)).cuda()
    amps = torch.zeros(m, 2, dtype=torch.float64, device="cuda")
    g.amplitudes(bits, amps)
    ref = st.amplitudes(b)
    assert normwise_rel(to_complex(amps), ref) < 1e-12


def test_xeb(env, case):
    rcs, torch = env
    name, c, st, g = case
    n = 4000
    bits = torch.zeros(n, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    g.sample(bits, l2, seed=5)
    ob, ol2, _ = sample.sample(st, n, 5)
    p = np.exp2(ol2)
    f_ref, se_ref = sample.linear_xeb(c.n, p)
    f, se = rcs.xeb_log2(c.n, l2)
    assert abs(f - f_ref) < 1e-10 and abs(se - se_ref) < 1e-10
    f2, se2 = rcs.xeb(c.n, torch.from_numpy(p).cuda())
    assert abs(f2 - f_ref) < 1e-12 and abs(se2 - se_ref) < 1e-12
    f3, se3 = g.xeb_of(bits)
    assert abs(f3 - f_ref) < 1e-10


def test_exact_state_probabilities(env):
    rcs, torch = env
    c = oc.Circuit(3, 4, 8, seed=2)
    st = mps.build(c, 64, 0.0)
    g = _import(rcs, st)
    bits = torch.arange(4096, dtype=torch.int64, device="cuda")
    amps = torch.zeros(4096, 2, dtype=torch.float64, device="cuda")
    g.amplitudes(bits, amps)
    psi = dense.simulate(c)
    assert np.abs(to_complex(amps) - psi).max() < 1e-13


def test_edge_cases(env):
    rcs, torch = env
    c = oc.Circuit(2, 2, 3, seed=9)
    st = mps.build(c, 4, 0.0)
    g = _import(rcs, st)
    one = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.sample(one, seed=3)
    ob, _, _ = sample.sample(st, 1, 3)
    assert int(one.item()) == int(ob[0])
    empty = torch.zeros(0, dtype=torch.int64, device="cuda")
    g.sample(empty, seed=3)      # no-op
    with pytest.raises(rcs.RcsError):
        rcs.State.from_host([1, 3, 1], [0, 1], [np.zeros((1, 2, 3)), np.zeros((3, 2, 1))])
    with pytest.raises(rcs.RcsError):
        rcs.State.from_host([1, 2, 1], [0, 0], [np.zeros((1, 2, 2)), np.zeros((2, 2, 1))])


def test_batch_build_and_graph_sampler(env):
    """Batched build equals per-circuit builds; the graph-captured grouped
    sampler equals per-state sampling bit for bit, on two calls in a row with
    eager work in between."""
    rcs, torch = env
    specs = inputs.batch_circuits(5, seed=7, n_lo=8, n_hi=14, cyc_lo=4, cyc_hi=8, chis=(8, 16, 32))
    circs = [rcs.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"]) for s in specs]
    chis = [s["chi"] for s in specs]
    states = rcs.State.build_batch(circs, chis, [1e-10] * len(circs))
    for c, chi, st in zip(circs, chis, states):
        ref = rcs.State.build(c, chi, 1e-10).to_host()
        got = st.to_host()
        assert all(np.array_equal(x, y) for x, y in zip(ref[2], got[2]))
    n_shots = 1000 + 17
    eager = torch.zeros(len(states), n_shots, dtype=torch.int64, device="cuda")
    eager_l = torch.zeros(len(states), n_shots, dtype=torch.float64, device="cuda")
    for i, st in enumerate(states):
        b = torch.zeros(n_shots, dtype=torch.int64, device="cuda")
        l2 = torch.zeros(n_shots, dtype=torch.float64, device="cuda")
        st.sample(b, l2, seed=99)
        eager[i] = b
        eager_l[i] = l2
    for rep in range(2):
        bits = torch.zeros(len(states), n_shots, dtype=torch.int64, device="cuda")
        l2 = torch.zeros(len(states), n_shots, dtype=torch.float64, device="cuda")
        rcs.sample_batch(states, n_shots, 99, bits, l2)
        torch.cuda.synchronize()
        assert torch.equal(bits, eager)
        assert torch.equal(l2, eager_l)
        _ = (eager.float() * 2).sum().item()      # eager work between calls
