"""Parity at the benchmark's full size (53 qubits, chi = 1024) on sampled
outputs the oracle can compute one at a time.

* Build: the GPU runs the 53-qubit 14-cycle schedule to a point where the
  bonds are saturated, exports the (mixed-canonical) state, and the oracle
  applies the next two-site update to that state; the GPU's state after the
  same update must agree on random amplitudes.
* Sampling: a right-canonical MPS with the chi = 1024 bond profile (random
  tensors canonicalised by the oracle) is imported; the GPU draws 1,000,000
  shots in the benchmark's launch configuration and a sample of the shots is
  recomputed one by one by the oracle sampler.
"""
import numpy as np
import pytest

from oracle import circuit as oc, mps, sample
from tests import inputs
from tests.gpu_util import get_rcs, oracle_state_from, compare_shots, to_complex, normwise_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def test_saturated_update_matches_oracle(env):
    rcs, torch = env
    wl = inputs.WORKLOADS["rcs53_6x9_c14_chi1024"]
    c = rcs.Circuit(wl["rows"], wl["cols"], wl["cycles"], 1, n_removed_random=1)
    oc_ = oc.Circuit(wl["rows"], wl["cols"], wl["cycles"], 1, n_removed_random=1)
    _, ops = mps.schedule(oc_)
    # the first two-site update at or after op 560 (bonds are near the cap there)
    N = 560
    while ops[N][0] != "u":
        N += 1
    st_n = rcs.State.build(c, wl["chi"], wl["eps"], max_ops=N, canonicalize=False)
    dims, snake, tens = st_n.to_host()
    assert max(dims) >= 512
    o = oracle_state_from((dims, snake, tens))
    o.center = st_n.info().center
    _, i, kind, t = ops[N]
    G = oc_.gate2 if kind == "fsim" else oc.SWAP
    o.update(i, G, wl["chi"], wl["eps"])
    if kind == "swap":
        o.swap_positions(i)
    g = rcs.State.build(c, wl["chi"], wl["eps"], max_ops=N + 1, canonicalize=False)
    b = inputs.random_bitstrings(c.n, 200, seed=5)
    bits = torch.from_numpy(b.astype(np.int64)).cuda()
    amps = torch.zeros(len(b), 2, dtype=torch.float64, device="cuda")
    g.amplitudes(bits, amps)
    got, ref = to_complex(amps), o.amplitudes(b)
    rec = o.records[-1]
    s, k = rec["spectrum"], rec["k"]
    kappa = s[k - 1] / (s[k - 1] - s[k]) if k < len(s) and s[k - 1] > s[k] else 1.0
    assert normwise_rel(got, ref) < max(1e-10, 1e-13 * kappa)
    assert abs(np.log1p(-rec["eps"]) - (g.info().log_fidelity_est - st_n.info().log_fidelity_est)) < 1e-9


def test_million_shots_sampled_parity(env):
    rcs, torch = env
    n, chi = 53, 1024
    dims = [1] + [min(2 ** min(k, n - k), chi) for k in range(1, n)] + [1]
    A = inputs.random_site_tensors(dims, seed=17)
    o = mps.MPS(n, list(inputs.rng(3).permutation(n)))
    o.A = [a / np.sqrt(a.shape[0]) for a in A]
    o.center = n - 1
    o.right_canonicalize()
    g = rcs.State.from_host(dims, o.pi, o.A, canonical=True)
    shots = 1_000_000
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(shots, dtype=torch.float64, device="cuda")
    g.sample(bits, l2, seed=1003)
    pick = np.concatenate([np.arange(5), inputs.rng(4).integers(0, shots, 10), [shots - 1]])
    gb = bits.cpu().numpy()[pick]
    gl = l2.cpu().numpy()[pick]
    for idx, b_gpu, l_gpu in zip(pick, gb, gl):
        ob, ol, tight = sample.sample(o, 1, 1003, first_shot=int(idx))
        ok, _, _ = compare_shots(np.array([b_gpu]), ob, tight)
        assert ok, "shot %d differs" % idx
        assert abs(l_gpu - ol[0]) < 1e-9
    # every shot is a valid bitstring of 53 qubits with a finite probability
    assert int((bits >> 53).abs().max().item()) == 0
    assert torch.isfinite(l2).all()
