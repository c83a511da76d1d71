"""Parity at the workloads' full sizes on sampled outputs the oracle can
compute one at a time.

* 53 qubits, chi = 1024, build: the GPU runs the 14-cycle schedule to a point
  where the bonds are saturated, exports the (mixed-canonical) state, and
  the oracle applies the next two-site update to that state; the GPU's state
  after the same update must agree on random amplitudes.
* 53 qubits, chi = 1024, sampling: a right-canonical MPS with the chi = 1024
  bond profile (random tensors canonicalised by the oracle) is imported; the
  GPU draws 1,000,000 shots in the benchmark's launch configuration and a
  sample of the shots is recomputed one by one by the oracle sampler.
* 30 qubits (5x6, 14 cycles, chi 256, eps 1e-8): the whole state is built
  on the GPU and compared with the oracle values stored by
  tests/golden/make_rcs30_reference.py (fp64: 1,000 random amplitudes;
  complex64: bond dimensions and estimated fidelity), and 100,000 shots
  are drawn from the complex64 build, a sample of them recomputed by the
  oracle sampler on the exported state.
* 53 qubits at the bond cap 2048: the last 100,000 of 2,500,000 shots from
  a right-canonical MPS with that bond profile, sampled as above.
"""
import json
import os

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


def _rcs30_reference():
    path = os.path.join(os.path.dirname(__file__), "golden", "rcs30_5x6_c14_chi256.json")
    with open(path) as f:
        ref = json.load(f)
    ri = np.asarray(ref["amplitudes_re_im"])
    ref["amplitudes"] = ri[:, 0] + 1j * ri[:, 1]
    ref["bits"] = inputs.random_bitstrings(ref["rows"] * ref["cols"], ref["n_bitstrings"], ref["bitstring_seed"])
    return ref


def _sampled_shot_parity(rcs, torch, g, shots, seed, n_pick):
    """Draws `shots` shots in one call and recomputes a sample of them (the
    first and last few, plus random indices) with the oracle sampler on the
    exported state."""
    o = oracle_state_from(g.to_host())
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(shots, dtype=torch.float64, device="cuda")
    g.sample(bits, l2, seed=seed)
    pick = np.concatenate([np.arange(5), inputs.rng(6).integers(0, shots, n_pick), [shots - 1]])
    gb, gl = bits.cpu().numpy()[pick], l2.cpu().numpy()[pick]
    for idx, b_gpu, l_gpu in zip(pick, gb, gl):
        ob, ol, tight = sample.sample(o, 1, seed, first_shot=int(idx))
        ok, _, _ = compare_shots(np.array([b_gpu]), ob, tight)
        assert ok, "shot %d differs" % idx
        assert abs(l_gpu - ol[0]) < 1e-9
    return bits, l2


@pytest.mark.parametrize("contraction", ["c128", "c64"])
def test_rcs30_full_build_against_stored_oracle(env, contraction):
    """The whole 30-qubit build on the GPU against the stored oracle values.

    This schedule (972 truncations, log F_est -19) amplifies a small error
    made at each truncation roughly linearly and about 1e8-fold: the stored
    file holds the oracle's own change under seeded per-step perturbations of
    relative size delta.  fp64 bar: twice the change at delta = 1e-13 (the
    per-step backward error of an fp64 SVD; twice for the spread between
    noise draws).  complex64 contractions (delta = 2^-24 sqrt(4 chi)) move
    the oracle itself to a different truncated state (normwise change ~0.8),
    so amplitudes are not compared pointwise there: bond dimensions, the
    truncation count and the estimated fidelity are held to the oracle's
    own response instead, and shots drawn from the GPU's state are checked
    bit for bit against the oracle sampler on that state."""
    rcs, torch = env
    ref = _rcs30_reference()
    resp = {("c128" if r["delta"] == 1e-13 else "c64"): r for r in ref["perturbation_response"]}[contraction]
    c = rcs.Circuit(ref["rows"], ref["cols"], ref["cycles"], ref["circuit_seed"])
    g = rcs.State.build(c, ref["chi"], ref["eps"], contraction=contraction)
    inf = g.info()
    assert list(g.layout()[0]) == ref["bond_dims"]
    assert inf.n_truncations == ref["n_truncations"]
    assert inf.canonical == 1
    f_tol = max(1e-6 * abs(ref["log_fidelity_est"]), 2.0 * abs(resp["log_fidelity_change"]))
    assert abs(inf.log_fidelity_est - ref["log_fidelity_est"]) <= f_tol
    if contraction == "c128":
        bits = torch.from_numpy(ref["bits"].astype(np.int64)).cuda()
        amps = torch.zeros(len(bits), 2, dtype=torch.float64, device="cuda")
        g.amplitudes(bits, amps)
        err = normwise_rel(to_complex(amps), ref["amplitudes"])
        assert err < 2.0 * resp["normwise_rel_change"], (err, resp)
    else:
        bits, l2 = _sampled_shot_parity(rcs, torch, g, 100_000, 1002, 10)
        assert int((bits >> 30).abs().max().item()) == 0
        assert torch.isfinite(l2).all()


def _right_canonical_profile(n, chi, seed):
    """Random right-canonical site tensors (dims[k], 2, dims[k+1]) with the
    bond profile min(2^k, 2^(n-k), chi): each site reshaped to a
    dims[k] x 2 dims[k+1] matrix has orthonormal rows.  Rows come from the
    Q factor of a Gaussian matrix; all sites of the saturated middle share
    one Q, each with its own random row phases and column permutation (both
    keep the rows orthonormal), which keeps the set-up to one large QR."""
    g = inputs.rng(seed)
    dims = [1] + [min(2 ** min(k, n - k), chi) for k in range(1, n)] + [1]
    shared = None
    tens = []
    for k in range(n):
        dl, L = dims[k], 2 * dims[k + 1]
        if (dl, L) == (chi, 2 * chi):
            if shared is None:
                shared = np.linalg.qr(g.standard_normal((L, dl)) + 1j * g.standard_normal((L, dl)))[0].conj().T
            phase = np.exp(2j * np.pi * g.random(dl))
            m = (phase[:, None] * shared)[:, g.permutation(L)]
        else:
            m = np.linalg.qr(g.standard_normal((L, dl)) + 1j * g.standard_normal((L, dl)))[0].conj().T
        tens.append(np.ascontiguousarray(m.reshape(dl, 2, dims[k + 1])))
    return dims, tens


def test_chi2048_profile_last_shots_sampled_parity(env):
    """The 20-cycle workload's sampling shape: 53 qubits, bond cap 2048
    (16,384 shots per pass), shot seed 1005, and the last 100,000 of its
    2,500,000 shots drawn as one range; a sample of them is recomputed one by
    one by the oracle sampler on the same tensors."""
    rcs, torch = env
    wl = inputs.WORKLOADS["rcs53_6x9_c20_chi2048"]
    n, chi, total, seed = 53, wl["chi"], wl["shots"], 1005
    dims, tens = _right_canonical_profile(n, chi, seed=19)
    snake = [int(x) for x in inputs.rng(8).permutation(n)]
    g = rcs.State.from_host(dims, snake, tens, canonical=True)
    o = mps.MPS(n, snake)
    o.A = tens
    first, shots = total - 100_000, 100_000
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(shots, dtype=torch.float64, device="cuda")
    g.sample(bits, l2, seed=seed, first_shot=first)
    pick = np.concatenate([np.arange(3), inputs.rng(9).integers(0, shots, 10), [shots - 1]])
    gb, gl = bits.cpu().numpy()[pick], l2.cpu().numpy()[pick]
    for idx, b_gpu, l_gpu in zip(pick, gb, gl):
        ob, ol, tight = sample.sample(o, 1, seed, first_shot=first + int(idx))
        ok, _, _ = compare_shots(np.array([b_gpu]), ob, tight)
        assert ok, "shot %d differs" % (first + idx)
        assert abs(l_gpu - ol[0]) < 1e-9
    assert int((bits >> 53).abs().max().item()) == 0
    assert torch.isfinite(l2).all()
