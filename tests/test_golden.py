"""Integrity of the stored oracle values for the 30-qubit workload
(tests/golden/rcs30_5x6_c14_chi256.json), against what the mathematics and
the schedule fix without rebuilding the state."""
import json
import os

import numpy as np

from oracle import circuit as oc, mps
from tests import inputs

PATH = os.path.join(os.path.dirname(__file__), "golden", "rcs30_5x6_c14_chi256.json")


def _load():
    with open(PATH) as f:
        return json.load(f)


def test_fixture_describes_the_workload():
    ref = _load()
    wl = inputs.WORKLOADS[ref["workload"]]
    assert (ref["rows"], ref["cols"], ref["cycles"], ref["chi"], ref["eps"]) == (
        wl["rows"], wl["cols"], wl["cycles"], wl["chi"], wl["eps"])
    n = ref["rows"] * ref["cols"]
    assert len(ref["amplitudes_re_im"]) == ref["n_bitstrings"] == 1000
    # a saturated random state: every bond at min(2^k, 2^(n-k), chi)
    assert ref["bond_dims"] == [min(2 ** min(k, n - k), ref["chi"]) for k in range(1, n)]
    # one truncation per two-site update of the schedule
    _, ops = mps.schedule(oc.Circuit(ref["rows"], ref["cols"], ref["cycles"], ref["circuit_seed"]))
    assert ref["n_truncations"] == sum(1 for op in ops if op[0] == "u")


def test_fixture_amplitudes_are_normalised():
    """For any unit-norm state, 2^n |a(x)|^2 at uniformly drawn bitstrings x
    has mean exactly 1 (the sum of all probabilities is 1).  The sample mean
    over the 1,000 stored bitstrings must lie within four standard errors of
    it; a wrong normalisation, a dropped factor or amplitudes of another
    qubit count fail this.  (The truncated state is heavier-tailed than
    Porter-Thomas, so only the mean is fixed.)"""
    ref = _load()
    ri = np.asarray(ref["amplitudes_re_im"])
    p = 2.0 ** (ref["rows"] * ref["cols"]) * (ri[:, 0] ** 2 + ri[:, 1] ** 2)
    assert np.all(np.isfinite(p)) and np.all(p >= 0.0)
    assert abs(p.mean() - 1.0) < 4.0 * p.std(ddof=1) / np.sqrt(len(p))
    assert p.max() > 0.0


def test_fixture_perturbation_response():
    """The recorded responses: delta = 1e-13 and the complex64 size
    2^-24 sqrt(4 chi); a larger per-step error moves the result more, the
    fp64-sized one leaves the estimated fidelity unchanged to 1e-6."""
    ref = _load()
    r = sorted(ref["perturbation_response"], key=lambda x: x["delta"])
    assert [x["delta"] for x in r] == [1e-13, 2.0 ** -24 * np.sqrt(4.0 * ref["chi"])]
    assert 0.0 < r[0]["normwise_rel_change"] < r[1]["normwise_rel_change"] <= 2.0
    assert abs(r[0]["log_fidelity_change"]) < 1e-6 * abs(ref["log_fidelity_est"])
    assert all(x["bond_dims_equal"] for x in r)


def test_perturbation_hook():
    """perturb=None is the plain method bit for bit; on a short exact
    schedule (no truncation, no amplification) noise of relative size 1e-10
    per step moves the state by about that much, and no more than the number
    of steps times it."""
    from tests.gpu_util import relative_noise
    c = oc.Circuit(3, 3, 4, seed=2)
    a = mps.build(c, 64, 0.0)
    b = mps.build(c, 64, 0.0, perturb=None)
    assert all(np.array_equal(x, y) for x, y in zip(a.A, b.A))
    bits = inputs.random_bitstrings(c.n, 200, seed=4)
    ref = a.amplitudes(bits)
    p = mps.build(c, 64, 0.0, perturb=relative_noise(1e-10, 5))
    d = np.linalg.norm(p.amplitudes(bits) - ref) / np.linalg.norm(ref)
    assert 1e-12 < d < 1e-10 * len(p.records)
