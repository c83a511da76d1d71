"""GPU parity for the 64-circuit batch (batch seed 7: n ~ U{20..40} on
near-square grids, cycles ~ U{8..20}, chi ~ U{64, 128, 256, 512}) on its
eight cheapest circuits, the subset the oracle builds in seconds.  They are
built concurrently by rcs_build_batch with complex64 contractions and fp64
SVD, 50,000 shots each come from the graph-captured grouped sampler, and per
circuit the oracle MPS (same schedule, fp64) scores a sample of the GPU's
shots: the GPU's log2 probabilities, the linear XEB computed from them and
the estimated fidelity must match the oracle's to within the change that
complex64-sized per-step noise makes in the oracle itself (the longer
circuits here amplify a per-step error far beyond its first-order bound)."""
import numpy as np
import pytest

from oracle import circuit as oc, mps
from tests import inputs
from tests.gpu_util import get_rcs, truncated_tolerance, relative_noise, normwise_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def test_batch_per_circuit_against_oracle(env):
    rcs, torch = env
    wl = inputs.WORKLOADS["rcs_batch64_n20to40"]
    batch = inputs.batch_circuits(wl["batch"], seed=wl["batch_seed"], n_lo=wl["n_lo"], n_hi=wl["n_hi"],
                                  cyc_lo=wl["cyc_lo"], cyc_hi=wl["cyc_hi"], chis=wl["chis"])
    # cheapest by the build's leading term: cycles x sites x (saturated bond)^3
    specs = sorted(batch, key=lambda s: s["cycles"] * s["n"] * min(s["chi"], 2 ** (s["n"] // 2)) ** 3)[:8]
    eps, shots, n_check = wl["eps"], wl["shots"], 2_000
    circs = [rcs.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"]) for s in specs]
    states = rcs.State.build_batch(circs, [s["chi"] for s in specs], [eps] * len(specs), contraction="c64")
    bits = torch.zeros(len(states), shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(len(states), shots, dtype=torch.float64, device="cuda")
    rcs.sample_batch(states, shots, 1004, bits, l2)
    torch.cuda.synchronize()
    for i, (s, st) in enumerate(zip(specs, states)):
        oc_ = oc.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"])
        om = mps.build(oc_, s["chi"], eps)
        b = bits[i, :n_check].cpu().numpy().astype(np.uint64)
        assert int((bits[i] >> s["n"]).abs().max().item()) == 0
        amp_or = np.abs(om.amplitudes(b))
        # complex64 contractions err by about 2^-24 sqrt(4 chi) per step; the
        # bar is twice the larger change that per-step noise of that size
        # makes in the oracle itself (two seeded draws), and never below the
        # first-order bound (per-step error times the summed cut conditioning)
        delta = 2.0 ** -24 * np.sqrt(4.0 * s["chi"])
        change, f_change = 0.0, 0.0
        for k in range(2):
            op = mps.build(oc_, s["chi"], eps, perturb=relative_noise(delta, 1000 + 10 * i + k))
            change = max(change, normwise_rel(np.abs(op.amplitudes(b)), amp_or))
            f_change = max(f_change, abs(op.log_fest - om.log_fest))
        bar = max(2e-4, delta * truncated_tolerance(om) / 1e-13, 2.0 * change)
        amp_gpu = np.sqrt(np.exp2(l2[i, :n_check].cpu().numpy()))
        err = np.linalg.norm(amp_gpu - amp_or) / np.linalg.norm(amp_or)
        assert err < bar, (i, s, err, bar)
        x_or = 2.0 ** s["n"] * np.mean(amp_or ** 2) - 1.0
        x_gpu, _ = rcs.xeb_log2(s["n"], l2[i, :n_check].contiguous())
        assert abs(x_gpu - x_or) <= 2.0 * bar * (abs(x_or) + 1.0), (i, x_gpu, x_or)
        f_tol = max(1e-3, 2.0 * f_change)
        assert abs(st.info().log_fidelity_est - om.log_fest) < f_tol, (i, st.info().log_fidelity_est, om.log_fest)
        assert st.info().canonical == 1
