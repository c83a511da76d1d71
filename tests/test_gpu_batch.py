"""GPU parity for the heterogeneous batch at the small-cost end of its
distribution: circuits drawn like the 64-circuit batch (near-square grids,
uneven qubit counts and depths), built concurrently by rcs_build_batch with
complex64 contractions and fp64 SVD, 50,000 shots each from the
graph-captured grouped sampler.  Per circuit, the oracle MPS (same schedule,
fp64) scores a sample of the GPU's shots: the GPU's log2 probabilities, the
linear XEB computed from them and the estimated fidelity must match the
oracle's."""
import numpy as np
import pytest

from oracle import circuit as oc, mps
from tests import inputs
from tests.gpu_util import get_rcs, truncated_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def test_batch_per_circuit_against_oracle(env):
    rcs, torch = env
    specs = inputs.batch_circuits(8, seed=7, n_lo=20, n_hi=24, cyc_lo=8, cyc_hi=10, chis=(64,))
    eps, shots, n_check = 1e-8, 50_000, 2_000
    circs = [rcs.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"]) for s in specs]
    states = rcs.State.build_batch(circs, [s["chi"] for s in specs], [eps] * len(specs), contraction="c64")
    bits = torch.zeros(len(states), shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(len(states), shots, dtype=torch.float64, device="cuda")
    rcs.sample_batch(states, shots, 1004, bits, l2)
    torch.cuda.synchronize()
    for i, (s, st) in enumerate(zip(specs, states)):
        om = mps.build(oc.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"]),
                       s["chi"], eps)
        # complex64 contractions: per-contraction error 2^-24 sqrt(4 chi),
        # amplified by the summed cut conditioning (as for single builds)
        bar = max(2e-4, 2.0 ** -24 * np.sqrt(4.0 * s["chi"]) * truncated_tolerance(om) / 1e-13)
        b = bits[i, :n_check].cpu().numpy().astype(np.uint64)
        assert int((bits[i] >> s["n"]).abs().max().item()) == 0
        amp_or = np.abs(om.amplitudes(b))
        amp_gpu = np.sqrt(np.exp2(l2[i, :n_check].cpu().numpy()))
        err = np.linalg.norm(amp_gpu - amp_or) / np.linalg.norm(amp_or)
        assert err < bar, (i, s, err, bar)
        x_or = 2.0 ** s["n"] * np.mean(amp_or ** 2) - 1.0
        x_gpu, _ = rcs.xeb_log2(s["n"], l2[i, :n_check].contiguous())
        assert abs(x_gpu - x_or) <= 2.0 * bar * (abs(x_or) + 1.0), (i, x_gpu, x_or)
        assert abs(st.info().log_fidelity_est - om.log_fest) < 1e-3, (i, st.info().log_fidelity_est, om.log_fest)
        assert st.info().canonical == 1
