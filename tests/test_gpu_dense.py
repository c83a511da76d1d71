"""GPU dense state vector (the exact reference for true-fidelity XEB,
Section 5.1) against the oracle's dense simulator, and its use: the true
linear XEB of MPS samples against the exact probabilities."""
import numpy as np
import pytest

from oracle import circuit as oc, dense, sample as osample
from tests import inputs
from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _dense_gpu(rcs, torch, c):
    psi = torch.zeros(1 << c.n, dtype=torch.complex128, device="cuda")
    rcs.dense_simulate(c, psi)
    torch.cuda.synchronize()
    return psi


@pytest.mark.parametrize("rows,cols,cyc,seed,removed", [(3, 4, 8, 1, ()), (2, 3, 5, 2, ()), (4, 5, 10, 3, ()),
                                                        (4, 5, 9, 4, (7,)), (5, 4, 12, 5, (0, 13)),
                                                        (4, 6, 6, 6, (23,))])
def test_dense_matches_oracle(env, rows, cols, cyc, seed, removed):
    """Every amplitude equals the oracle's dense simulation to fp64
    rounding (1e-12 2^(-n/2))."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cyc, seed, removed=removed)
    psi = _dense_gpu(rcs, torch, c).cpu().numpy()
    ref = dense.simulate(oc.Circuit(rows, cols, cyc, seed, removed=list(removed) or None))
    assert np.abs(psi - ref).max() <= 1e-12 * 2.0 ** (-c.n / 2)


@pytest.mark.parametrize("pattern", ["ABCDCDAB", "EFGH"])
def test_dense_rotated_lattice_matches_oracle(env, pattern):
    rcs, torch = env
    c = rcs.Circuit(4, 5, 10, 2, pattern=pattern, removed=(7,), lattice="rotated")
    psi = _dense_gpu(rcs, torch, c).cpu().numpy()
    ref = dense.simulate(oc.Circuit(4, 5, 10, 2, pattern=pattern, removed=[7], lattice="rotated"))
    assert np.abs(psi - ref).max() <= 1e-12 * 2.0 ** (-c.n / 2)


def test_dense_gather(env):
    rcs, torch = env
    c = rcs.Circuit(3, 4, 8, 1)
    psi = _dense_gpu(rcs, torch, c)
    b = inputs.random_bitstrings(c.n, 500, seed=3)
    bits = torch.from_numpy(b.astype(np.int64)).cuda()
    p = torch.zeros(500, dtype=torch.float64, device="cuda")
    a = torch.zeros(500, dtype=torch.complex128, device="cuda")
    rcs.dense_gather(psi, c.n, bits, p, probabilities=True)
    rcs.dense_gather(psi, c.n, bits, a, probabilities=False)
    host = psi.cpu().numpy()
    assert np.array_equal(a.cpu().numpy(), host[b.astype(np.int64)])
    h = host[b.astype(np.int64)]
    assert np.allclose(p.cpu().numpy(), h.real ** 2 + h.imag ** 2, rtol=1e-15, atol=0)


def test_dense_30_qubits_norm_and_porter_thomas(env):
    """30 qubits (16 GiB), beyond the oracle's reach: unit norm to 1e-11 and
    Porter-Thomas statistics of 2^n p (mean 1 exactly, second moment 2)."""
    rcs, torch = env
    c = rcs.Circuit(5, 6, 14, 1, network="interleaved")
    psi = _dense_gpu(rcs, torch, c)
    p = psi.real ** 2 + psi.imag ** 2
    assert abs(float(p.sum()) - 1.0) < 1e-11
    x = p[::64] * float(1 << c.n)
    assert abs(float((x * x).mean()) - 2.0) < 0.02
    del psi, p, x
    torch.cuda.empty_cache()


def test_true_xeb_of_mps_samples(env):
    """Samples of a truncated 20-qubit MPS scored against the exact
    probabilities: the true linear XEB tracks the state's fidelity to the
    exact state (F_true, from all 2^n amplitudes), and so does F_est; exact
    MPS samples score the closed form 2^n sum p^2 - 1 within 5 standard
    errors."""
    rcs, torch = env
    c = rcs.Circuit(4, 5, 12, 7, network="interleaved")
    psi = _dense_gpu(rcs, torch, c)
    n_sh = 200000
    bits = torch.zeros(n_sh, dtype=torch.int64, device="cuda")
    p = torch.zeros(n_sh, dtype=torch.float64, device="cuda")
    for chi, exact in ((1024, True), (384, False)):
        st = rcs.State.build(c, chi, 0.0 if exact else 1e-8)
        st.sample(bits, seed=5)
        rcs.dense_gather(psi, c.n, bits, p, probabilities=True)
        xeb, se = rcs.xeb(c.n, p)
        if exact:
            pp = (psi.real ** 2 + psi.imag ** 2)
            closed = float((pp * pp).sum()) * float(1 << c.n) - 1.0
            assert abs(xeb - closed) < 5 * se
        else:
            allb = torch.arange(1 << c.n, dtype=torch.int64, device="cuda")
            amps = torch.zeros(1 << c.n, 2, dtype=torch.float64, device="cuda")
            st.amplitudes(allb, amps)
            a = torch.view_as_complex(amps)
            f_true = float(abs(torch.vdot(psi, a)) ** 2)
            f_est = float(np.exp(st.info().log_fidelity_est))
            # the oracle's build of this circuit at chi 384: F_true 0.187, F_est 0.187
            assert 0.1 < f_true < 0.3
            assert abs(xeb - f_true) < 0.1 + 5 * se
            assert abs(f_est - f_true) / f_true < 0.1
