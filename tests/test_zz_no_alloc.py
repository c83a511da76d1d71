"""The allocation-free sampler entry point against the allocating one.

rcs_sample_range_noalloc keeps its workspace in the library's static
per-device scratch array; its shots must equal rcs_sample_range's bit for
bit (same Philox draws, same fp64 decisions), on two calls in a row on the
same GPU, the second with a smaller input, so that the second call runs on
the array as the first call left it."""
import numpy as np
import pytest

from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _shots(torch, n, fn, **kw):
    bits = torch.zeros(n, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    fn(bits, l2, **kw)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), l2.cpu().numpy()


def test_noalloc_sampler_equals_allocating_sampler(env):
    rcs, torch = env
    # first call: a 30-qubit chi-64 state, 5,000 shots from shot 123 on
    # (several 960+-shot passes would need chi >= 1024; at chi 64 a pass
    # holds all 5,000, so a third call below forces multiple passes)
    big = rcs.State.build(rcs.Circuit(5, 6, 10, 3, network="interleaved"), 64, 1e-10)
    small = rcs.State.build(rcs.Circuit(3, 4, 8, 1), 64, 0.0)
    for st, n, first, seed in ((big, 5000, 123, 77), (small, 700, 0, 5)):
        ref_b, ref_l = _shots(torch, n, st.sample, seed=seed, first_shot=first)
        got_b, got_l = _shots(torch, n, st.sample_noalloc, seed=seed, first_shot=first)
        assert np.array_equal(got_b, ref_b)
        assert np.array_equal(got_l, ref_l)


def test_noalloc_sampler_multi_pass_then_smaller(env):
    """A chi-1024 bond profile needs passes of 960 shots in the 64 MiB array:
    2,500 shots span three passes, bit-exact against the allocating call
    (which uses one pass); then a smaller call on the same array."""
    rcs, torch = env
    from tests import inputs
    n = 24
    dims = [1] + [min(2 ** min(k, n - k), 1024) for k in range(1, n)] + [1]
    A = inputs.random_site_tensors(dims, seed=41)
    from oracle import mps as omps            # canonical form from the oracle (test input only)
    o = omps.MPS(n, list(range(n)))
    o.A = [a.copy() for a in A]
    o.center = n - 1
    o.right_canonicalize()
    st = rcs.State.from_host(dims, list(range(n)), o.A)
    for cnt, first, seed in ((2500, 5, 9), (130, 0, 10)):
        ref_b, ref_l = _shots(torch, cnt, st.sample, seed=seed, first_shot=first)
        got_b, got_l = _shots(torch, cnt, st.sample_noalloc, seed=seed, first_shot=first)
        assert np.array_equal(got_b, ref_b)
        assert np.array_equal(got_l, ref_l)


def test_noalloc_sampler_argument_errors(env):
    rcs, torch = env
    st = rcs.State.build(rcs.Circuit(3, 4, 8, 1), 64, 0.0)
    with pytest.raises(rcs.RcsError) as ei:
        rcs._check(rcs._lib.rcs_sample_range_noalloc(st.h, 0, 10, 1, None, None))
    assert ei.value.status == 1
    bits = torch.zeros(0, dtype=torch.int64, device="cuda")
    st.sample_noalloc(bits, n_shots=0, seed=1)       # zero shots: nothing to do, no error
