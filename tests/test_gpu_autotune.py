"""GPU test of the Jacobi autotuner through the C-ABI: the tuned table picks
the fastest measured candidate per bucket, round-trips through its JSON
cache, every candidate setting computes a correct SVD (LAPACK's singular
values), and a build under the loaded table equals, bit for bit, a build
under the same settings registered by hand."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu

CANDIDATES = [(16, 1), (16, 2), (32, 1)]


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _amps(torch, st, n):
    bits = torch.arange(1 << n, dtype=torch.int64, device="cuda")
    a = torch.zeros(bits.numel(), dtype=torch.complex128, device="cuda")
    st.amplitudes(bits, a)
    return a.cpu().numpy()


def test_every_candidate_gives_a_correct_svd(env):
    rcs, torch = env
    M = inputs.planted_matrix(150, 130, 10.0 ** (-np.linspace(0, 8, 130)), seed=21)
    s_ref = np.linalg.svd(M, compute_uv=False)
    try:
        for block, inner in CANDIDATES:
            rcs.tuning_clear()
            rcs.tuning_set(1 << 30, block, inner)
            x = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
            s = torch.zeros(130, dtype=torch.float64, device="cuda")
            u = torch.zeros(130, 150, dtype=torch.complex128, device="cuda")
            rcs.svd_jacobi(x, s, u)
            err = np.abs(s.cpu().numpy() - s_ref).max()
            assert err <= 1e-13 * s_ref[0] * np.sqrt(150), (block, inner, err)
    finally:
        rcs.tuning_clear()


def test_tuned_table_roundtrip_and_bitwise_builds(env, tmp_path):
    rcs, torch = env
    from paper_2512_07311_amd import autotune
    try:
        table = autotune.tune(torch, buckets=(64, 128), candidates=CANDIDATES, max_n=128, reps=1)
        assert [e["cnt_max"] for e in table] == [64, 128]
        for e in table:
            assert (e["block"], e["inner"]) in CANDIDATES
            assert e["seconds"] == min(e["candidates"].values())
            assert e["candidates"]["%d/%d" % (e["block"], e["inner"])] == e["seconds"]
        path = tmp_path / "tuning.json"
        autotune.save(str(path), table, torch)
        rcs.tuning_clear()
        assert autotune.load(str(path), torch)
        c = rcs.Circuit(3, 5, 8, 4)
        a_loaded = _amps(torch, rcs.State.build(c, 64, 1e-10), c.n)
        rcs.tuning_clear()
        for e in table:
            rcs.tuning_set(e["cnt_max"], e["block"], e["inner"])
        a_hand = _amps(torch, rcs.State.build(c, 64, 1e-10), c.n)
        assert np.array_equal(a_loaded, a_hand)
        # an unknown architecture key loads nothing
        other = tmp_path / "other.json"
        other.write_text('{"gfx000": []}')
        assert not autotune.load(str(other), torch)
    finally:
        rcs.tuning_clear()
