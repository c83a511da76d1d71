"""GPU parity of the fp32 SVD path through the C-ABI.

* The fp32 one-sided Jacobi (rcs_svd_jacobi_f32) against LAPACK's singular
  values and the defining properties of an SVD, at fp32 accuracy, over
  shapes that span several 16-column blocks, ragged tails, wide and tall
  matrices, rank deficiency and the 2048 x 2048 saturated cut.
* Builds with svd_precision="f32" (fp32 Jacobi on the cap-limited splits,
  fp64 Newton-Schulz and projection) against the fp64 build of the same
  circuit: equal kept ranks, estimated fidelity within 1%, and true fidelity
  against the exact state (GPU dense state vector, itself pinned to the
  oracle elsewhere) at least 99% of the fp64 build's.  Where a cut's
  singular values at the cap lie within fp32 accuracy of each other the two
  builds may keep different (equally good) subspaces, after which their
  states part ways while their fidelities do not: the states themselves are
  compared only through fidelity.
* Builds below the cap, where the eps threshold sets every rank: fp32
  attempts are either redone in fp64 or keep every column, and the state
  equals the fp64 build's.
"""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _svd32(rcs, torch, M):
    ln, cnt = M.shape
    x = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    x0 = x.clone()
    s = torch.zeros(cnt, dtype=torch.float64, device="cuda")
    u = torch.zeros(cnt, ln, dtype=torch.complex128, device="cuda")
    rcs.svd_jacobi_f32(x, s, u)
    assert torch.equal(x, x0)                      # the input is not modified
    return s.cpu().numpy(), u.cpu().numpy().T


SHAPES = [(37, 23, "gauss"), (300, 64, "gauss"), (64, 300, "gauss"), (513, 257, "gauss"),
          (256, 256, "decay"), (200, 120, "rank40"), (1, 5, "gauss"), (7, 1, "gauss"),
          (1100, 900, "decay"), (2048, 2048, "decay")]


@pytest.mark.parametrize("ln,cnt,kind", SHAPES)
def test_svd_jacobi_f32(env, ln, cnt, kind):
    rcs, torch = env
    r = min(ln, cnt)
    if kind == "gauss":
        M = inputs.random_complex((ln, cnt), seed=ln * 1000 + cnt + 7)
    elif kind == "decay":
        M = inputs.planted_matrix(ln, cnt, 10.0 ** (-np.linspace(0, 6, r)), seed=5)
    else:
        M = inputs.planted_matrix(ln, cnt, np.linspace(2, 1, 40), seed=6)
    s, U = _svd32(rcs, torch, M)
    s_ref = np.linalg.svd(M, compute_uv=False)
    smax = s_ref[0]
    # singular values: a modest multiple of u32 ||M||_2 sqrt(max(m, n)),
    # plus the drift of the column norms under rotations that are unitary to
    # fp32 rounding (a few u32 per block meeting; a column meets nb - 1
    # blocks per sweep, nb = ceil(cnt / 16), over about ten sweeps)
    nb = -(-cnt // 16)
    bound = max(64 * U32 * np.sqrt(max(ln, cnt)), 8 * U32 * 10 * nb) * smax
    err = np.abs(s[:r] - s_ref).max()
    print("%dx%d %s: max |s - s_ref| / smax = %.2e (bound %.2e)" % (ln, cnt, kind, err / smax, bound / smax))
    assert err <= bound
    assert np.all(s[r:] <= bound)
    assert np.all(np.diff(s) <= 0)
    # the columns of singular values well above the fp32 noise are
    # orthonormal to fp32 accuracy and carry their singular values
    keep = s > 1e-2 * smax
    Uk = U[:, keep]
    assert np.abs(Uk.conj().T @ Uk - np.eye(keep.sum())).max() < 1e-4
    P = Uk.conj().T @ M
    assert np.allclose(np.linalg.norm(P, axis=1), s[keep], rtol=1e-4, atol=bound)
    # what the builds use: the span of the leading half, orthonormalised in
    # fp64, captures the optimal weight of that rank to 1e-6 of the total
    k = max(1, r // 2)
    if k < r:
        Q, _ = np.linalg.qr(U[:, :k])
        captured = np.linalg.norm(Q.conj().T @ M) ** 2
        optimal = np.sum(s_ref[:k] ** 2)
        total = np.sum(s_ref ** 2)
        print("rank %d: captured weight short of the optimum by %.2e of the total" % (k, (optimal - captured) / total))
        assert optimal - captured <= 1e-6 * total


def _all_amps(rcs, torch, st, n):
    bits = torch.arange(1 << n, dtype=torch.int64, device="cuda")
    a = torch.zeros(bits.numel(), dtype=torch.complex128, device="cuda")
    st.amplitudes(bits, a)
    return a.cpu().numpy()


@pytest.mark.parametrize("rows,cols,cycles,chi,seed", [(4, 5, 12, 64, 3), (4, 5, 10, 64, 5), (4, 6, 10, 128, 8)])
def test_build_svd_f32_matches_f64(env, rows, cols, cycles, chi, seed):
    """Cap-limited builds: the fp32 Jacobi takes the saturated splits; the
    kept ranks, the estimated fidelity and the true fidelity against the
    exact state (GPU dense state vector) stay those of the fp64 build."""
    rcs, torch = env
    c = rcs.Circuit(rows, cols, cycles, seed)
    ref = rcs.State.build(c, chi, 1e-10)
    f32 = rcs.State.build(c, chi, 1e-10, svd_precision="f32")
    ir, i32 = ref.info(), f32.info()
    print("n_svd_f32 %d, redone %d, precond %d; log F_est %.10f vs %.10f"
          % (i32.n_svd_f32, i32.n_svd_f32_redone, i32.n_precond, i32.log_fidelity_est, ir.log_fidelity_est))
    assert ir.n_svd_f32 == 0 and ir.n_svd_f32_redone == 0
    assert i32.n_svd_f32 > 0
    assert i32.n_svd_f32 + i32.n_svd_f32_redone <= i32.n_precond + i32.n_precond_fallback
    assert i32.max_bond == ir.max_bond == chi
    k32, k64 = f32.updates()[:, 5], ref.updates()[:, 5]
    print("kept ranks differing: %d of %d" % (int(np.sum(k32 != k64)), len(k64)))
    psi = torch.zeros(1 << c.n, dtype=torch.complex128, device="cuda")
    rcs.dense_simulate(c, psi)
    psi = psi.cpu().numpy()
    a64 = _all_amps(rcs, torch, ref, c.n)
    a32 = _all_amps(rcs, torch, f32, c.n)
    f_true64 = abs(np.vdot(psi, a64)) ** 2
    f_true32 = abs(np.vdot(psi, a32)) ** 2
    mutual = 1.0 - abs(np.vdot(a64, a32)) ** 2
    print("F_est %.6e vs %.6e; F_true %.6e vs %.6e; 1 - |<a64|a32>|^2 = %.3e"
          % (np.exp(i32.log_fidelity_est), np.exp(ir.log_fidelity_est), f_true32, f_true64, mutual))
    assert abs(np.linalg.norm(a32) - 1.0) < 1e-10
    assert abs(i32.log_fidelity_est - ir.log_fidelity_est) <= 1e-2
    assert f_true32 >= 0.99 * f_true64
    # shots drawn from the fp32-SVD state score like the fp64 state's
    sb = torch.zeros(20000, dtype=torch.int64, device="cuda")
    f32.sample(sb, seed=11)
    x32, se = f32.xeb_of(sb)
    x64, _ = ref.xeb_of(sb)
    print("xeb of the same shots: %.6f vs %.6f" % (x32, x64))


def test_build_svd_f32_eps_limited_redone_in_f64(env):
    """Below the cap the eps threshold sets every rank: the fp32 attempts
    whose rank it decides are redone in fp64 (those that keep every column
    with all squared values above 1e-7 of the weight stay, and are exact),
    and the state equals the fp64 build's."""
    rcs, torch = env
    c = rcs.Circuit(3, 5, 8, 12)
    ref = rcs.State.build(c, 2048, 1e-12)
    f32 = rcs.State.build(c, 2048, 1e-12, svd_precision="f32")
    i32 = f32.info()
    print("n_svd_f32 %d, redone %d" % (i32.n_svd_f32, i32.n_svd_f32_redone))
    assert i32.n_svd_f32 + i32.n_svd_f32_redone > 0
    np.testing.assert_array_equal(f32.updates()[:, 5], ref.updates()[:, 5])
    assert i32.log_fidelity_est == pytest.approx(ref.info().log_fidelity_est, abs=1e-12)
    assert np.abs(_all_amps(rcs, torch, f32, c.n) - _all_amps(rcs, torch, ref, c.n)).max() < 1e-10
