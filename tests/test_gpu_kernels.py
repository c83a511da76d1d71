"""GPU parity of the stage-level kernels through the C-ABI: the fp64
one-sided Jacobi SVD against the defining properties of an SVD and LAPACK,
the centre moves' QR against LAPACK's, and the two-site contraction against
the oracle's definition."""
import numpy as np
import pytest

from oracle import circuit as oc, mps
from tests import inputs
from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _svd_gpu(rcs, torch, M):
    ln, cnt = M.shape
    x = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()          # columns contiguous
    s = torch.zeros(cnt, dtype=torch.float64, device="cuda")
    u = torch.zeros(cnt, ln, dtype=torch.complex128, device="cuda")
    rcs.svd_jacobi(x, s, u)
    return s.cpu().numpy(), u.cpu().numpy().T


# up to the shapes of saturated cuts: 2 chi x 2 chi at chi = 1024 and at the
# largest cap, chi = 2048 (4096 columns, the widest the rank kernel takes)
SHAPES = [(37, 23, "gauss"), (100, 100, "gauss"), (300, 64, "gauss"), (64, 300, "gauss"),
          (513, 257, "gauss"), (256, 256, "decay"), (200, 120, "rank40"), (1, 5, "gauss"),
          (7, 1, "gauss"), (2048, 2048, "decay"), (4096, 700, "gauss"), (700, 4096, "gauss"),
          (4096, 4096, "decay")]


@pytest.mark.parametrize("ln,cnt,kind", SHAPES)
def test_svd_jacobi(env, ln, cnt, kind):
    rcs, torch = env
    r = min(ln, cnt)
    if kind == "gauss":
        M = inputs.random_complex((ln, cnt), seed=ln * 1000 + cnt)
    elif kind == "decay":
        M = inputs.planted_matrix(ln, cnt, 10.0 ** (-np.linspace(0, 12, r)), seed=3)
    else:
        M = inputs.planted_matrix(ln, cnt, np.linspace(2, 1, 40), seed=4)
    s, U = _svd_gpu(rcs, torch, M)
    s_ref = np.linalg.svd(M, compute_uv=False)
    smax = s_ref[0]
    # singular values: absolute accuracy of an fp64 SVD
    assert np.abs(s[:r] - s_ref).max() <= 1e-13 * smax * np.sqrt(max(ln, cnt))
    assert np.all(s[r:] <= 1e-13 * smax * np.sqrt(max(ln, cnt)))
    assert np.all(np.diff(s) <= 0)
    keep = s > 1e-10 * smax
    Uk = U[:, keep]
    # the kept columns are orthonormal and span the dominant left subspace
    assert np.abs(Uk.conj().T @ Uk - np.eye(keep.sum())).max() < 1e-9
    P = Uk.conj().T @ M
    assert np.allclose(np.linalg.norm(P, axis=1), s[keep], rtol=1e-9, atol=1e-13 * smax)
    resid = M - Uk @ P
    assert np.linalg.norm(resid) <= 1e-10 * smax * np.sqrt(cnt) + np.sqrt(np.sum(s_ref[keep.sum():] ** 2)) * 1.0001


def test_two_site_contraction(env):
    rcs, torch = env
    g = inputs.rng(5)
    for dl, dm, dr in [(1, 2, 1), (3, 5, 7), (64, 65, 63), (130, 70, 96)]:
        A = g.standard_normal((dl, 2, dm)) + 1j * g.standard_normal((dl, 2, dm))
        B = g.standard_normal((dm, 2, dr)) + 1j * g.standard_normal((dm, 2, dr))
        G = oc.fsim(np.pi / 2, np.pi / 6)
        st = mps.MPS(2, [0, 1])
        st.A = [A, B]
        ref, _, _ = st.two_site_matrix(0, G)
        out = torch.zeros(2 * dr, 2 * dl, dtype=torch.complex128, device="cuda")
        rcs.two_site(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), G, out)
        got = out.cpu().numpy().T
        assert np.abs(got - ref).max() <= 1e-14 * np.sqrt(dm) * np.abs(ref).max()


@pytest.mark.parametrize("precision", ["c64", "split_bf16"])
def test_two_site_reduced_precision(env, precision):
    """Reduced-precision contraction against the oracle's exact emulation of
    the same rounding (complex64 inputs / three-product bf16 split), to
    within fp32 accumulation-order noise."""
    from oracle import precision as prec
    rcs, torch = env
    g = inputs.rng(9)
    G = oc.fsim(np.pi / 2, np.pi / 6)
    G4 = G.reshape(2, 2, 2, 2)
    for dl, dm, dr in [(3, 5, 7), (64, 65, 63), (100, 130, 90)]:
        A = g.standard_normal((dl, 2, dm)) + 1j * g.standard_normal((dl, 2, dm))
        B = g.standard_normal((dm, 2, dr)) + 1j * g.standard_normal((dm, 2, dr))
        mm = prec.matmul_c64 if precision == "c64" else prec.matmul_split_bf16_complex
        T = np.zeros((2, 2, dl, dr), dtype=complex)
        for s1 in range(2):
            for s2 in range(2):
                T[s1, s2] = mm(A[:, s1, :], B[:, s2, :])
        thetap = np.einsum("xyst,stac->axyc", G4, T)
        ref = thetap.transpose(1, 0, 2, 3).reshape(2 * dl, 2 * dr)
        out = torch.zeros(2 * dr, 2 * dl, dtype=torch.complex128, device="cuda")
        rcs.two_site(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), G, out, precision=precision)
        got = out.cpu().numpy().T
        # fp32 accumulation of dm terms of size |a||b| ~ 2: noise ~ 2^-24 sqrt(dm) per term
        scale = np.sqrt(2 * dm) * 2.0
        assert np.abs(got - ref).max() <= 8 * 2.0 ** -24 * scale * np.sqrt(dm)
        exact = np.einsum("xyst,stac->axyc", G4, np.einsum("asb,btc->stac", A, B)).transpose(1, 0, 2, 3).reshape(2 * dl, 2 * dr)
        rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        assert rel < (2.0 ** -20 if precision == "c64" else 2.0 ** -14)


# ------------------------------------------------------------------ QR
def _qr_gpu(rcs, torch, M):
    ln, cnt = M.shape
    x = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    q = torch.zeros(cnt, ln, dtype=torch.complex128, device="cuda")
    r = torch.zeros(cnt, cnt, dtype=torch.complex128, device="cuda")
    rcs.cholqr(x, q, r)
    return q.cpu().numpy().T, r.cpu().numpy().T


QR_SHAPES = [(2048, 1024, 1e3), (300, 130, 1e2), (1100, 1100, 1e4), (2048, 2048, 1e5), (512, 64, 10.0)]


@pytest.mark.parametrize("ln,cnt,cond", QR_SHAPES)
def test_cholqr_against_numpy_qr(env, ln, cnt, cond):
    """The centre moves' QR (CholeskyQR + Newton-Schulz) against LAPACK's
    Householder QR: orthonormal Q and X = Q R to rounding (all a centre move
    needs: the state is unchanged for any orthonormal Q with X = Q R), R
    upper triangular up to the Newton-Schulz correction, and the same
    factorisation as numpy's up to the phase of each column (Q_np^H Q
    diagonal and unimodular, |diag R| equal) within CholeskyQR's forward
    error, which grows like u cond(X)^2 (the Gram squares the conditioning;
    Householder's grows like u cond(X))."""
    rcs, torch = env
    M = inputs.planted_matrix(ln, cnt, np.geomspace(1.0, 1.0 / cond, cnt), seed=ln + cnt)
    Q, R = _qr_gpu(rcs, torch, M)
    nrm = np.linalg.norm(M)
    assert np.abs(Q.conj().T @ Q - np.eye(cnt)).max() < 1e-13
    assert np.linalg.norm(M - Q @ R) <= 1e-14 * nrm * np.sqrt(cnt)
    assert np.abs(np.tril(R, -1)).max() <= 1e-10 * np.abs(R).max()
    Qn, Rn = np.linalg.qr(M)
    D = Qn.conj().T @ Q
    fwd = max(1e-10, 1e-15 * cond ** 2)
    assert np.abs(D - np.diag(np.diag(D))).max() < fwd
    assert np.abs(np.abs(np.diag(D)) - 1.0).max() < fwd
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rn)), rtol=fwd, atol=1e-14 * nrm)


@pytest.mark.parametrize("kind", ["rank_deficient", "ill_conditioned"])
def test_cholqr_refuses_what_it_cannot_orthogonalise(env, kind):
    """Rank-deficient and badly conditioned inputs are reported (NUMERIC), not
    returned with a non-orthonormal Q; the build then takes the Jacobi path."""
    rcs, torch = env
    spec = np.r_[np.ones(200), np.zeros(56)] if kind == "rank_deficient" else np.geomspace(1.0, 1e-9, 256)
    M = inputs.planted_matrix(600, 256, spec, seed=9)
    with pytest.raises(rcs.RcsError) as ei:
        _qr_gpu(rcs, torch, M)
    assert ei.value.status == 5
