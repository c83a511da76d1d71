"""Helpers for GPU parity tests (no method arithmetic)."""
import numpy as np
import pytest


def get_rcs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_07311_amd as rcs     # raises if the library is not built
    return rcs, torch


def to_complex(a):
    a = a.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def normwise_rel(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def oracle_state_from(st_host):
    """Oracle MPS object holding exported/imported tensors."""
    from oracle import mps
    dims, snake, tens = st_host
    o = mps.MPS(len(snake), list(int(x) for x in snake))
    o.A = [np.asarray(t) for t in tens]
    return o


def compare_shots(gpu_bits, oracle_bits, tight):
    """All shots equal except those whose oracle decision margin was below
    the exemption threshold somewhere (counted, expected ~0)."""
    g = np.asarray(gpu_bits).astype(np.uint64)
    ok = (g == oracle_bits) | (tight >= 0)
    return bool(np.all(ok)), int(np.sum(tight >= 0)), int(np.sum(g != oracle_bits))


def truncated_tolerance(om):
    """Amplitude bar for a truncated fp64 build against the oracle.

    A truncation keeps the span of the top-k singular vectors; a backward
    error e in the two-site matrix rotates that span by about
    e * s_k / (s_k - s_{k+1}) (first-order perturbation of singular
    subspaces, Wedin 1972).  Both SVDs have e of order 1e-13 relative
    (sqrt(m) u times the sweep count of a Jacobi or bidiagonal method), so the
    bar is 1e-13 times the summed conditioning of the cuts, never below 1e-10.
    """
    return max(1e-10, 1e-13 * cut_conditioning(om.records))


def cut_conditioning(records):
    """Sum over the truncated cuts of s_k / (s_k - s_{k+1}) (1-based k kept):
    the first-order amplification of a backward error into the kept
    subspace, summed along the schedule."""
    kappa = 0.0
    for rec in records:
        s, k = rec["spectrum"], rec["k"]
        if k < len(s) and s[k] > 1e-12 * s[0] and s[k - 1] > s[k]:
            kappa += s[k - 1] / (s[k - 1] - s[k])
    return kappa


def relative_noise(delta, seed):
    """A perturbation for the oracle's truncating updates: adds seeded
    Gaussian noise of relative Frobenius size delta to each two-site matrix
    before its SVD.  Rebuilding with it measures how strongly a schedule
    amplifies a per-step error of that size (the scale of another correct
    implementation's rounding)."""
    g = np.random.default_rng(seed)

    def perturb(m):
        e = g.standard_normal(m.shape) + 1j * g.standard_normal(m.shape)
        return m + (delta * np.linalg.norm(m) / np.linalg.norm(e)) * e
    return perturb
