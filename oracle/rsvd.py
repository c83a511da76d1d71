"""Randomized truncated SVD and the accept-or-fall-back judge (fp64 reference).

Halko, Martinsson, Tropp, "Finding structure with randomness", SIAM Review
2011: randomized range finder with power iterations (their Algorithm 4.4)
followed by the direct SVD of the projected matrix (their Algorithm 5.1):

  1. Omega (n x l, l = k_hat + p) with entries in {1, i, -1, -i}: entry
     (r, c) is {1, i, -1, -i}[x0 & 3], x0 = word 0 of
     Philox(seed; (r, c, step, stream 4));
  2. Q = orth(M Omega);
  3. q times: Q = orth(M orth(M^H Q));
  4. B = Q^H M = U_b S V^H, U = Q U_b;
  5. ||M||_F^2 in fp64; the kept rank is the smallest k <= l with
     ||M||_F^2 - sum_{r<k} s_r^2 <= eps ||M||_F^2, else l; then capped at
     chi; eps_rand = (||M||_F^2 - sum_{r<k} s_r^2) / ||M||_F^2.

Judge: the randomized split is accepted when eps_rand <= max(eps,
eps_pred(k)) + tau, else the full fp64 SVD with the plain rank rule is used
and a fall-back is counted.
"""
import numpy as np

from .philox import philox4x32_10, key_of, STREAM_SKETCH

_PHASES = np.array([1.0, 1j, -1.0, -1j], dtype=np.complex128)


def sketch(n, l, seed, step):
    k0, k1 = key_of(seed)
    r = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(l, dtype=np.uint64)[None, :]
    x0, _, _, _ = philox4x32_10(r, c, step, STREAM_SKETCH, k0, k1)
    return _PHASES[(x0 & np.uint64(3)).astype(np.int64)]


def orth(y):
    q, _ = np.linalg.qr(y)
    return q


def rsvd(M, l, q_iters, seed, step):
    """Return (U, s, Vh) of rank l from the randomized range finder."""
    n = M.shape[1]
    om = sketch(n, l, seed, step)
    Q = orth(M @ om)
    for _ in range(q_iters):
        Q = orth(M @ orth(M.conj().T @ Q))
    B = Q.conj().T @ M
    Ub, s, Vh = np.linalg.svd(B, full_matrices=False)
    return Q @ Ub, s, Vh


def rsvd_rank(s, fro2, chi, eps):
    kept = np.cumsum(np.asarray(s, dtype=np.float64) ** 2)
    l = len(s)
    k = l
    for kk in range(1, l + 1):
        if fro2 - kept[kk - 1] <= eps * fro2:
            k = kk
            break
    k = min(k, int(chi))
    return k, float((fro2 - kept[k - 1]) / fro2)


def judge_accepts(eps_rand, eps, eps_pred, tau):
    return eps_rand <= max(eps, eps_pred) + tau
