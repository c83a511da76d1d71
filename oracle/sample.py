"""Sequential conditional sampling from a right-canonical MPS, and linear XEB.

Section 3.2 draws measurement shots from the persisted state and Section 5.1
scores them by linear cross-entropy benchmarking.  The sampler here is the
textbook chain-rule sampler: for a right-canonical MPS with unit norm the
marginal probability of a prefix b_0..b_k (in MPS order) is ||v||^2 with
v = A_0^{b_0} ... A_k^{b_k}.  For shot i and site k:

    w_s = v A_k^s (s = 0, 1),  p_s = ||w_s||^2 (fp64),
    u   = U53 of Philox(seed; (i_lo, i_hi, k >> 1, stream 2)),
    s_k = 0 if u (p0 + p1) < p0 else 1,   v <- w_{s_k}.

v starts as [1] and is never rescaled (|psi|^2 >= 2^-64-ish is far from
underflow for n <= 64).  Outputs: the bitstring (bit pi[k] = s_k) and
log2 p(b) = log2 of the final ||v||^2.

Linear XEB (Section 5.1): F = 2^n mean_i p_ref(b_i) - 1, with standard error
std(2^n p_ref) / sqrt(M) (sample standard deviation, M - 1 denominator).
"""
import numpy as np

from .philox import shot_uniform


def sample(st, n_shots, seed, first_shot=0, margin_delta=1e-12, chunk=4096):
    """Returns (bits uint64[n], log2p float64[n], first_tight_site int64[n]).

    first_tight_site[i] is the first site whose decision margin
    |u (p0+p1) - p0| / (p0+p1) is below margin_delta (-1 if none): from that
    site on, another fp64 evaluation order may legitimately decide otherwise.
    """
    n = st.n
    bits_all = np.zeros(n_shots, dtype=np.uint64)
    log2p_all = np.zeros(n_shots, dtype=np.float64)
    tight_all = np.full(n_shots, -1, dtype=np.int64)
    for c0 in range(0, n_shots, chunk):
        c1 = min(n_shots, c0 + chunk)
        idx = np.arange(first_shot + c0, first_shot + c1, dtype=np.uint64)
        m = c1 - c0
        v = np.ones((m, 1), dtype=np.complex128)
        bits = np.zeros(m, dtype=np.uint64)
        tight = np.full(m, -1, dtype=np.int64)
        last_p = None
        for k in range(n):
            w0 = v @ st.A[k][:, 0, :]
            w1 = v @ st.A[k][:, 1, :]
            p0 = np.sum(w0.real ** 2 + w0.imag ** 2, axis=1)
            p1 = np.sum(w1.real ** 2 + w1.imag ** 2, axis=1)
            u = shot_uniform(seed, idx, k)
            tot = p0 + p1
            s = u * tot >= p0
            marg = np.abs(u * tot - p0) / tot
            newly = (tight < 0) & (marg < margin_delta)
            tight[newly] = k
            bits |= s.astype(np.uint64) << np.uint64(st.pi[k])
            v = np.where(s[:, None], w1, w0)
            last_p = np.where(s, p1, p0)
        bits_all[c0:c1] = bits
        log2p_all[c0:c1] = np.log2(last_p)
        tight_all[c0:c1] = tight
    return bits_all, log2p_all, tight_all


def linear_xeb(n_qubits, p_ref):
    """(F_XEB, standard error) from reference probabilities of the samples."""
    x = (2.0 ** n_qubits) * np.asarray(p_ref, dtype=np.float64)
    m = len(x)
    f = float(np.mean(x) - 1.0)
    se = float(np.std(x, ddof=1) / np.sqrt(m)) if m > 1 else float("nan")
    return f, se


def fidelity_estimate(log_fest):
    """F_est = prod_steps (1 - eps_step) = exp(sum log(1 - eps_step))."""
    return float(np.exp(log_fest))
