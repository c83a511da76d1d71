"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and the benchmark.  Holds none of the method's arithmetic: only random
numbers (numpy's PCG64 streams) and workload descriptions.
"""
import math

import numpy as np

# The workloads: grid, cycles, bond cap, truncation threshold, shots.
WORKLOADS = {
    # 12 qubits, 3x4, 8 cycles, exact (chi 64, no truncation), complex128
    "rcs12_3x4_c8_chi64_exact": dict(rows=3, cols=4, cycles=8, removed_random=0,
                                     chi=64, eps=0.0, shots=10_000, precision="c128"),
    # 30 qubits, 5x6, 14 cycles, chi 256, eps 1e-8, complex64 contractions
    "rcs30_5x6_c14_chi256": dict(rows=5, cols=6, cycles=14, removed_random=0,
                                 chi=256, eps=1e-8, shots=100_000, precision="c64"),
    # 53 qubits, 6x9 minus one seed-chosen site, 14 cycles, chi 1024
    "rcs53_6x9_c14_chi1024": dict(rows=6, cols=9, cycles=14, removed_random=1,
                                  chi=1024, eps=1e-8, shots=1_000_000,
                                  precision="split_bf16"),
    # 64 independent circuits: n ~ U{20..40} on near-square grids, cycles ~
    # U{8..20}, chi ~ U{64, 128, 256, 512} (batch seed 7), 50,000 shots each
    "rcs_batch64_n20to40": dict(batch=64, batch_seed=7, n_lo=20, n_hi=40, cyc_lo=8, cyc_hi=20,
                                chis=(64, 128, 256, 512), eps=1e-8, shots=50_000, precision="c64"),
    # 30 qubits, 5x6, 8/10/12 cycles: plain and learned builds at chi 1024
    # and 256, 1M shots each scored by linear XEB against the exact
    # probabilities (GPU dense state vector); the rank network is trained on
    # a 14-cycle circuit of another seed
    "rcs30_true_xeb": dict(rows=5, cols=6, cycles=14, score_cycles=(8, 10, 12), removed_random=0,
                           chis=(1024, 256), eps=1e-8, shots=1_000_000, precision="split_bf16", true_xeb=True),
    # 53 qubits, 20 cycles, chi cap 2048, 2.5M shots
    "rcs53_6x9_c20_chi2048": dict(rows=6, cols=9, cycles=20, removed_random=1,
                                  chi=2048, eps=1e-8, shots=2_500_000,
                                  precision="split_bf16"),
}


def rng(seed):
    return np.random.default_rng(seed)


def random_bitstrings(n_qubits, m, seed):
    g = rng(seed)
    hi = g.integers(0, 1 << 32, size=m, dtype=np.uint64)
    lo = g.integers(0, 1 << 32, size=m, dtype=np.uint64)
    x = (hi << np.uint64(32)) | lo
    if n_qubits < 64:
        x &= np.uint64((1 << n_qubits) - 1)
    return x


def random_complex(shape, seed, scale=1.0):
    g = rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) * scale


def random_site_tensors(dims, seed):
    """Raw random site tensors A_k (dims[k], 2, dims[k+1]); not canonical."""
    g = rng(seed)
    out = []
    for k in range(len(dims) - 1):
        shp = (dims[k], 2, dims[k + 1])
        out.append(g.standard_normal(shp) + 1j * g.standard_normal(shp))
    return out


def planted_matrix(m, n, spectrum, seed):
    """U diag(spectrum) V^H with Haar-like random unitaries (QR of Gaussians)."""
    g = rng(seed)
    r = len(spectrum)
    a = g.standard_normal((m, r)) + 1j * g.standard_normal((m, r))
    b = g.standard_normal((n, r)) + 1j * g.standard_normal((n, r))
    u, _ = np.linalg.qr(a)
    v, _ = np.linalg.qr(b)
    return (u * np.asarray(spectrum)) @ v.conj().T


def batch_circuits(count, seed, n_lo=20, n_hi=40, cyc_lo=8, cyc_hi=20,
                   chis=(64, 128, 256, 512)):
    """Heterogeneous batch: qubit counts, cycles and bond caps drawn uniformly."""
    g = rng(seed)
    out = []
    for i in range(count):
        n = int(g.integers(n_lo, n_hi + 1))
        R = int(math.isqrt(n))
        C = -(-n // R)
        out.append(dict(n=n, rows=R, cols=C, removed=list(range(n, R * C)),
                        cycles=int(g.integers(cyc_lo, cyc_hi + 1)),
                        chi=int(chis[int(g.integers(0, len(chis)))]),
                        seed=int(g.integers(1, 1 << 62))))
    return out


def mlp_init(seed):
    """He-normal initial weights for the 66-128-128-32 network, zero biases."""
    g = rng(seed)
    shapes = [(128, 66), (128,), (128, 128), (128,), (32, 128), (32,)]
    out = []
    for shp in shapes:
        if len(shp) == 2:
            out.append(g.standard_normal(shp) * math.sqrt(2.0 / shp[1]))
        else:
            out.append(np.zeros(shp))
    return np.concatenate([x.reshape(-1) for x in out])
