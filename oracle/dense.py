"""Dense state-vector simulation (complex128), for n <= 28.

psi has 2^n entries; basis index i = sum_q b_q 2^q, so bit q of the index is
the outcome of qubit q (the same convention as the 64-bit bitstrings used
everywhere).  Gates are applied in circuit order from |0...0>.  This is the
plain definition of the circuit's output state; the MPS method of the
hot path reaches it exactly whenever no truncation happens.
"""
import numpy as np

from .circuit import ONE_QUBIT_GATES


def apply_1q(psi, n, q, U):
    v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    return np.einsum("st,atb->asb", U, v).reshape(-1)


def apply_2q(psi, n, qa, qb, G):
    """G acts on |s_a s_b> with index 2*s_a + s_b."""
    if qa == qb:
        raise ValueError("two-qubit gate on one qubit")
    hi, lo = max(qa, qb), min(qa, qb)
    v = psi.reshape(1 << (n - hi - 1), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    G4 = G.reshape(2, 2, 2, 2)                  # [sa', sb', sa, sb]
    if qa == hi:   # axis 1 is qa, axis 3 is qb
        out = np.einsum("xyst,asbtc->axbyc", G4, v)
    else:          # axis 1 is qb, axis 3 is qa
        out = np.einsum("xyst,atbsc->aybxc", G4, v)
    return out.reshape(-1)


def simulate(circ, max_layers=None):
    n = circ.n
    if n > 28:
        raise ValueError("dense oracle is limited to 28 qubits")
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for li, (kind, data) in enumerate(circ.layers):
        if max_layers is not None and li >= max_layers:
            break
        if kind == "1q":
            for q in range(n):
                psi = apply_1q(psi, n, q, ONE_QUBIT_GATES[int(data[q])])
        else:
            for qa, qb in data:
                psi = apply_2q(psi, n, qa, qb, circ.gate2)
    return psi


def probabilities(psi):
    return (psi.real ** 2 + psi.imag ** 2)
