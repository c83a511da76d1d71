"""Philox4x32-10, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11: a 128-bit counter and a 64-bit key go through ten rounds; each round
multiplies counter words 0 and 2 by two fixed 32-bit multipliers, swaps the
halves of the 64-bit products with words 1 and 3 xor the key, and the key is
bumped by two Weyl constants between rounds.

Vectorised over numpy arrays of counters (values kept in uint64 holding
32-bit words).  Test infrastructure only.

Stream layout used throughout (every random number the method draws is a
pure function of (seed, counter)):
  key   = (seed & 0xffffffff, seed >> 32)
  ctr.w = stream id: 0 gate draws, 1 removed site, 2 shots, 3 test
          bitstrings, 4 sketch matrices, 5 network init, 6 batch seeds.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

STREAM_CIRCUIT = 0
STREAM_LAYOUT = 1
STREAM_SHOTS = 2
STREAM_TESTBITS = 3
STREAM_SKETCH = 4
STREAM_MLP = 5
STREAM_BATCH = 6


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words for counters (c0..c3), key (k0,k1).

    Inputs may be python ints or numpy integer arrays (broadcast together).
    Outputs are uint64 arrays holding 32-bit values.
    """
    c0, c1, c2, c3 = np.broadcast_arrays(*[np.asarray(c, dtype=np.uint64) & _MASK
                                           for c in (c0, c1, c2, c3)])
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for _ in range(10):
        p0 = m0 * c0          # exact: both factors < 2^32
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def key_of(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def u53(lo, hi):
    """Uniform double in [0,1) from two 32-bit words: top 53 of (hi:lo)."""
    x = (np.asarray(hi, dtype=np.uint64) << np.uint64(32)) | np.asarray(lo, dtype=np.uint64)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def shot_uniform(seed, shot, site):
    """Uniform for shot index `shot` at MPS site `site` (stream 2).

    Counter (shot_lo, shot_hi, site >> 1, 2); words (x0, x1) serve even
    sites, (x2, x3) odd sites.
    """
    k0, k1 = key_of(seed)
    shot = np.asarray(shot, dtype=np.uint64)
    site = np.asarray(site, dtype=np.uint64)
    x0, x1, x2, x3 = philox4x32_10(shot & _MASK, shot >> np.uint64(32),
                                   site >> np.uint64(1), STREAM_SHOTS, k0, k1)
    odd = (site & np.uint64(1)).astype(bool)
    lo = np.where(odd, x2, x0)
    hi = np.where(odd, x3, x1)
    return u53(lo, hi)
