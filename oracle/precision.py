"""Exact emulation of the reduced-precision contraction modes.

* complex64: inputs rounded to float32 (round-to-nearest-even), products
  accumulated in float32;
* split-bf16: each float32 x is split as hi = bf16(x), lo = bf16(x - hi)
  (bf16 = round-to-nearest-even to 8 significant bits, done on the float32
  bit pattern); a real product a*b is formed as hi_a hi_b + hi_a lo_b +
  lo_a hi_b with float32 accumulation (Henry, Tang, Heinecke, "Leveraging
  the bfloat16 artificial intelligence datatype for higher-precision
  computations", ARITH 2019); complex products use the four-real-product
  form.

The emulated products are exact in float64 (a bf16 x bf16 product has 16
significant bits), so the emulation here accumulates in float64: the result
is the exact value of the three-product sum, against which a float32
accumulation differs only by accumulation-order rounding.
"""
import numpy as np


def bf16_rne(x):
    """Round float32 values to bfloat16 (returned as float32), RNE."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32)


def split_bf16(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def matmul_split_bf16_real(a, b):
    """a @ b with the three-product split, exact (float64) accumulation."""
    ah, al = split_bf16(a)
    bh, bl = split_bf16(b)
    f = lambda x: x.astype(np.float64)
    return f(ah) @ f(bh) + f(ah) @ f(bl) + f(al) @ f(bh)


def matmul_split_bf16_complex(a, b):
    ar, ai = a.real.astype(np.float32), a.imag.astype(np.float32)
    br, bi = b.real.astype(np.float32), b.imag.astype(np.float32)
    m = matmul_split_bf16_real
    return (m(ar, br) - m(ai, bi)) + 1j * (m(ar, bi) + m(ai, br))


def matmul_c64(a, b):
    """Inputs rounded to complex64, exact products, float64 accumulation."""
    a32 = a.astype(np.complex64).astype(np.complex128)
    b32 = b.astype(np.complex64).astype(np.complex128)
    return a32 @ b32
