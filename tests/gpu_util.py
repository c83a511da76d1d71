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
