"""Autotuner of the fp64 Jacobi SVD launch parameters (block width, inner
sweeps) per column-count bucket, timed on the device through the C ABI.

The cache is a JSON file keyed by the GPU architecture name:
  {"gfx950": [{"cnt_max": 128, "block": 16, "inner": 1, "seconds": ...}, ...]}
`load()` registers a cached table with the library (rcs_tuning_set).
`python -m paper_2512_07311_amd.autotune OUT.json` tunes on the current GPU
and writes the table; `TUNING_FILE` (next to this module) is the table the
benchmark loads when it exists.
"""
import json
import os
import time

import numpy as np

import paper_2512_07311_amd as rcs

BUCKETS = (64, 128, 256, 512, 1024, 2048, 4096)
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
CANDIDATES = [(16, 1), (16, 2), (32, 1), (32, 2)]


def _arch(torch):
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "unknown").split(":")[0]


def _time_svd(torch, n, block, inner, reps=1, seed=0):
    g = np.random.default_rng(seed + n)
    M = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    x0 = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    s = torch.zeros(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(n, n, dtype=torch.complex128, device="cuda")
    rcs.tuning_clear()
    rcs.tuning_set(1 << 30, block, inner)
    best = float("inf")
    for _ in range(reps):
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rcs.svd_jacobi(x, s, u)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(torch, buckets=BUCKETS, candidates=CANDIDATES, max_n=2048, reps=1):
    table = []
    for b in buckets:
        n = min(b, max_n)
        timings = [(c, _time_svd(torch, n, c[0], c[1], reps)) for c in candidates]
        (blk, inner), sec = min(timings, key=lambda t: t[1])
        table.append(dict(cnt_max=b, block=blk, inner=inner, seconds=sec,
                          candidates={"%d/%d" % c: t for c, t in timings}))
    rcs.tuning_clear()
    for e in table:
        rcs.tuning_set(e["cnt_max"], e["block"], e["inner"])
    return table


def save(path, table, torch):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[_arch(torch)] = table
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def load(path, torch):
    with open(path) as f:
        data = json.load(f)
    table = data.get(_arch(torch))
    if not table:
        return False
    rcs.tuning_clear()
    for e in table:
        rcs.tuning_set(e["cnt_max"], e["block"], e["inner"])
    return True


if __name__ == "__main__":
    import sys
    import torch
    out = sys.argv[1] if len(sys.argv) > 1 else TUNING_FILE
    table = tune(torch)
    save(out, table, torch)
    for e in table:
        print(json.dumps(e), flush=True)
