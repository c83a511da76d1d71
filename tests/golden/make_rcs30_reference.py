"""Writes the stored oracle values for the 30-qubit workload (5x6 grid,
14 cycles, chi 256, eps 1e-8): the plain CPU MPS of the snake schedule
(fp64 contractions and SVD), evaluated on 1,000 random bitstrings.

    python -m tests.golden.make_rcs30_reference

Calls only oracle/ (and the seeded input streams); takes about seven
minutes on eight cores.  The output is rcs30_5x6_c14_chi256.json beside
this file.

Besides the reference values it records how strongly this schedule
amplifies a small error made at each truncation: the oracle is rebuilt with
every two-site matrix perturbed, before its SVD, by seeded Gaussian noise of
relative Frobenius size delta, and the normwise change of the 1,000
amplitudes is stored.  delta = 1e-13 stands for the backward error of an
fp64 SVD; delta = 2^-24 sqrt(4 chi) for complex64 contractions.
"""
import json
import os
import time

import numpy as np

from oracle import circuit as oc, mps
from tests import inputs
from tests.gpu_util import cut_conditioning, relative_noise

NAME = "rcs30_5x6_c14_chi256"
CIRCUIT_SEED = 1
BITSTRING_SEED = 3
N_BITSTRINGS = 1000


def main():
    wl = inputs.WORKLOADS[NAME]
    t0 = time.time()
    c = oc.Circuit(wl["rows"], wl["cols"], wl["cycles"], CIRCUIT_SEED)
    st = mps.build(c, wl["chi"], wl["eps"])
    b = inputs.random_bitstrings(c.n, N_BITSTRINGS, seed=BITSTRING_SEED)
    amps = st.amplitudes(b)
    out = {
        "workload": NAME,
        "rows": wl["rows"], "cols": wl["cols"], "cycles": wl["cycles"], "circuit_seed": CIRCUIT_SEED,
        "chi": wl["chi"], "eps": wl["eps"],
        "bitstring_seed": BITSTRING_SEED, "n_bitstrings": N_BITSTRINGS,
        "bond_dims": [int(x) for x in st.bond_dims()],
        "log_fidelity_est": float(st.log_fest),
        "n_truncations": len(st.records),
        "cut_conditioning": float(cut_conditioning(st.records)),
        "perturbation_response": [],
        "amplitudes_re_im": [[float(a.real), float(a.imag)] for a in amps],
    }
    for delta, seed in [(1e-13, 101), (2.0 ** -24 * np.sqrt(4.0 * wl["chi"]), 102)]:
        sp = mps.build(c, wl["chi"], wl["eps"], perturb=relative_noise(delta, seed))
        ap = sp.amplitudes(b)
        out["perturbation_response"].append(dict(
            delta=float(delta), noise_seed=seed,
            normwise_rel_change=float(np.linalg.norm(ap - amps) / np.linalg.norm(amps)),
            log_fidelity_change=float(sp.log_fest - st.log_fest),
            bond_dims_equal=bool(sp.bond_dims() == st.bond_dims())))
        print(out["perturbation_response"][-1], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), NAME + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("wrote %s in %.0f s (log F_est %.6f, conditioning %.3g, |amp|^2 sum x 2^n / m = %.4f)" % (
        path, time.time() - t0, st.log_fest, out["cut_conditioning"],
        float(np.sum(np.abs(amps) ** 2)) * 2.0 ** c.n / N_BITSTRINGS))


if __name__ == "__main__":
    main()
