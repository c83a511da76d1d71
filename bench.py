#!/usr/bin/env python3
"""Benchmark of the random-circuit-sampling hot path on one MI355X.

One step = build the MPS output state of the 53-qubit (6x9 grid minus one
seed-chosen site), 14-cycle ABCDCDAB circuit at bond cap chi = 1024, draw
1,000,000 shots from it, and score them by linear XEB (self-XEB from the
shots' own log2 probabilities).  `value` is the whole step's throughput in
shots per second; the state-build seconds and the sampling rate are reported
beside it.  Inputs (the circuit description, the shot buffers) are resident
before the timed region starts.

Forms: "plain" = complex128 contractions and the fp64 full SVD; "learned" =
split-bf16 contractions, network-predicted ranks, fp32 randomized range
finder with fp64 fall-back (weights from --mlp, or trained before the timed
region on spectra of a differently seeded circuit).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--form plain|learned]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="rcs53_6x9_c14_chi1024")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--form", default="plain", choices=["plain", "learned"])
    ap.add_argument("--mlp", default=None, help=".npy packed network weights (learned form)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--profile-every", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-ops", type=int, default=-1, help="truncate the schedule (debugging only)")
    ap.add_argument("--hbm-copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 8 device-to-device copies of MIB MiB (scales rocprofv3 FETCH/WRITE_SIZE)")
    return ap.parse_args()


# the source file of each probed kernel class (its hash ties counter data to
# the kernel version it was taken on)
KERNEL_SOURCE = {"k_chain_gemm": "sample.hip", "k_jac_gram": "jacobi.hip", "k_jac_rotate": "jacobi.hip",
                 "k_two_site": "build.hip", "k_range_finder": "rsvd.hip"}


def source_hash(kernel):
    import hashlib
    path = os.path.join(ROOT, "paper_2512_07311_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, workload, form):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (FETCH_SIZE and WRITE_SIZE runs of this workload, calibrated by a
    copy kernel), or None when there are none for the current kernel source."""
    import glob
    want = {"kernel": kernel, "workload": workload, "form": form, "source_sha": source_hash(kernel)}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(path) as f:
            for line in f:
                if line.startswith("traffic-json: "):
                    d = json.loads(line[len("traffic-json: "):])
                    if all(d.get(k) == v for k, v in want.items()):
                        return d["bytes_per_launch"]
    return None


def cpu_baseline(wl, seed, budget_s=20.0):
    """The oracle (numpy fp64) timed on a bounded sample of the same workload
    and scaled to end-to-end shots/s for the full schedule and shot count:
    one saturated two-site update at half the bond cap (cost scales as
    chi^3: x8), and chain-rule shots on an MPS with the workload's bond
    profile."""
    import numpy as np
    from oracle import circuit as oc, mps, sample
    from tests import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    c = oc.Circuit(wl["rows"], wl["cols"], wl["cycles"], seed, n_removed_random=wl["removed_random"])
    _, ops = mps.schedule(c)
    n_upd = sum(1 for o in ops if o[0] == "u")
    chi = wl["chi"]
    half = max(1, chi // 2)
    g = inputs.rng(11)
    st = mps.MPS(3, [0, 1, 2])
    shp = [(half, 2, half), (half, 2, half), (half, 2, half)]
    st.A = [(g.standard_normal(s_) + 1j * g.standard_normal(s_)) / np.sqrt(2 * half) for s_ in shp]
    st.center = 1
    t0 = time.time()
    st.update(0, c.gate2, half, wl["eps"])
    t_upd = (time.time() - t0) * 8.0
    dims = [1] + [min(2 ** min(k, c.n - k), chi) for k in range(1, c.n)] + [1]
    A = inputs.random_site_tensors(dims, seed=12)
    st2 = mps.MPS(c.n, list(range(c.n)))
    st2.A = [a / np.sqrt(2 * a.shape[2]) for a in A]
    t1 = time.time()
    n_sh = 0
    while time.time() - t1 < budget_s * 0.4 or n_sh == 0:
        sample.sample(st2, 8, seed=1003, first_shot=n_sh)
        n_sh += 8
    t_shot = (time.time() - t1) / n_sh
    shots = wl["shots"]
    total = n_upd * t_upd + shots * t_shot
    return {"value": shots / total, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": ("numpy fp64 oracle on %d host threads: one two-site update at chi=%d "
                       "(%.2f s, x8 for chi=%d, x%d updates) + %d chain-rule shots on a chi=%d "
                       "bond profile (%.4f s each, x%d shots); extrapolated end-to-end"
                       % (threads, half, t_upd / 8, chi, n_upd, n_sh, chi, t_shot, shots))}


def batch_step_fn(rcs, torch, wl, args):
    """Heterogeneous batch: all circuits built concurrently (rcs_build_batch),
    all shots drawn by the graph-captured grouped sampler, one XEB per circuit."""
    from tests import inputs
    specs = inputs.batch_circuits(wl["batch"], wl["batch_seed"], wl["n_lo"], wl["n_hi"], wl["cyc_lo"],
                                  wl["cyc_hi"], wl["chis"])
    circs = [rcs.Circuit(s["rows"], s["cols"], s["cycles"], s["seed"], removed=s["removed"]) for s in specs]
    chis = [s["chi"] for s in specs]
    shots = args.shots or wl["shots"]
    bits = torch.zeros(len(circs), shots, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(len(circs), shots, dtype=torch.float64, device="cuda")
    kw = dict(contraction=wl["precision"])

    def step():
        t0 = time.time()
        states = rcs.State.build_batch(circs, chis, [wl["eps"]] * len(circs), **kw)
        torch.cuda.synchronize()
        t_b = time.time()
        print("bench: %d states built in %.1f s" % (len(states), t_b - t0), file=sys.stderr, flush=True)
        rcs.sample_batch(states, shots, 1004, bits, l2)
        xs = [rcs.xeb_log2(c.n, l2[i])[0] for i, c in enumerate(circs)]
        torch.cuda.synchronize()
        print("bench: %d x %d shots sampled and scored in %.2f s" % (len(states), shots, time.time() - t_b),
              file=sys.stderr, flush=True)
        return states, t_b - t0, time.time() - t_b, xs
    return specs, step


def main_batch(args, wl):
    import numpy as np
    import torch
    import paper_2512_07311_amd as rcs
    from paper_2512_07311_amd import autotune
    torch.cuda.set_device(0)
    tuned = os.path.exists(autotune.TUNING_FILE) and autotune.load(autotune.TUNING_FILE, torch)
    specs, step = batch_step_fn(rcs, torch, wl, args)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.time()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    sec = (time.time() - t0) / args.steps
    states, t_build, t_sample, xs = res[-1]
    shots = (args.shots or wl["shots"]) * len(states)
    infos = [s.info() for s in states]
    out = {
        "metric": "batched state-build + shots/s per MI355X (64 heterogeneous circuits)",
        "value": shots / sec, "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64/f64", "data": "synthetic (seeded random circuits)",
        "config": {"workload": args.workload, "circuits": len(states), "shots_per_circuit": shots // len(states),
                   "qubits": [s["n"] for s in specs], "cycles": [s["cycles"] for s in specs],
                   "chi": [s["chi"] for s in specs], "eps": wl["eps"], "contraction": wl["precision"],
                   "autotuned": bool(tuned)},
        "state_build_s": t_build, "sample_s": t_sample,
        "self_xeb_mean": float(np.mean(xs)), "log_fidelity_est": [i.log_fidelity_est for i in infos],
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # the state build reports its progress on stderr every 20 s
    os.environ.setdefault("RCS_PROGRESS", "20")
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.hbm_copy_calibration:
        # a plain copy of known size: each launch reads and writes MIB MiB
        torch.cuda.set_device(0)
        n = args.hbm_copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(8):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"hbm_copy_calibration_mib": args.hbm_copy_calibration, "launches": 8}), flush=True)
        return
    import paper_2512_07311_amd as rcs
    from tests import inputs
    torch.cuda.set_device(0)
    wl = dict(inputs.WORKLOADS[args.workload])
    if "batch" in wl:
        return main_batch(args, wl)
    shots = args.shots or wl["shots"]
    circ = rcs.Circuit(wl["rows"], wl["cols"], wl["cycles"], args.seed,
                       n_removed_random=wl["removed_random"])
    kw = dict(contraction="c128", rank_mode=0)
    mlp_w = None
    if args.form == "learned":
        kw = dict(contraction=wl["precision"], rank_mode=1, fallback_tau=1e-6)
        if args.mlp:
            mlp_w = np.load(args.mlp).astype(np.float32)
        else:
            from paper_2512_07311_amd import learn
            tr = inputs.WORKLOADS["rcs30_5x6_c14_chi256"]
            tc = rcs.Circuit(tr["rows"], tr["cols"], tr["cycles"], args.seed + 1)
            st = rcs.State.build(tc, tr["chi"], tr["eps"], log_spectra=True)
            X, Y = learn.dataset(st.spectra(), tc.n, tr["cycles"], torch)
            print("bench: %d training spectra logged" % X.shape[0], file=sys.stderr, flush=True)
            mlp_w, _ = learn.train(X, Y, torch, steps=1500, batch=256, seed=args.seed)
            print("bench: rank network trained", file=sys.stderr, flush=True)
            del st
        kw["mlp_weights"] = mlp_w
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    log2p = torch.zeros(shots, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        st = rcs.State.build(circ, wl["chi"], wl["eps"], stream=stream, max_ops=args.max_ops, **kw)
        print("bench: state built in %.1f s" % st.info().build_seconds, file=sys.stderr, flush=True)
        t_b = time.time()
        st.sample(bits, log2p, seed=1003)
        x, se = rcs.xeb_log2(circ.n, log2p)
        torch.cuda.synchronize()
        print("bench: %d shots sampled and scored in %.2f s" % (shots, time.time() - t_b), file=sys.stderr,
              flush=True)
        return st, time.time() - t_b, x, se

    for _ in range(args.warmup):
        step()
    rcs.profile_enable(args.profile_every)
    torch.cuda.synchronize()
    t0 = time.time()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.time()
    prof = [rcs.profile_read(k) for k in range(len(rcs.KERNEL_CLASSES))]
    rcs.profile_enable(0)
    st, t_sample, xeb, se = res[-1]
    inf = st.info()
    sec = (t1 - t0) / args.steps
    # dominant kernel: largest estimated total time (timed share scaled up)
    est = [p["seconds"] * (p["launches"] / p["timed"]) if p["timed"] else 0.0 for p in prof]
    dom = int(np.argmax(est))
    p = prof[dom]
    dt = {0: "fp64", 1: "fp64", 2: "fp64", 3: {"c128": "fp64", "c64": "fp32", "split_bf16": "bf16"}.get(
        kw["contraction"], "fp64"), 4: "fp32"}[dom]
    # the roof is set by the kernel's algorithmic intensity against the ridge
    # point of its datatype: below it the kernel is bound by HBM bandwidth
    intensity = p["flops"] / max(p["bytes"], 1.0)
    if intensity < PEAKS[dt] / PEAKS["hbm"]:
        achieved = p["bytes"] / p["seconds"] if p["seconds"] > 0 else 0.0
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAKS["hbm"] / 1e9, "unit": "GB/s",
                "frac": achieved / PEAKS["hbm"]}
    else:
        achieved = p["flops"] / p["seconds"] if p["seconds"] > 0 else 0.0
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAKS[dt] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAKS[dt]}
    roof.update({"traffic": measured_traffic(p["name"], args.workload, args.form),
            "intensity_flop_per_byte": intensity, "dtype": dt,
            "kernel": p["name"], "kernel_source_sha": source_hash(p["name"]),
            "avg_launch_us": 1e6 * p["seconds"] / max(p["timed"], 1),
            "launches_per_step": p["launches"] // max(args.steps, 1),
            "kernel_share_of_step": est[dom] / max(t1 - t0, 1e-9)})
    out = {
        "metric": "state-build s + shots/s per MI355X at chi=1024, learned/FP32 vs plain FP64, XEB",
        "value": shots / sec, "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.form == "plain" else "bf16x3/f32/f64",
        "data": "synthetic (seeded random circuit)",
        "config": {"workload": args.workload, "qubits": circ.n, "cycles": wl["cycles"], "chi": wl["chi"],
                   "eps": wl["eps"], "shots": shots, "form": args.form, "contraction": kw["contraction"],
                   "circuit_seed": args.seed, "max_ops": args.max_ops},
        "state_build_s": inf.build_seconds, "sample_shots_per_s": shots / t_sample,
        "self_xeb": xeb, "self_xeb_stderr": se, "log_fidelity_est": inf.log_fidelity_est,
        "max_bond": inf.max_bond, "n_fallbacks": inf.n_fallbacks, "n_rsvd_accepted": inf.n_rsvd_accepted,
        "roofline": roof,
        "kernels": {q["name"]: {"launches": q["launches"], "timed": q["timed"],
                                "avg_us": 1e6 * q["seconds"] / max(q["timed"], 1),
                                "flop_per_launch": q["flops"] / max(q["timed"], 1),
                                "bytes_per_launch": q["bytes"] / max(q["timed"], 1),
                                "est_total_s": e} for q, e in zip(prof, est)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
