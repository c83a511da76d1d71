#!/usr/bin/env python3
"""Benchmark of the random-circuit-sampling hot path on one MI355X.

One step = build the MPS output state of the 53-qubit (6x9 grid minus one
seed-chosen site), 14-cycle ABCDCDAB circuit at bond cap chi = 1024, draw
1,000,000 shots from it, and score them by linear XEB (self-XEB from the
shots' own log2 probabilities).  `value` is the whole step's throughput in
shots per second of the plain form (complex128 contractions, fp64 full SVD);
the state-build seconds and the sampling rate are reported beside it, and
so is one step of the learned form (split-bf16 contractions,
network-predicted ranks, fp32 randomized range finder with the fp64 judge),
timed the same way.  Inputs (the circuit description, the shot buffers) are
resident before the timed region starts.

Wall-clock budget: one full step takes minutes, so --steps and --warmup are
upper limits.  The warm-up runs on the 30-qubit chi-256 circuit (it loads
every kernel class, and its logged spectra train the rank network); timed
steps continue only while the next one, the learned step and the CPU
baseline still fit in --budget-s seconds from process start.  The line
reports the steps and warm-ups actually run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s S]
"""
import time

T_PROC0 = time.time()

import argparse  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import os  # noqa: E402
import sys  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}
CPU_BASELINE_S = 25.0     # wall-clock of the oracle sample


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget from process start; steps stop when the next would overrun")
    ap.add_argument("--workload", default="rcs53_6x9_c14_chi1024")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--form", default="both", choices=["plain", "learned", "both"])
    ap.add_argument("--mlp", default=None, help=".npy packed network weights (learned form)")
    ap.add_argument("--learned-svd", default="f32", choices=["f32", "f64"],
                    help="precision of the learned form's full SVDs")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--network", default="interleaved", choices=["interleaved", "snake"],
                    help="MPS order and swap network of the schedule")
    ap.add_argument("--profile-every", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-ops", type=int, default=-1, help="truncate the schedule (debugging only)")
    ap.add_argument("--hbm-copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 8 device-to-device copies of MIB MiB (scales rocprofv3 FETCH/WRITE_SIZE)")
    return ap.parse_args()


def elapsed():
    return time.time() - T_PROC0


def log(msg):
    print("bench [%6.1f s]: %s" % (elapsed(), msg), file=sys.stderr, flush=True)


# the source file of each probed kernel class (its hash ties counter data to
# the kernel version it was taken on)
KERNEL_SOURCE = {"k_chain_gemm": "sample.hip", "k_jac_gram": "jacobi.hip", "k_jac_rotate": "jacobi.hip",
                 "k_two_site": "build.hip", "k_range_finder": "rsvd.hip", "k_factor_other": "chol.hip"}


def source_hash(kernel):
    import hashlib
    path = os.path.join(ROOT, "paper_2512_07311_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# kernels of the fp64 factorisation stage (Jacobi passes and the probed
# factorisation class) and the sources that hold them
STAGE_KERNELS = ("k_jac_gram", "k_jac_rotate", "k_cgemm_cm", "k_chol_panel", "k_chol_to_y", "k_chol_update",
                 "k_colnorm", "k_gather_normalize", "k_gram_upper", "k_max_dev_identity", "k_ns_apply", "k_ns_gram",
                 "k_permute_cols", "k_project", "k_project_rows", "k_sort_rank", "k_sum_sq", "k_unpermute_rows")
STAGE_SOURCES = ("jacobi.hip", "chol.hip", "build.hip")


def stage_hash():
    import hashlib
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_07311_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_stage_traffic(workload, form):
    """HBM bytes per step of the factorisation stage from the committed
    rocprofv3 counter summaries (calibrated FETCH_SIZE + WRITE_SIZE over
    every dispatch of STAGE_KERNELS in one step), or None when there are none
    for the current sources."""
    import glob
    want = {"stage": "factorisation", "workload": workload, "form": form, "source_sha": stage_hash()}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(path) as f:
            for line in f:
                if line.startswith("stage-traffic-json: "):
                    d = json.loads(line[len("stage-traffic-json: "):])
                    if all(d.get(k) == v for k, v in want.items()):
                        return d["bytes_per_step"]
    return None


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


def cpu_baseline(wl, seed, update_shapes, budget_s=CPU_BASELINE_S):
    """The oracle (numpy fp64) timed on a bounded sample of the same workload
    and scaled to end-to-end shots/s: two-site updates timed at three bond
    sizes give a power law in the SVD's m n min(m, n), which is summed over
    the real shapes of every update of the GPU build; chain-rule shots on an
    MPS with the workload's bond profile give the per-shot time."""
    import numpy as np
    from oracle import circuit as oc, mps, sample
    from tests import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    c = oc.Circuit(wl["rows"], wl["cols"], wl["cycles"], seed, n_removed_random=wl["removed_random"])
    t_begin = time.time()

    def cost(dl, dr):
        m, n = 2 * dl, 2 * dr
        return float(m) * n * min(m, n)

    def time_update(d):
        g = inputs.rng(11 + d)
        st = mps.MPS(3, [0, 1, 2])
        shp = (d, 2, d)
        st.A = [(g.standard_normal(shp) + 1j * g.standard_normal(shp)) / np.sqrt(2 * d) for _ in range(3)]
        st.center = 1
        t0 = time.time()
        st.update(0, c.gate2, d, wl["eps"])
        return time.time() - t0

    time_update(32)                    # first-call overheads out of the fit
    sizes, times = [], []
    for d in (128, 256, 512):
        t = time_update(d)
        sizes.append(cost(d, d))
        times.append(t)
        if time.time() - t_begin > 0.6 * budget_s:
            break
    if len(sizes) >= 2:
        p, logc = np.polyfit(np.log(sizes), np.log(times), 1)
    else:
        p, logc = 1.0, np.log(times[0] / sizes[0])
    t_updates = float(sum(np.exp(logc) * cost(int(u[2]), int(u[4])) ** p for u in update_shapes))
    dims = [1] + [min(2 ** min(k, c.n - k), wl["chi"]) for k in range(1, c.n)] + [1]
    A = inputs.random_site_tensors(dims, seed=12)
    st2 = mps.MPS(c.n, list(range(c.n)))
    st2.A = [a / np.sqrt(2 * a.shape[2]) for a in A]
    t1 = time.time()
    n_sh = 0
    while time.time() - t1 < max(0.3 * budget_s, 1.0) or n_sh == 0:
        sample.sample(st2, 8, seed=1003, first_shot=n_sh)
        n_sh += 8
    t_shot = (time.time() - t1) / n_sh
    shots = wl["shots"]
    total = t_updates + shots * t_shot
    return {"value": shots / total, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": ("numpy fp64 oracle on %d host threads: two-site updates timed at chi %s "
                       "(%s s), fitted t = c (m n min(m,n))^%.2f and summed over the %d real update "
                       "shapes of the GPU build (%.0f s); %d chain-rule shots on a chi=%d bond profile "
                       "(%.4f s each, x%d shots); %.0f s of CPU time measured"
                       % (threads, [int(round((s / 8) ** (1 / 3))) for s in sizes],
                          ", ".join("%.2f" % t for t in times), p, len(update_shapes), t_updates, n_sh,
                          wl["chi"], t_shot, shots, time.time() - t_begin)),
            "projected_build_s": t_updates, "per_shot_s": t_shot}


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
        log("%d states built in %.1f s" % (len(states), t_b - t0))
        rcs.sample_batch(states, shots, 1004, bits, l2)
        xs = [rcs.xeb_log2(c.n, l2[i])[0] for i, c in enumerate(circs)]
        torch.cuda.synchronize()
        log("%d x %d shots sampled and scored in %.2f s" % (len(states), shots, time.time() - t_b))
        return states, t_b - t0, time.time() - t_b, xs
    return specs, step


def main_true_xeb(args, wl):
    """True linear XEB (Section 5.1: scored against the circuit's exact
    output probabilities) of plain and learned builds of 30-qubit circuits
    at several depths: the exact state comes from the GPU dense state vector
    (16 GiB), each build draws wl["shots"] shots, and each shot is scored by
    its exact probability, next to the build's own fidelity estimate.  The
    rank network is trained on the spectra of another seed's build.  Prints
    one JSON line; not the headline benchmark."""
    import numpy as np
    import torch
    import paper_2512_07311_amd as rcs
    from paper_2512_07311_amd import learn
    torch.cuda.set_device(0)
    tc = rcs.Circuit(wl["rows"], wl["cols"], wl["cycles"], args.seed + 1, network=args.network)
    wst = rcs.State.build(tc, 256, wl["eps"], log_spectra=True)
    X, Y = learn.dataset(wst.spectra(), tc.n, wl["cycles"], torch)
    mlp_w, _ = learn.train(X, Y, torch, steps=1500, batch=256, seed=args.seed)
    del wst
    log("rank network trained on %d spectra" % X.shape[0])
    shots = args.shots or wl["shots"]
    psi = torch.zeros(1 << tc.n, dtype=torch.complex128, device="cuda")
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    p = torch.zeros(shots, dtype=torch.float64, device="cuda")
    forms = {"plain": dict(contraction="c128", rank_mode=0),
             "learned": dict(contraction=wl["precision"], rank_mode=1, fallback_tau=1e-6, mlp_weights=mlp_w,
                             svd_precision=args.learned_svd)}
    rows = []
    for cyc in wl["score_cycles"]:
        circ = rcs.Circuit(wl["rows"], wl["cols"], cyc, args.seed, network=args.network)
        t0 = time.time()
        rcs.dense_simulate(circ, psi)
        torch.cuda.synchronize()
        log("exact %d-qubit %d-cycle state in %.2f s" % (circ.n, cyc, time.time() - t0))
        for chi in wl["chis"]:
            for form, kw in forms.items():
                st = rcs.State.build(circ, chi, wl["eps"], **kw)
                inf = st.info()
                st.sample(bits, seed=1003)
                rcs.dense_gather(psi, circ.n, bits, p, probabilities=True)
                xeb, se = rcs.xeb(circ.n, p)
                rows.append({"cycles": cyc, "chi": chi, "form": form, "state_build_s": inf.build_seconds,
                             "fidelity_est": float(np.exp(inf.log_fidelity_est)), "true_xeb": xeb,
                             "true_xeb_stderr": se, "n_rsvd_accepted": inf.n_rsvd_accepted,
                             "n_fallbacks": inf.n_fallbacks})
                log("cycles %d chi %d %s: build %.2f s, F_est %.4f, true XEB %.4f +- %.4f"
                    % (cyc, chi, form, inf.build_seconds, rows[-1]["fidelity_est"], xeb, se))
                del st
    out = {"metric": "true linear XEB (exact probabilities) of plain and learned builds",
           "value": rows[0]["true_xeb"], "unit": "xeb", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded random circuit)",
           "config": {"workload": args.workload, "qubits": tc.n, "score_cycles": list(wl["score_cycles"]),
                      "eps": wl["eps"], "shots": shots, "swap_network": args.network, "circuit_seed": args.seed},
           "rows": rows}
    print(json.dumps(out), flush=True)


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


def learned_vs_plain(plain_build_s, plain_step_s, plain_logf, learned_build_s, learned_step_s, learned_logf):
    """The learned form's standing against the plain form: faster in state
    build and in the whole step (shots/s), at an estimated fidelity within
    1% of the plain form's."""
    rel = math.exp(learned_logf - plain_logf) - 1.0
    return {"build_faster": learned_build_s < plain_build_s, "step_faster": learned_step_s < plain_step_s,
            "fest_within_1pct": abs(rel) <= 0.01,
            "met": learned_build_s < plain_build_s and learned_step_s < plain_step_s and abs(rel) <= 0.01}


def svd_roofline(prof, inf, floor_s, steps, workload=None, form=None):
    """Roofline of the fp64 factorisation stage, every kernel that computes
    the build's SVDs and centre moves (Jacobi Gram and rotation passes, the
    Gram/Cholesky preconditioner, CholeskyQR, projections, Newton-Schulz):
    algorithmic work = the nominal flops of those factorisations (thin SVD
    4 (14 m n^2 + 8 n^3) per update, Householder QR 4 (2 m n^2 - 2 n^3 / 3)
    per centre move); time = each class's probed average launch time times
    its launches.  The probe's event interval is what rocprofv3 reports as
    the kernel's duration (the two agree on the committed kernel-trace
    summary), so the empty-launch floor is reported but not subtracted."""
    by = {p["name"]: p for p in prof}
    t_total, launches, detail = 0.0, 0, {}
    for name in ("k_jac_gram", "k_jac_rotate", "k_factor_other"):
        p = by[name]
        if not p["timed"]:
            continue
        avg = p["seconds"] / p["timed"]
        t_total += avg * p["launches"]
        launches += p["launches"]
        detail[name] = {"avg_launch_us": 1e6 * avg, "launches_per_step": p["launches"] // max(steps, 1)}
    work = steps * (inf.nominal_svd_flops + inf.nominal_qr_flops)
    achieved = work / t_total if t_total > 0 else 0.0
    traffic = measured_stage_traffic(workload, form) if workload else None
    return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAKS["fp64"] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAKS["fp64"], "traffic": traffic,
            "traffic_basis": "HBM bytes per step over every factorisation-stage dispatch (calibrated counters)",
            "kernel": "k_jac_rotate + k_jac_gram + k_factor_other (fp64 SVDs and centre moves)",
            "kernel_source_sha": stage_hash(), "dtype": "fp64",
            "work_per_step_flop": inf.nominal_svd_flops + inf.nominal_qr_flops,
            "nominal_svd_flop": inf.nominal_svd_flops, "nominal_qr_flop": inf.nominal_qr_flops,
            "kernel_seconds_per_step": t_total / max(steps, 1), "event_floor_us": 1e6 * floor_s,
            "per_kernel": detail}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # the state build reports its progress on stderr every 30 s
    os.environ.setdefault("RCS_PROGRESS", "30")
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
    if wl.get("true_xeb"):
        return main_true_xeb(args, wl)
    shots = args.shots or wl["shots"]
    circ = rcs.Circuit(wl["rows"], wl["cols"], wl["cycles"], args.seed,
                       n_removed_random=wl["removed_random"], network=args.network)
    stream = torch.cuda.current_stream()
    bits = torch.zeros(shots, dtype=torch.int64, device="cuda")
    log2p = torch.zeros(shots, dtype=torch.float64, device="cuda")
    run_plain = args.form in ("plain", "both")
    run_learned = args.form in ("learned", "both")
    log("library loaded; workload %s, %d qubits, %d updates" % (args.workload, circ.n, circ.n_updates))

    # ---- warm-up on the 30-qubit chi-256 circuit (every kernel class); its
    # logged spectra are the rank network's training data
    tr = inputs.WORKLOADS["rcs30_5x6_c14_chi256"]
    tc = rcs.Circuit(tr["rows"], tr["cols"], tr["cycles"], args.seed + 1, network=args.network)
    n_warm = 0
    mlp_w = None
    if args.warmup > 0 or (run_learned and not args.mlp):
        wst = rcs.State.build(tc, tr["chi"], tr["eps"], log_spectra=run_learned and not args.mlp,
                              stream=stream)
        wbits = torch.zeros(tr["shots"], dtype=torch.int64, device="cuda")
        wl2 = torch.zeros(tr["shots"], dtype=torch.float64, device="cuda")
        wst.sample(wbits, wl2, seed=1003)
        rcs.xeb_log2(tc.n, wl2)
        torch.cuda.synchronize()
        n_warm = 1 if args.warmup > 0 else 0
        log("warm-up: 30-qubit chi-256 build + %d shots done" % tr["shots"])
        if run_learned and not args.mlp:
            from paper_2512_07311_amd import learn
            X, Y = learn.dataset(wst.spectra(), tc.n, tr["cycles"], torch)
            mlp_w, _ = learn.train(X, Y, torch, steps=1500, batch=256, seed=args.seed)
            log("rank network trained on %d spectra" % X.shape[0])
        del wst
    if run_learned and args.mlp:
        mlp_w = np.load(args.mlp).astype(np.float32)
    floor_s = rcs.profile_event_floor()

    def step(kw):
        st = rcs.State.build(circ, wl["chi"], wl["eps"], stream=stream, max_ops=args.max_ops, **kw)
        t_build = st.info().build_seconds
        log("state built in %.1f s" % t_build)
        t_b = time.time()
        st.sample(bits, log2p, seed=1003)
        x, se = rcs.xeb_log2(circ.n, log2p)
        torch.cuda.synchronize()
        t_s = time.time() - t_b
        log("%d shots sampled and scored in %.2f s" % (shots, t_s))
        return st, t_s, x, se

    plain_kw = dict(contraction="c128", rank_mode=0)
    learned_kw = dict(contraction=wl["precision"], rank_mode=1, fallback_tau=1e-6, mlp_weights=mlp_w,
                      svd_precision=args.learned_svd)
    main_kw = plain_kw if run_plain else learned_kw
    reserve_cpu = 0.0 if args.no_cpu_baseline else CPU_BASELINE_S + 10.0

    # ---- timed region: whole steps of the main form
    rcs.profile_enable(args.profile_every)
    torch.cuda.synchronize()
    t0 = time.time()
    res = []
    t_step = None
    while len(res) < max(1, args.steps):
        if res:
            reserve = reserve_cpu + ((1.2 * t_step + 30.0) if (run_plain and run_learned) else 0.0)
            if elapsed() + 1.15 * t_step + reserve > args.budget_s:
                log("budget: stopping after %d timed steps" % len(res))
                break
        ts = time.time()
        res.append(step(main_kw))
        torch.cuda.synchronize()
        t_step = time.time() - ts
    t1 = time.time()
    prof = [rcs.profile_read(k) for k in range(len(rcs.KERNEL_CLASSES))]
    rcs.profile_enable(0)
    n_steps = len(res)
    st, t_sample, xeb, se = res[-1]
    inf = st.info()
    upd = st.updates()
    sec = (t1 - t0) / n_steps
    roof = svd_roofline(prof, inf, floor_s, n_steps, args.workload, "plain" if run_plain else "learned")
    est = {p["name"]: p["seconds"] * (p["launches"] / p["timed"]) if p["timed"] else 0.0 for p in prof}
    roof["factorisation_share_of_step"] = roof["kernel_seconds_per_step"] / sec
    out = {
        "metric": "state-build s + shots/s per MI355X at chi=1024, learned/FP32 vs plain FP64, XEB",
        "value": shots / sec, "unit": "shots/s", "n_gpus": 1, "steps": n_steps, "warmup": n_warm,
        "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if run_plain else "bf16x3/f32/f64",
        "data": "synthetic (seeded random circuit)",
        "config": {"workload": args.workload, "qubits": circ.n, "cycles": wl["cycles"], "chi": wl["chi"],
                   "eps": wl["eps"], "shots": shots, "form": "plain" if run_plain else "learned",
                   "swap_network": args.network,
                   "contraction": main_kw["contraction"], "circuit_seed": args.seed, "max_ops": args.max_ops,
                   "warmup_workload": "rcs30_5x6_c14_chi256" if n_warm else None},
        "requested": {"steps": args.steps, "warmup": args.warmup, "budget_s": args.budget_s},
        "state_build_s": inf.build_seconds, "sample_shots_per_s": shots / t_sample,
        "self_xeb": xeb, "self_xeb_stderr": se, "log_fidelity_est": inf.log_fidelity_est,
        "fidelity_est": float(np.exp(inf.log_fidelity_est)),
        "max_bond": inf.max_bond, "n_updates": int(len(upd)), "n_center_moves": inf.n_center_moves,
        "roofline": roof,
        "kernels": {q["name"]: {"launches": q["launches"], "timed": q["timed"],
                                "avg_us_event": 1e6 * q["seconds"] / max(q["timed"], 1),
                                "est_total_s": est[q["name"]]} for q in prof},
    }
    del res, st

    # ---- the learned form, one step, timed the same way (outside the timed region)
    if run_plain and run_learned:
        if elapsed() + 1.2 * sec + reserve_cpu <= args.budget_s:
            ts = time.time()
            lst, lt_sample, lxeb, lse = step(learned_kw)
            torch.cuda.synchronize()
            lsec = time.time() - ts
            li = lst.info()
            out["learned"] = {
                "step_s": lsec, "shots_per_s": shots / lsec, "state_build_s": li.build_seconds,
                "sample_shots_per_s": shots / lt_sample, "self_xeb": lxeb, "self_xeb_stderr": lse,
                "log_fidelity_est": li.log_fidelity_est, "fidelity_est": float(np.exp(li.log_fidelity_est)),
                "fest_rel_diff_vs_plain": float(np.exp(li.log_fidelity_est - inf.log_fidelity_est) - 1.0),
                "build_speedup_vs_plain": inf.build_seconds / li.build_seconds,
                "n_rsvd_accepted": li.n_rsvd_accepted, "n_fallbacks": li.n_fallbacks,
                "n_svd_f32": li.n_svd_f32, "n_svd_f32_redone": li.n_svd_f32_redone,
                "contraction": wl["precision"], "svd_precision": args.learned_svd,
                "bar_vs_plain": learned_vs_plain(inf.build_seconds, sec, inf.log_fidelity_est,
                                                 li.build_seconds, lsec, li.log_fidelity_est)}
            del lst
        else:
            out["learned"] = {"skipped": "wall-clock budget"}
            log("budget: learned step skipped")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.seed, upd)
        log("cpu baseline done")
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
