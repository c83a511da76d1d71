"""Host-side checks (no GPU): the C-ABI library loads and exports every
declared symbol; the C++ circuit generator and schedule compiler agree with
the oracle's, op by op; argument validation."""
import os
import re

import numpy as np
import pytest

from oracle.circuit import Circuit as OCircuit
from oracle import mps as omps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rcs():
    from paper_2512_07311_amd import build_lib
    if not os.path.exists(build_lib.LIB):
        build_lib.build(verbose=False)
    import paper_2512_07311_amd as m
    return m


def test_exports_every_declared_symbol(rcs):
    hdr = open(os.path.join(ROOT, "include", "rcs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(rcs_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 30
    import ctypes
    lib = ctypes.CDLL(rcs.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(rcs.EXPORTED)
    assert "gfx950" in rcs.version()


CONFIGS = [(3, 4, 8, 0), (5, 6, 14, 0), (6, 9, 14, 1), (6, 9, 20, 1), (4, 5, 3, 0), (2, 7, 9, 0)]


@pytest.mark.parametrize("network", ["snake", "interleaved"])
@pytest.mark.parametrize("rows,cols,cyc,rr", CONFIGS)
@pytest.mark.parametrize("seed", [1, 2, 12345678901234])
def test_generator_and_schedule_match_oracle(rcs, rows, cols, cyc, rr, seed, network):
    c = rcs.Circuit(rows, cols, cyc, seed, n_removed_random=rr, network=network)
    o = OCircuit(rows, cols, cyc, seed, n_removed_random=rr)
    assert c.n == o.n
    assert np.array_equal(c.one_qubit_gates(), o.one_qubit_draws())
    snake, ops = c.schedule()
    pi, oops = omps.schedule(o, network)
    assert list(snake) == pi
    ref = []
    for op in oops:
        if op[0] == "1q":
            ref.append((0, None, 0, op[2]))
        else:
            ref.append((1, op[1], 0 if op[2] == "fsim" else 1, op[3]))
    assert len(ops) == len(ref)
    for got, exp in zip(ops, ref):
        assert got[0] == exp[0] and got[3] == exp[3]
        if exp[0] == 1:
            assert got[1] == exp[1] and got[2] == exp[2]
    assert c.n_updates == sum(1 for r in ref if r[0] == 1)


@pytest.mark.parametrize("network", ["snake", "interleaved"])
def test_explicit_removed_sites_and_pattern(rcs, network):
    c = rcs.Circuit(4, 5, 6, 9, pattern="ACBD", removed=[0, 7], network=network)
    o = OCircuit(4, 5, 6, 9, pattern="ACBD", removed=[0, 7])
    assert c.n == o.n == 18
    assert np.array_equal(c.one_qubit_gates(), o.one_qubit_draws())
    snake, ops = c.schedule()
    pi, oops = omps.schedule(o, network)
    assert list(snake) == pi
    assert [tuple(x[1:3]) for x in ops if x[0] == 1] == \
        [(op[1], 0 if op[2] == "fsim" else 1) for op in oops if op[0] == "u"]


def test_c3_update_count(rcs):
    c = rcs.Circuit(6, 9, 14, 1, n_removed_random=1)
    assert c.n == 53 and c.n_updates == 2113
    c = rcs.Circuit(6, 9, 14, 1, n_removed_random=1, network="interleaved")
    assert c.n == 53 and c.n_updates == 1233


def test_invalid_network(rcs):
    with pytest.raises(KeyError):
        rcs.Circuit(3, 3, 2, 1, network="ladder")


@pytest.mark.parametrize("kw,msg", [
    (dict(rows=1, cols=5, n_cycles=2, seed=1), "at least 2x2"),
    (dict(rows=9, cols=9, n_cycles=2, seed=1), "qubits"),
    (dict(rows=3, cols=3, n_cycles=2, seed=1, pattern="ABE"), "pattern"),
    (dict(rows=3, cols=3, n_cycles=2, seed=1, removed=[9]), "out of range"),
    (dict(rows=3, cols=3, n_cycles=-1, seed=1), "n_cycles"),
])
def test_invalid_arguments(rcs, kw, msg):
    with pytest.raises(rcs.RcsError) as ei:
        rcs.Circuit(**kw)
    assert ei.value.status == 1 and msg in str(ei.value)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark covers one GPU: asking for more exits with status 2 and
    says so, before any GPU work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_without_a_gpu_fails_loudly():
    """No silent CPU path: without a GPU the benchmark exits non-zero and
    prints no result line."""
    import subprocess
    import sys
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr and '"metric"' not in r.stdout


def test_binding_without_the_library_raises(tmp_path):
    """The Python binding has no fallback: loaded from a folder without
    librcs.so it raises ImportError instead of importing."""
    import importlib.util
    import shutil
    pkg = tmp_path / "pkg_without_lib"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2512_07311_amd", "__init__.py"), pkg / "__init__.py")
    spec = importlib.util.spec_from_file_location("pkg_without_lib", str(pkg / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="librcs.so is not built"):
        spec.loader.exec_module(mod)


def test_state_file_header_checks_need_no_gpu(rcs, tmp_path):
    """rcs_state_load rejects files that are not state files before any
    device work: bad magic, and a header cut short."""
    p = tmp_path / "junk.mps"
    p.write_bytes(b"NOTASTATEFILE" + bytes(64))
    with pytest.raises(rcs.RcsError, match="magic") as ei:
        rcs.State.load(str(p))
    assert ei.value.status == 1
    p.write_bytes(b"RCSMPS1\n" + bytes(6))
    with pytest.raises(rcs.RcsError, match="truncated"):
        rcs.State.load(str(p))
    with pytest.raises(rcs.RcsError, match="cannot open"):
        rcs.State.load(str(tmp_path / "missing.mps"))


@pytest.mark.parametrize("network", ["snake", "interleaved"])
@pytest.mark.parametrize("rows,cols,cyc,rr,pattern", [(6, 9, 14, 1, "ABCDCDAB"), (6, 9, 14, 1, "EFGH"),
                                                      (6, 9, 20, 1, "ABCDCDAB"), (4, 5, 9, 0, "GHEFDCBA"),
                                                      (3, 4, 8, 0, "EFGH")])
def test_rotated_lattice_schedule_matches_oracle(rcs, rows, cols, cyc, rr, pattern, network):
    """The rotated-lattice circuits (couplers, gate draws, schedule) equal the
    oracle's op by op, for both networks."""
    c = rcs.Circuit(rows, cols, cyc, 7, pattern=pattern, n_removed_random=rr, network=network, lattice="rotated")
    o = OCircuit(rows, cols, cyc, 7, pattern=pattern, n_removed_random=rr, lattice="rotated")
    assert c.n == o.n
    assert np.array_equal(c.one_qubit_gates(), o.one_qubit_draws())
    snake, ops = c.schedule()
    pi, oops = omps.schedule(o, network)
    assert list(snake) == pi
    assert [tuple(x[1:3]) if x[0] == 1 else (x[3],) for x in ops] == \
        [(op[1], 0 if op[2] == "fsim" else 1) if op[0] == "u" else (op[2],) for op in oops]


def test_rotated_lattice_pattern_letters(rcs):
    with pytest.raises(rcs.RcsError, match="A-D"):
        rcs.Circuit(3, 3, 2, 1, pattern="ABE")
    rcs.Circuit(3, 3, 2, 1, pattern="ABEH", lattice="rotated")
    with pytest.raises(rcs.RcsError, match="A-H"):
        rcs.Circuit(3, 3, 2, 1, pattern="ABI", lattice="rotated")


def _write_csv(path, header, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_rocprof_stage_totals(tmp_path, capsys):
    """The profile tooling sums the named kernels' dispatches: counter
    values per counter, or calls and durations from kernel statistics, and
    matches kernel names without namespace or template arguments."""
    from paper_2512_07311_amd import rocprof_summary as rs
    cc = tmp_path / "c"
    cc.mkdir()
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    _write_csv(cc / "x_counter_collection.csv", hdr, [
        ["void rcs::k_jac_gram<32, double>(rcs::JacArgs<double>)", "FETCH_SIZE", 10.5, 0, 100],
        ["void rcs::k_jac_gram<32, double>(rcs::JacArgs<double>)", "FETCH_SIZE", 4.5, 0, 100],
        ["void rcs::k_chol_panel(double*)", "FETCH_SIZE", 2.0, 0, 10],
        ["void rcs::k_chain_gemm(rcs::ChainArgs)", "FETCH_SIZE", 1000.0, 0, 10]])
    rs.stage(str(cc), ["k_jac_gram", "k_chol_panel"])
    assert "stage FETCH_SIZE: 3 dispatches, sum 17.0" in capsys.readouterr().out
    st = tmp_path / "s"
    st.mkdir()
    _write_csv(st / "y_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs",
                                            "Percentage"], [
        ["rcs::k_jac_rotate<32, float>", 4, 4.0e9, 1e9, 1e9, 1e9, 50.0],
        ["rcs::k_jac_rotate<32, double>", 2, 1.0e9, 5e8, 5e8, 5e8, 25.0],
        ["rcs::k_chain_gemm", 1, 1.0e9, 1e9, 1e9, 1e9, 25.0]])
    rs.stage(str(st), ["k_jac_rotate"])
    assert "stage duration: 6 dispatches, total 5.0000 s" in capsys.readouterr().out


def test_bench_traffic_only_for_current_sources(tmp_path, monkeypatch):
    """bench.py reports a stage's HBM traffic only from a committed summary
    whose source hash matches the current kernel sources."""
    import sys
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = bench.stage_hash()
    (prof / "a.md").write_text(
        'stage-traffic-json: {"stage": "factorisation", "workload": "w", "form": "plain", '
        '"source_sha": "%s", "bytes_per_step": 123.0}\n'
        'stage-traffic-json: {"stage": "factorisation", "workload": "w", "form": "plain", '
        '"source_sha": "0000000000000000", "bytes_per_step": 999.0}\n' % sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash reads the sources under ROOT: point it back at the real tree
    monkeypatch.setattr(bench, "stage_hash", lambda: sha)
    assert bench.measured_stage_traffic("w", "plain") == 123.0
    assert bench.measured_stage_traffic("w", "learned") is None
    assert bench.measured_stage_traffic("other", "plain") is None


def test_bench_learned_vs_plain_bar(monkeypatch):
    """The bench line's verdict on the learned form: faster build and step
    at an estimated fidelity within 1% of the plain form's."""
    import math
    import sys
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    import bench
    lf = -29.86
    ok = bench.learned_vs_plain(66.4, 76.6, lf, 52.3, 62.6, lf + math.log(1 - 0.0075))
    assert ok == {"build_faster": True, "step_faster": True, "fest_within_1pct": True, "met": True}
    far = bench.learned_vs_plain(66.4, 76.6, lf, 52.3, 62.6, lf + math.log(1 - 0.02))
    assert far["fest_within_1pct"] is False and far["met"] is False
    slow = bench.learned_vs_plain(66.4, 76.6, lf, 70.0, 80.0, lf)
    assert slow["build_faster"] is False and slow["step_faster"] is False and slow["met"] is False


def test_bench_stage_roofline_arithmetic(monkeypatch):
    """The headline roofline: nominal SVD + QR flops over the probed stage
    time (each class's average launch time times its launches), against the
    fp64 peak."""
    import sys
    import types
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    import bench
    prof = [dict(name="k_chain_gemm", launches=10, timed=10, seconds=1.0),
            dict(name="k_jac_gram", launches=1600, timed=100, seconds=2e-3),        # 20 us each
            dict(name="k_jac_rotate", launches=1600, timed=100, seconds=4e-3),      # 40 us each
            dict(name="k_factor_other", launches=50, timed=50, seconds=5e-3)]        # 100 us each
    inf = types.SimpleNamespace(nominal_svd_flops=6.0e12, nominal_qr_flops=1.0e11)
    r = bench.svd_roofline(prof, inf, 4e-6, 1)
    t = 1600 * 20e-6 + 1600 * 40e-6 + 50 * 100e-6
    assert abs(r["kernel_seconds_per_step"] - t) < 1e-12
    assert abs(r["achieved"] - 6.1e12 / t / 1e12) < 1e-9
    assert abs(r["frac"] - 6.1e12 / t / 78.6e12) < 1e-12
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["per_kernel"]["k_jac_rotate"]["launches_per_step"] == 1600
