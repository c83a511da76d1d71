"""Persistence and independent shot-range jobs (Section 3.2, stages 2-3):
a saved state loads back bit for bit, separate processes sampling disjoint
shot ranges from the file merge into exactly the shots of one call, an
independent numpy reader of the file format recovers the state (the
oracle's sampler on it draws the same shots), and corrupt files are
refused."""
import os
import struct
import subprocess
import sys

import numpy as np
import pytest

from oracle import sample as osample
from tests.gpu_util import get_rcs, oracle_state_from, compare_shots

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def env():
    return get_rcs()


@pytest.fixture(scope="module")
def saved(env, tmp_path_factory):
    rcs, torch = env
    st = rcs.State.build(rcs.Circuit(5, 6, 10, 4, network="interleaved"), 64, 1e-9)
    path = str(tmp_path_factory.mktemp("state") / "rcs30.mps")
    st.save(path)
    return st, path


def read_state_file(path):
    """The documented file layout, read with numpy only."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"RCSMPS1\n"
    version, n, canonical, _ = struct.unpack_from("<4i", raw, 8)
    (log_fest,) = struct.unpack_from("<d", raw, 24)
    off = 32
    dims = np.frombuffer(raw, dtype="<i4", count=n + 1, offset=off)
    off += 4 * (n + 1)
    snake = np.frombuffer(raw, dtype="<i4", count=n, offset=off)
    off += 4 * n
    tens = []
    for k in range(n):
        cnt = int(dims[k]) * 2 * int(dims[k + 1])
        tens.append(np.frombuffer(raw, dtype="<c16", count=cnt, offset=off).reshape(dims[k], 2, dims[k + 1]))
        off += 16 * cnt
    (stored,) = struct.unpack_from("<Q", raw, off)
    assert off + 8 == len(raw)
    # FNV-1a over 64-bit words, then trailing bytes
    h, mask = 1469598103934665603, (1 << 64) - 1
    words = np.frombuffer(raw[:off - off % 8], dtype="<u8")
    for w in words.tolist():
        h = ((h ^ w) * 1099511628211) & mask
    for b in raw[off - off % 8:off]:
        h = ((h ^ b) * 1099511628211) & mask
    assert h == stored
    return version, n, canonical, log_fest, dims, snake, tens


def _shots(torch, st, first, count, seed):
    bits = torch.zeros(count, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(count, dtype=torch.float64, device="cuda")
    st.sample(bits, l2, seed=seed, first_shot=first)
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint64), l2.cpu().numpy()


def test_load_is_bit_identical(env, saved):
    rcs, torch = env
    st, path = saved
    ld = rcs.State.load(path)
    a, b = st.to_host(), ld.to_host()
    assert list(a[0]) == list(b[0]) and list(a[1]) == list(b[1])
    assert all(np.array_equal(x, y) for x, y in zip(a[2], b[2]))
    assert ld.info().log_fidelity_est == st.info().log_fidelity_est
    assert ld.info().canonical == 1


def test_independent_jobs_merge_into_one_call(env, saved, tmp_path):
    """Two sequential processes, each loading the file and sampling its own
    shot range, reproduce one in-process call over the whole range."""
    rcs, torch = env
    st, path = saved
    n_all, split, seed = 20000, 12345, 77
    ref_b, ref_l = _shots(torch, st, 0, n_all, seed)
    outs = []
    for first, count in ((0, split), (split, n_all - split)):
        out = str(tmp_path / ("shard_%d.npz" % first))
        r = subprocess.run([sys.executable, "-m", "paper_2512_07311_amd.shard_sample", path, str(first), str(count),
                            str(seed), out], cwd=ROOT, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(np.load(out))
    bits = np.concatenate([o["bits"] for o in outs])
    l2 = np.concatenate([o["log2p"] for o in outs])
    assert np.array_equal(bits, ref_b)
    assert np.array_equal(l2, ref_l)


def test_file_read_independently_samples_like_the_gpu(env, saved):
    """The file, parsed by numpy from the documented layout, is the state:
    the oracle's sampler on it draws the GPU's shots."""
    rcs, torch = env
    st, path = saved
    version, n, canonical, log_fest, dims, snake, tens = read_state_file(path)
    assert (version, n, canonical) == (1, 30, 1)
    assert log_fest == st.info().log_fidelity_est
    o = oracle_state_from((dims, snake, [np.array(t) for t in tens]))
    ob, _, tight = osample.sample(o, 2000, 91)
    gb, _ = _shots(torch, st, 0, 2000, 91)
    ok, n_exempt, _ = compare_shots(gb, ob, tight)
    assert ok and n_exempt == 0


def test_corrupt_files_are_refused(env, saved, tmp_path):
    rcs, torch = env
    _, path = saved
    raw = bytearray(open(path, "rb").read())
    bad = tmp_path / "flipped.mps"
    raw2 = bytearray(raw)
    raw2[len(raw2) // 2] ^= 0x10
    bad.write_bytes(bytes(raw2))
    with pytest.raises(rcs.RcsError, match="checksum") as ei:
        rcs.State.load(str(bad))
    assert ei.value.status == 1
    short = tmp_path / "short.mps"
    short.write_bytes(bytes(raw[:len(raw) // 3]))
    with pytest.raises(rcs.RcsError, match="truncated"):
        rcs.State.load(str(short))
