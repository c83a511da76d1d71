"""GPU parity of the learned path's decisions and of the multi-panel range
finder, through the C-ABI.

* Every randomized split of a learned build is recomputed by the oracle from
  the values the build logged: network inputs and outputs, predicted rank,
  sketch width, randomized rank and discarded fraction, predicted fraction
  at the kept rank, and the judge's accept / early-reject decision.
* The range finder with sketches of several 64-column panels (block
  Gram-Schmidt across panels) against the oracle's randomized SVD, and the
  orthonormality of its basis.
* A split-bf16 learned build at 22 qubits and bond cap 256 (sketches of up to
  five panels) against the oracle's exact state, beside the rsvd-at-cap and
  plain builds of the same circuit (the three-way comparison of the learned
  part's gain), and the learned form with the fp32 SVD of cap-limited cuts.
"""
import math

import numpy as np
import pytest

from oracle import mlp as omlp, rsvd as orsvd
from tests import inputs
from tests.gpu_util import get_rcs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return get_rcs()


def _cap(pos, n, chi):
    """Bond cap of the bond right of position pos."""
    return min(chi, 2 ** min(pos + 1, n - pos - 1))


def _margin(total, s, k, eps):
    """Relative distance of the rank rule's comparison at k from its threshold."""
    kept = float(np.sum(np.asarray(s[:k], dtype=np.float64) ** 2))
    return abs(total - kept - eps * total) / total


def test_learned_decisions_match_oracle(env):
    from paper_2512_07311_amd import learn
    rcs, torch = env
    cyc, chi, eps, tau, p = 10, 32, 1e-9, 1e-6, 4
    c = rcs.Circuit(4, 5, cyc, 41)
    plain = rcs.State.build(c, chi, eps, log_spectra=True)
    X, Y = learn.dataset(plain.spectra(), c.n, cyc, torch)
    w, _ = learn.train(X, Y, torch, steps=300, batch=128, seed=3)
    st = rcs.State.build(c, chi, eps, rank_mode=1, mlp_weights=w, fallback_tau=tau, rsvd_oversample=p,
                         log_spectra=True)
    log = st.rsvd_log()
    spectra = st.spectra()
    upd = st.updates()
    assert len(spectra) == len(upd) == c.n_updates
    assert len(log) > 10
    params = omlp.unpack(np.asarray(w, dtype=np.float64))
    n_acc = n_rej = n_early = n_margin = 0
    for rec in log:
        u, i = rec["update"], rec["pos"]
        cap = _cap(i, c.n, chi)
        # network inputs: the kept spectrum of this bond's previous truncation
        prev = None
        for r in spectra[:u]:
            if r["pos"] == i:
                prev = r["values"][:r["kept"]]
        feat = omlp.features(prev, i, c.n, rec["cycle"], cyc)
        assert np.abs(rec["feat"] - feat).max() < 1e-6, (u, i)
        y_ref, _ = omlp.forward(params, feat[None, :])
        y = rec["y"].astype(np.float64)
        assert np.abs(y - y_ref[0]).max() < 1e-4 * max(1.0, np.abs(y_ref).max()), (u, i)
        # predicted rank and sketch width (same fp64 arithmetic on the same outputs)
        assert rec["k_hat"] == omlp.predict_rank(y, rec["m"], cap, eps), (u, i)
        assert rec["l"] == min(rec["k_hat"] + p, rec["m"])
        if rec["early"]:
            k_forced = min(rec["l"], cap)
            ep = omlp.predicted_eps(y, k_forced, rec["m"])
            assert rec["k"] == k_forced
            assert rec["eps_pred"] == pytest.approx(ep, rel=1e-12)
            assert rec["outside"] > eps * rec["total"]
            assert not orsvd.judge_accepts(rec["outside"] / rec["total"], eps, ep, tau)
            assert upd[u][6] == 2
            n_early += 1
            continue
        vals = rec["values"]
        assert len(vals) == rec["l"]
        k_ref, e_ref = orsvd.rsvd_rank(vals, rec["total"], cap, eps)
        if rec["k"] != k_ref:
            # only a comparison within rounding of its threshold may differ
            assert min(_margin(rec["total"], vals, rec["k"], eps),
                       _margin(rec["total"], vals, k_ref, eps)) < 1e-12, (u, i, rec["k"], k_ref)
            n_margin += 1
            continue
        assert rec["eps_rand"] == pytest.approx(e_ref, rel=1e-9, abs=1e-15), (u, i)
        ep = omlp.predicted_eps(y, rec["k"], rec["m"])
        assert rec["eps_pred"] == pytest.approx(ep, rel=1e-12), (u, i)
        assert rec["accepted"] == orsvd.judge_accepts(rec["eps_rand"], eps, rec["eps_pred"], tau)
        assert rec["accepted"] == orsvd.judge_accepts(e_ref, eps, ep, tau) or \
            abs(e_ref - (max(eps, ep) + tau)) < 1e-12
        assert upd[u][6] == (1 if rec["accepted"] else 2)
        if rec["accepted"]:
            assert upd[u][5] == rec["k"]
            n_acc += 1
        else:
            n_rej += 1
    print("randomized splits: %d accepted, %d rejected after the projected SVD, %d early, %d at margin"
          % (n_acc, n_rej, n_early, n_margin))
    assert n_acc > 0 and n_acc + n_rej + n_early + n_margin == len(log)
    assert n_margin <= 1
    inf = st.info()
    assert inf.n_rsvd_accepted == n_acc
    assert inf.n_fallbacks == n_rej + n_early


@pytest.mark.parametrize("ln,cnt,l,q", [(300, 260, 65, 2), (1100, 900, 200, 1), (2048, 2048, 1040, 2)])
def test_rsvd_multi_panel_matches_oracle(env, ln, cnt, l, q):
    """Sketches of 2, 4 and 17 column panels: the basis stays orthonormal to
    fp64 rounding across panels, and the singular values of Q^H M agree with
    the oracle's randomized SVD on the same sketch to the fp32 accuracy of
    the range finder's products."""
    rcs, torch = env
    spec = 0.995 ** np.arange(min(ln, cnt))          # every panel carries weight
    M = inputs.planted_matrix(ln, cnt, spec, seed=7)
    x = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
    s = torch.zeros(l, dtype=torch.float64, device="cuda")
    fro2 = rcs.rsvd(x, l, q, 91, 5, s)
    qd = torch.zeros(l, ln, dtype=torch.complex128, device="cuda")
    rcs.rsvd_basis(x, l, q, 91, 5, qd)
    torch.cuda.synchronize()
    Q = qd.cpu().numpy().T                           # ln x l
    orth = np.abs(Q.conj().T @ Q - np.eye(l)).max()
    assert orth < 1e-13 * math.sqrt(ln), orth
    _, s_ref, _ = orsvd.rsvd(M, l, q, 91, 5)
    got = s.cpu().numpy()
    assert abs(fro2 - np.sum(np.abs(M) ** 2)) < 1e-12 * fro2
    assert np.abs(got - s_ref).max() < 2e-5 * s_ref[0], np.abs(got - s_ref).max()
    # the weight the basis captures equals that of the oracle's basis
    cap_gpu = np.sum(np.abs(Q.conj().T @ M) ** 2) / fro2
    assert abs(cap_gpu - np.sum(s_ref ** 2) / fro2) < 1e-5
    # interlacing with the exact spectrum
    assert np.all(got <= spec[:l] * (1 + 1e-12) + 1e-12)


def test_split_bf16_learned_build_22q_against_exact_state(env):
    """22 qubits (4x6 grid minus two sites), 12 cycles, bond cap 256, eps
    1e-8.  Learned (split-bf16 contractions, network ranks trained on another
    seed's spectra), rsvd-at-cap and plain fp64 builds, each scored by its
    true fidelity |<psi_exact|psi>|^2 against the oracle's dense state.  The
    learned build must accept randomized splits wider than one panel, keep
    F_est faithful to its true fidelity (same band as the plain build) and
    lose little true fidelity against the plain build."""
    from oracle import circuit as oc, dense
    from paper_2512_07311_amd import learn
    rcs, torch = env
    rows, cols, cyc, chi, eps = 4, 6, 12, 256, 1e-8
    removed = [22, 23]
    train = rcs.Circuit(rows, cols, cyc, 72, removed=removed)
    c = rcs.Circuit(rows, cols, cyc, 71, removed=removed)
    assert c.n == 22
    tst = rcs.State.build(train, chi, eps, log_spectra=True)
    X, Y = learn.dataset(tst.spectra(), train.n, cyc, torch)
    w, _ = learn.train(X, Y, torch, steps=1500, batch=256, seed=4)
    del tst
    plain = rcs.State.build(c, chi, eps)
    learned = rcs.State.build(c, chi, eps, contraction="split_bf16", rank_mode=1, mlp_weights=w,
                              fallback_tau=1e-6)
    atcap = rcs.State.build(c, chi, eps, contraction="split_bf16", rank_mode=2, fallback_tau=1e-6)
    learned32 = rcs.State.build(c, chi, eps, contraction="split_bf16", rank_mode=1, mlp_weights=w,
                                fallback_tau=1e-6, svd_precision="f32")
    psi = dense.simulate(oc.Circuit(rows, cols, cyc, 71, removed=removed))
    bits = torch.arange(1 << c.n, dtype=torch.int64, device="cuda")

    def fid(st):
        amps = torch.zeros(1 << c.n, 2, dtype=torch.float64, device="cuda")
        st.amplitudes(bits, amps)
        a = amps.cpu().numpy()
        return abs(np.vdot(psi, a[:, 0] + 1j * a[:, 1])) ** 2

    rows_out = []
    for name, st in (("plain", plain), ("learned", learned), ("rsvd-at-cap", atcap), ("learned-f32", learned32)):
        inf = st.info()
        rows_out.append((name, inf.build_seconds, inf.n_rsvd_accepted, inf.n_fallbacks,
                         math.exp(inf.log_fidelity_est), fid(st)))
    for r in rows_out:
        print("%-12s build %.2f s  accepted %4d  fall-backs %4d  F_est %.5f  F_true %.5f" % r)
    i32 = learned32.info()
    print("learned-f32: %d fp32 splits, %d redone" % (i32.n_svd_f32, i32.n_svd_f32_redone))
    _, _, _, _, fe_p, ft_p = rows_out[0]
    _, _, acc_l, _, fe_l, ft_l = rows_out[1]
    assert learned.info().canonical == 1
    wide = [r for r in learned.rsvd_log() if r["accepted"] and r["l"] > 64]
    assert acc_l > 0 and len(wide) > 0
    r_plain = ft_p / fe_p
    assert 0.5 * r_plain <= ft_l / fe_l <= 2.0 * r_plain
    assert ft_l >= 0.5 * ft_p
    # the fp32-SVD learned form: cap-limited cuts through the fp32 Jacobi,
    # estimated fidelity within 1% of the plain build's and true fidelity
    # no lower than 99% of it
    _, _, _, _, fe_32, ft_32 = rows_out[3]
    assert i32.n_svd_f32 > 0
    assert abs(fe_32 / fe_p - 1.0) <= 0.01
    assert ft_32 >= 0.99 * ft_p
