"""Training driver of the rank-prediction network (orchestration only).

Every arithmetic step runs in librcs kernels: spectrum features and targets,
forward/backward passes and Adam updates.  This module only moves device
tensors between those calls.

Data: the per-update singular spectra a plain fp64 build logs
(``State.build(..., log_spectra=True)``).  The features of an update are the
kept spectrum of the previous truncation at the same bond (zero histogram for
a bond's first truncation) plus bond and cycle; the targets are the discarded
weight fractions of the update's own full spectrum at 32 relative ranks.
"""
import numpy as np

import paper_2512_07311_amd as rcs


def dataset(records, n_sites, n_cycles, torch):
    """(X [N, 66], Y [N, 32]) float32 device tensors from logged records."""
    n = len(records)
    X = torch.zeros(n, 66, dtype=torch.float32, device="cuda")
    Y = torch.zeros(n, 32, dtype=torch.float32, device="cuda")
    last = {}
    empty = torch.zeros(1, dtype=torch.float64, device="cuda")
    for r, rec in enumerate(records):
        prev = last.get(rec["pos"])
        if prev is None:
            rcs.spectrum_features(empty, 0, rec["pos"], n_sites, rec["cycle"], n_cycles, X[r])
        else:
            rcs.spectrum_features(prev, prev.numel(), rec["pos"], n_sites, rec["cycle"], n_cycles, X[r])
        vals = torch.from_numpy(np.ascontiguousarray(rec["values"])).cuda()
        rcs.spectrum_targets(vals, rec["m"], Y[r])
        last[rec["pos"]] = vals[:rec["kept"]].contiguous()
    torch.cuda.synchronize()
    return X, Y


def he_init(seed):
    """He-normal weights, zero biases, packed W1,b1,W2,b2,W3,b3 (float32)."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in [(128, 66), (128, 128), (32, 128)]:
        parts.append((g.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(X, Y, torch, steps=2000, batch=256, lr=1e-3, init=None, seed=0, log_every=0):
    """Adam on the mean-squared error; returns (weights float32 ndarray, losses)."""
    w = torch.from_numpy(init if init is not None else he_init(seed)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    grad = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    g = np.random.default_rng(seed + 1)
    losses = []
    order = g.permutation(n)
    pos = 0
    for step in range(1, steps + 1):
        if pos + batch > n:
            order = g.permutation(n)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + min(batch, n)]).cuda()
        pos += batch
        xb = X.index_select(0, idx).contiguous()
        yb = Y.index_select(0, idx).contiguous()
        rcs.mlp_backward(w, xb, yb, grad, loss)
        rcs.mlp_adam(w, grad, m, v, step, lr=lr)
        if log_every and (step % log_every == 0 or step == 1):
            losses.append((step, float(loss.item())))
    torch.cuda.synchronize()
    return w.cpu().numpy(), losses


def predict(w, X, torch):
    out = torch.zeros(X.shape[0], 32, dtype=torch.float32, device="cuda")
    rcs.mlp_forward(torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda(), X, out)
    return out
