"""Rank-prediction network, fp64 reference (forward, backward, Adam).

The learned part predicts, per bond, how much discarded weight each kept
rank would leave, from the singular spectrum the method itself produced at
that bond's previous truncation.

Features (66): a 64-bin histogram of log10(s^2 / sum s^2) of the bond's kept
spectrum at its previous truncation (bins of 0.25 decade over [-16, 0);
values below -16 go to bin 0, values >= 0 to bin 63; normalised to sum 1;
all zeros when the bond was never truncated), then bond/(n-2) and
cycle/n_cycles.

Network: Linear(66,128) - ReLU - Linear(128,128) - ReLU - Linear(128,32).

Targets (32): y_j = log10(max(tail(ceil(f_j m)) / w, 1e-20)) at f_j = j/32,
j = 1..32, where m is the number of singular values of the two-site matrix
and tail/w the discarded-weight fraction of the rank rule.

Inference: y(f) is y_j linearly interpolated in f with y(0) = 0; f* is the
first f where y(f) <= log10(eps); k_hat = ceil(m f*) clamped to [1, chi];
the predicted discarded fraction at rank k is 10^y(k/m).

Training: mean-squared error over batch and outputs; Adam (lr 1e-3,
beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
"""
import math
import numpy as np

N_IN, N_HID, N_OUT = 66, 128, 32
N_BINS = 64
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)),
          ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]


def n_params():
    return sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


# ------------------------------------------------------------------ features
def spectrum_histogram(kept):
    kept = np.asarray(kept, dtype=np.float64)
    h = np.zeros(N_BINS)
    if kept.size == 0:
        return h
    s2 = kept ** 2
    tot = s2.sum()
    for v in s2:
        x = math.log10(v / tot) if v > 0 else -1e300
        b = int(math.floor((x + 16.0) / 0.25))
        h[min(max(b, 0), N_BINS - 1)] += 1.0
    return h / h.sum()


def features(kept_prev, bond, n_sites, cycle, n_cycles):
    h = spectrum_histogram(kept_prev) if kept_prev is not None else np.zeros(N_BINS)
    return np.concatenate([h, [bond / max(n_sites - 2, 1), cycle / max(n_cycles, 1)]])


def targets(spectrum, floor=1e-24):
    s2 = np.asarray(spectrum, dtype=np.float64) ** 2
    w = s2.sum()
    s2z = np.where(s2 <= floor * w, 0.0, s2)
    m = len(s2z)
    tail = np.zeros(m + 1)
    tail[:m] = np.cumsum(s2z[::-1])[::-1]
    y = np.empty(N_OUT)
    for j in range(1, N_OUT + 1):
        k = min(m, int(math.ceil(j / N_OUT * m)))
        y[j - 1] = math.log10(max(tail[k] / w, 1e-20))
    return y


# -------------------------------------------------------------- inference
def interp_y(y, f):
    fs = np.concatenate([[0.0], np.arange(1, N_OUT + 1) / N_OUT])
    ys = np.concatenate([[0.0], y])
    return float(np.interp(f, fs, ys))


def predict_rank(y, m, chi, eps):
    fs = np.concatenate([[0.0], np.arange(1, N_OUT + 1) / N_OUT])
    ys = np.concatenate([[0.0], np.asarray(y, dtype=np.float64)])
    target = math.log10(eps) if eps > 0 else -20.0
    fstar = 1.0
    for j in range(1, len(fs)):
        if ys[j] <= target:
            y0, y1 = ys[j - 1], ys[j]
            fstar = fs[j] if y1 == y0 else fs[j - 1] + (target - y0) / (y1 - y0) * (fs[j] - fs[j - 1])
            break
    k = int(math.ceil(m * fstar - 1e-12))
    return max(1, min(int(chi), k, m))


def predicted_eps(y, k, m):
    return 10.0 ** interp_y(y, k / m)


# ------------------------------------------------------------- fwd / bwd
def forward(p, x):
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"].T + p["b3"]
    return out, (x, z1, h1, z2, h2)


def loss(p, x, y):
    out, _ = forward(p, x)
    return float(np.mean((out - y) ** 2))


def backward(p, x, y):
    """Gradient of the mean-squared error with respect to every parameter."""
    out, (x, z1, h1, z2, h2) = forward(p, x)
    d_out = 2.0 * (out - y) / out.size
    g = {}
    g["W3"] = d_out.T @ h2
    g["b3"] = d_out.sum(axis=0)
    d_h2 = d_out @ p["W3"]
    d_z2 = d_h2 * (z2 > 0)
    g["W2"] = d_z2.T @ h1
    g["b2"] = d_z2.sum(axis=0)
    d_h1 = d_z2 @ p["W2"]
    d_z1 = d_h1 * (z1 > 0)
    g["W1"] = d_z1.T @ x
    g["b1"] = d_z1.sum(axis=0)
    return g


def adam_step(flat, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step >= 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
