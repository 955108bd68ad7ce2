"""Oracle of the learned-culling part, in plain numpy float64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network is Linear(16, 64) - ReLU - Linear(64, 64) - ReLU - Linear(64, 1)
trained by mean squared error with Adam; features summarise a replica's
trajectory at a checkpoint; culling ranks replicas and lets the bottom half
copy the top half.  The paper gives none of this (its trials are independent
and read out at their end, Section III); every definition here is the
reading the library documents, restated plainly.
"""
import math

import numpy as np

from . import philox, fields

NF, NH = 16, 64
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
TAG_MLP = 3


def unpack(theta):
    """Split the flat parameter vector into named arrays (views)."""
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def init_params(seed):
    """Kaiming-uniform weights sqrt(6 / fan_in) * (2u - 1), u = (Philox word
    >> 8) * 2^-24 with counter (index >> 2, 0, 0, 3); zero biases."""
    theta = np.zeros(N_PARAMS)
    k = 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        if name.startswith("W"):
            fan_in = shape[-1] if name != "W3" else NH
            a = math.sqrt(6.0 / fan_in)
            for i in range(k, k + size):
                word = int(philox(seed, (i >> 2, 0, 0, TAG_MLP))[i & 3])
                u = (word >> 8) * 2.0**-24
                theta[i] = a * (2.0 * u - 1.0)
        k += size
    return theta


def normalise(x, mean=None, std=None):
    x = np.asarray(x, np.float64)
    if mean is None:
        return x
    return (x - np.asarray(mean, np.float64)) / np.asarray(std, np.float64)


def standardize_groups(x, n_groups, rows, cols):
    """Per group and column: (x - mean) / std over the group's rows, with the
    population standard deviation floored at 1e-6, in float64, returned as
    float32 (the standing of each row within its population)."""
    a = np.asarray(x, np.float64).reshape(n_groups, rows, cols)
    mu = a.mean(axis=1, keepdims=True)
    sd = np.sqrt(((a - mu) ** 2).mean(axis=1, keepdims=True))
    sd = np.maximum(sd, 1e-6)
    return ((a - mu) / sd).astype(np.float32).reshape(np.shape(x))


def forward(theta, z):
    """Network output for inputs z [B][16] (already normalised)."""
    p = unpack(theta)
    a1 = z @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    return h2 @ p["W3"] + p["b3"][0]


def loss_grad(theta, z, target):
    """L = mean_b (y_b - t_b)^2 and dL/dtheta by the chain rule, layer by layer."""
    p = unpack(theta)
    B = z.shape[0]
    a1 = z @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"] + p["b3"][0]
    err = y - target
    loss = float(np.mean(err**2))
    dy = 2.0 * err / B                    # dL/dy
    g = {"W3": h2.T @ dy, "b3": np.array([dy.sum()])}
    d2 = np.outer(dy, p["W3"]) * (a2 > 0)  # dL/da2
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (a1 > 0)         # dL/da1
    g["W1"] = d1.T @ z
    g["b1"] = d1.sum(axis=0)
    grad = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss, grad


def adam_step(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015) with bias-corrected moments; returns new arrays."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad**2
    m_hat = m / (1.0 - beta1**step)
    v_hat = v / (1.0 - beta2**step)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def new_track(R):
    return dict(h_min=np.zeros(R, np.int64), h_prev=np.zeros(R, np.int64), flips_total=np.zeros(R, np.uint64),
                checkpoints=np.zeros(R, np.int32), last_improve=np.zeros(R, np.int32))


def features(dims, w, spins, energy, window_flips, track, sweeps_done, window, n_sweeps, beta, n_checkpoints):
    """The 16 checkpoint features of each replica; updates `track` in place.

    0 H/|E|; 1 lowest checkpoint H/|E|; 2 (H - H_prev)/|E| with H_prev = 0 at
    the first checkpoint; 3 window flips / (n window); 4 flips so far /
    (n sweeps_done); 5 beta; 6 sweeps_done / S; 7..13 fraction of sites with
    s_i f_i = -6, -4, ..., 6; 14 ln beta; 15 checkpoints since the lowest
    energy last decreased, / n_checkpoints."""
    R, n = spins.shape
    E = len(dims) * n
    out = np.zeros((R, NF))
    for r in range(R):
        H = int(energy[r])
        first = track["checkpoints"][r] == 0
        h_prev = 0 if first else int(track["h_prev"][r])
        h_min_old = None if first else int(track["h_min"][r])
        cp = int(track["checkpoints"][r]) + 1
        if h_min_old is None or H < h_min_old:
            track["h_min"][r] = H
            track["last_improve"][r] = cp
        track["flips_total"][r] += np.uint64(window_flips[r])
        sf = spins[r].astype(np.int64) * fields(dims, w, spins[r])
        hist = [np.count_nonzero(sf == v) / n for v in (-6, -4, -2, 0, 2, 4, 6)]
        out[r] = [H / E, int(track["h_min"][r]) / E, (H - h_prev) / E, int(window_flips[r]) / (n * window),
                  int(track["flips_total"][r]) / (n * sweeps_done), beta, sweeps_done / n_sweeps] + hist + \
                 [math.log(beta), (cp - int(track["last_improve"][r])) / n_checkpoints]
        track["h_prev"][r] = H
        track["checkpoints"][r] = cp
    return out


def cull_order(score):
    """Replica indices from best to worst: higher score first, ties by lower
    index, NaN last."""
    score = np.asarray(score, np.float64)
    keyed = [((1, 0.0) if math.isnan(s) else (0, -s), i) for i, s in enumerate(score)]
    return np.array([i for _, i in sorted(keyed)], np.int64)


def cull_clone(order, spins, track=None):
    """The j-th worst replica becomes a copy of the j-th best (in place)."""
    R = len(order)
    for j in range(R // 2):
        src, dst = order[j], order[R - 1 - j]
        spins[dst] = spins[src]
        if track is not None:
            for key in track:
                track[key][dst] = track[key][src]


def final_cut_score(w_total, n_edges, gain, feats):
    """Predicted final cut / |E| = cut now / |E| + gain, with
    cut now = (W_total - H) / 2 and feature 0 = H / |E|."""
    return 0.5 * (w_total / n_edges - np.asarray(feats, np.float64)[:, 0]) + np.asarray(gain, np.float64)
