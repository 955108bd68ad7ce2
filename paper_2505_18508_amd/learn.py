"""Learned replica culling on top of the sweep kernels.

A trial (paper, Section III) is a run of S sweeps read out at its end.  Here
R trials run together and, every `window` sweeps, each replica's trajectory
features go through a small network that predicts its end-of-trial cut
(label "final"), or the cut it will still gain (label "gain", scored as
current cut plus predicted gain), or its end-of-trial cut's standing among
the run's replicas from features standardised within the checkpoint's
population (label "relative"); the score ranks the replicas, and the
lower half is replaced by copies of the upper half.  Every
replica keeps its own Philox stream, so copies diverge at once.  The plain
form (no culling) runs the same windows and is what the learned form is
compared with, eq. (3)-(5) applied to both.

All arithmetic runs in the library's HIP kernels; this module sequences
them on one stream and holds the buffers (torch device tensors).
"""
import math
import time

import numpy as np

from . import (adam_step, create_graph, cull_clone, cut_labels, energy_score, feature_stats, features,
               final_cut_score, mlp_forward, mlp_init, mlp_loss_grad, mlp_workspace_floats, new_track, run_trials,
               schedule_beta, standardize_groups)
from . import metrics

METHODS = ("plain", "learned", "energy")


LABELS = ("final", "gain", "relative")


class Model:
    """Network parameters, the feature normalisation they were trained with,
    and what the output means: "final" = end-of-trial cut / |E|; "gain" = cut
    still to come / |E| (the score adds the current cut back); "relative" =
    end-of-trial cut standardised over the run's replicas, read from features
    standardised over the replicas at the same checkpoint (mean 0, std 1
    then stand for no further normalisation)."""

    def __init__(self, params, mean, std, label="final"):
        if label not in LABELS:
            raise ValueError("label must be one of %s" % (LABELS,))
        self.params, self.mean, self.std, self.label = params, mean, std, label

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), mean=self.mean.cpu().numpy(), std=self.std.cpu().numpy(),
                 label=np.array(LABELS.index(self.label)))

    @classmethod
    def load(cls, path, device="cuda"):
        import torch

        with np.load(path, allow_pickle=False) as z:
            arrs = [torch.from_numpy(z[k]).to(device) for k in ("params", "mean", "std")]
            return cls(*arrs, label=LABELS[int(z["label"])])


def checkpoints(n_sweeps, window):
    """Sweep counts after which the replicas are ranked (not after the last sweep)."""
    return [e for e in range(window, n_sweeps, window)]


def anneal(graph, n_replicas, n_sweeps, seed, schedule="geometric", beta0=0.05, beta1=4.0, window=2000,
           method="plain", model=None, layout="auto", on_checkpoint=None, on_window=None, stream=None):
    """One batch of R trials of S sweeps.  method: plain | learned | energy.

    Returns dict(spins, cut, energy, orders, seconds) with device tensors;
    `orders` lists each checkpoint's ranking (device int32 [R]) when culling;
    `on_checkpoint(k, sweeps_done, feats)` is called with each checkpoint's
    features (plain and learned forms compute them); `on_window(k, end, cut)`
    with the cuts at the end of every window (before any culling)."""
    import torch

    if method not in METHODS:
        raise ValueError("method must be one of %s" % (METHODS,))
    if method == "learned" and model is None:
        raise ValueError("the learned form needs a model")
    dev = torch.device("cuda")
    R, n = n_replicas, graph.n
    spins = torch.zeros((R, n), dtype=torch.int8, device=dev)
    cut = torch.zeros(R, dtype=torch.int64, device=dev)
    energy = torch.zeros(R, dtype=torch.int64, device=dev)
    flips = torch.zeros(R, dtype=torch.int32, device=dev)
    track = new_track(R, dev)
    feats = torch.zeros((R, 16), dtype=torch.float32, device=dev)
    score = torch.zeros(R, dtype=torch.float32, device=dev)
    cps = checkpoints(n_sweeps, window)
    orders = []
    want_features = method == "learned" or on_checkpoint is not None
    st = torch.cuda.current_stream() if stream is None else stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(st)
    begin = 0
    for k, end in enumerate(cps + [n_sweeps]):
        run_trials(graph, spins, seed, n_sweeps, begin, end, schedule, beta0, beta1, None, begin == 0, layout,
                   cut, energy, flips, stream=st)
        if on_window is not None:
            on_window(k, end, cut)
        if end < n_sweeps:
            if want_features:
                beta = schedule_beta(n_sweeps, end - 1, schedule, beta0, beta1)
                features(graph, spins, energy, flips, track, end, end - begin, n_sweeps, beta, len(cps), feats,
                         stream=st)
                if on_checkpoint is not None:
                    on_checkpoint(k, end, feats)
            if method != "plain":
                if method == "learned":
                    if model.label == "relative":  # each replica's standing at this checkpoint
                        standardize_groups(feats, 1, R, 16, stream=st)
                    mlp_forward(model.params, feats, score, mean=model.mean, std=model.std, stream=st)
                    if model.label == "gain":
                        final_cut_score(graph, score, feats, score, stream=st)
                else:
                    energy_score(energy, score, stream=st)
                order = torch.empty(R, dtype=torch.int32, device=dev)
                cull_clone(score, spins, track, order, stream=st)
                orders.append(order)
        begin = end
    t1.record(st)
    t1.synchronize()
    return dict(spins=spins, cut=cut, energy=energy, orders=orders, seconds=t0.elapsed_time(t1) / 1e3)


def trajectories(instances, n_replicas, n_sweeps, window, schedule="geometric", beta0=0.05, beta1=4.0,
                 layout="auto", label="final", log=None):
    """Training rows from plain runs: features at every checkpoint, labelled
    with the end-of-trial cut / |E| (label "final"), with the cut still to
    come, (final cut - cut at the checkpoint) / |E| (label "gain"), or with
    the end-of-trial cut standardised over the run's replicas, the features
    standardised over the replicas of their checkpoint (label "relative").
    instances: [(dims, weight_seed, run_seed)].  Returns device tensors
    X [N][16], Y [N] (instance-major, then checkpoint, then replica)."""
    import torch

    xs, ys = [], []
    R = n_replicas
    for dims, wseed, rseed in instances:
        g = create_graph(dims, wseed)
        rows, cuts = [], {}
        out = anneal(g, R, n_sweeps, rseed, schedule, beta0, beta1, window, "plain", layout=layout,
                     on_checkpoint=lambda k, e, f: rows.append(f.clone()),
                     on_window=lambda k, e, c: cuts.__setitem__(k, c.clone()))
        final = out["cut"]
        if log:
            log("  training run: %s weight seed %d, %.1f s" % ("x".join(map(str, dims)), wseed, out["seconds"]))
        if label == "relative":
            X = torch.cat(rows)
            standardize_groups(X, len(rows), R, 16)
            y = torch.empty(R, dtype=torch.float32, device=final.device)
            cut_labels(final, y)
            standardize_groups(y, 1, R, 1)
            xs.append(X)
            ys.extend([y] * len(rows))
        else:
            xs.extend(rows)
            for k in range(len(rows)):
                y = torch.empty(R, dtype=torch.float32, device=final.device)
                cut_labels(final, y, cuts[k] if label == "gain" else None, 1.0 / g.n_edges)
                ys.append(y)
        g.close()
    return torch.cat(xs), torch.cat(ys)


def train(X, Y, epochs=20, batch=8192, lr=1e-3, seed=3, log=None, label="final"):
    """Adam on the mean squared error, with the library's forward/backward
    kernels; deterministic given the seed (fixed shuffles, fixed-order
    reductions).  Returns (Model, per-epoch mean losses)."""
    import torch

    dev = X.device
    N = X.shape[0]
    mean = torch.zeros(16, dtype=torch.float32, device=dev)
    std = torch.ones(16, dtype=torch.float32, device=dev)
    if label != "relative":  # relative rows are standardised within their population already
        feature_stats(X, mean, std)
    params = torch.zeros(5313, dtype=torch.float32, device=dev)
    mlp_init(seed, params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    starts = list(range(0, N, batch))
    # one loss slot per step, read back once per epoch (no host sync per step)
    losses = torch.zeros(len(starts), dtype=torch.float32, device=dev)
    ws = torch.zeros(mlp_workspace_floats(batch), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    step = 0
    history = []
    for epoch in range(epochs):
        perm = torch.from_numpy(rng.permutation(N).astype(np.int32)).to(dev)
        for k, start in enumerate(starts):
            idx = perm[start:start + batch]
            mlp_loss_grad(params, X, Y, grad, ws, losses[k:k + 1], idx=idx, mean=mean, std=std)
            step += 1
            adam_step(params, grad, m, v, step, lr=lr)
        sizes = np.array([min(batch, N - s0) for s0 in starts], np.float64)
        history.append(float((losses.cpu().numpy().astype(np.float64) * sizes).sum() / N))
        if log:
            log("epoch %d loss %.6g" % (epoch, history[-1]))
    return Model(params, mean, std, label), history


def time_to_target(cuts, target, n_sweeps, seconds):
    """eq. (3)-(5) over one batch of R trials, with t_trial = batch time / R."""
    c = np.asarray(cuts)
    p_s = metrics.success_probability(c, target)
    r = metrics.repetitions(p_s)
    t_trial = seconds / len(c)
    return dict(P_s=p_s, r=r, STT=n_sweeps * r, TTT=t_trial * r, t_trial=t_trial, best=int(c.max()))


def median(xs):
    xs = sorted(xs)
    if not xs:
        return math.nan
    mid = len(xs) // 2
    return xs[mid] if len(xs) % 2 else 0.5 * (xs[mid - 1] + xs[mid])
