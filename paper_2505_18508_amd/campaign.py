"""Trial-length campaign: highest and average end-of-trial cut as a function
of the number of sweeps per trial, and the trial length that minimises the
time to target.

The paper tunes exactly one parameter per instance, the trial length in
sweeps (Section III), and plots the highest and average cut of 100-trial
campaigns against it (Fig. 1: 1e3 ... 3e6 sweeps).  Here each campaign runs R
independent trials of one trial length on the GPU; the target is 99.9% of
the best cut found over all campaigns of the instance (Table I's rule), and
each campaign's success probability gives r (eq. (3)), STT (eq. (4)) and TTT
(eq. (5)) with t_trial = batch time / R.  Long trials run as consecutive
windows of one schedule, which equals one uninterrupted run bit for bit.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import create_graph, metrics, run_trials

DEFAULT_SWEEPS = (1000, 3000, 10000, 30000, 100000, 300000, 1000000)


def one_campaign(g, n_replicas, n_sweeps, seed, schedule="geometric", beta0=0.05, beta1=4.0, window=100000,
                 stream=None):
    """R trials of n_sweeps sweeps: end-of-trial cuts (host int64) and GPU seconds."""
    import torch

    stream = stream or torch.cuda.current_stream()
    spins = torch.zeros((n_replicas, g.n), dtype=torch.int8, device="cuda")
    cut = torch.zeros(n_replicas, dtype=torch.int64, device="cuda")
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    b = 0
    while b < n_sweeps:
        e = min(n_sweeps, b + window)
        run_trials(g, spins, seed, n_sweeps, b, e, schedule, beta0, beta1, None, b == 0, "auto",
                   cut if e == n_sweeps else None, stream=stream)
        b = e
    end.record(stream)
    end.synchronize()
    return cut.cpu().numpy(), start.elapsed_time(end) / 1e3


def campaign(dims=(100, 200), weight_seed=81, n_replicas=1024, sweeps=DEFAULT_SWEEPS, seed=301,
             schedule="geometric", beta0=0.05, beta1=4.0, quality=0.999, reference_best=None, log=None):
    g = create_graph(list(dims), weight_seed)
    rows = []
    for S in sweeps:
        cuts, secs = one_campaign(g, n_replicas, S, seed + len(rows), schedule, beta0, beta1)
        rows.append((S, cuts, secs))
        if log:
            log("S %8d: best %d  mean %.2f  %.3f s" % (S, cuts.max(), cuts.mean(), secs))
    # the best cut found for the instance: these campaigns', or a larger one
    # found earlier (reference_best)
    best = max([int(c.max()) for _, c, _ in rows] + ([int(reference_best)] if reference_best else []))
    target = metrics.target_cut(best, quality)
    out = {"dims": list(dims), "weight_seed": weight_seed, "n_edges": g.n_edges, "replicas": n_replicas,
           "schedule": [schedule, beta0, beta1], "best_cut": best, "quality": quality, "target": target,
           "campaigns": []}
    for S, cuts, secs in rows:
        p_s = metrics.success_probability(cuts, target)
        p_best = metrics.success_probability(cuts, best)
        t_trial = secs / n_replicas
        ok = p_s > 0
        r = metrics.repetitions(p_s) if ok else None
        vals, counts = np.unique(cuts, return_counts=True)
        out["campaigns"].append({
            "sweeps": S, "best": int(cuts.max()), "mean": float(cuts.mean()), "min": int(cuts.min()),
            "batch_seconds": secs, "t_trial_s": t_trial, "P_s": p_s, "P_best": p_best,
            "r": r, "STT_sweeps": S * r if ok else None, "TTT_s": t_trial * r if ok else None,
            "cut_values": [int(v) for v in vals], "cut_counts": [int(c) for c in counts]})
    reached = [c for c in out["campaigns"] if c["TTT_s"] is not None]
    if reached:
        fastest = min(reached, key=lambda c: c["TTT_s"])
        out["best_trial_length"] = {"sweeps": fastest["sweeps"], "TTT_s": fastest["TTT_s"],
                                    "STT_sweeps": fastest["STT_sweeps"]}
    g.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="trial-length campaign: highest and average cut vs sweeps per trial")
    ap.add_argument("--dims", default="100x200")
    ap.add_argument("--weight-seed", type=int, default=81)
    ap.add_argument("--replicas", type=int, default=1024)
    ap.add_argument("--sweeps", default=",".join(str(s) for s in DEFAULT_SWEEPS))
    ap.add_argument("--seed", type=int, default=301)
    ap.add_argument("--quality", type=float, default=0.999)
    ap.add_argument("--reference-best", type=int, default=0,
                    help="best cut found on the instance by earlier runs (joins the target's best)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    dims = tuple(int(v) for v in args.dims.split("x"))
    sweeps = tuple(int(v) for v in args.sweeps.split(","))
    t0 = time.time()
    out = campaign(dims, args.weight_seed, args.replicas, sweeps, args.seed, quality=args.quality,
                   reference_best=args.reference_best or None, log=lambda m: print(m, flush=True))
    out["wall_seconds"] = time.time() - t0
    text = json.dumps(out)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(text)


if __name__ == "__main__":
    sys.exit(main())
