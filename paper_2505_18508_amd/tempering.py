"""Replica exchange (parallel tempering) as a trial: time to target.

Each of L ladders of K temperatures is one trial: after every checkpoint its
best cut so far is the largest end-of-round cut of its K replicas seen up to
then (a solver reports the best state it has met).  For each checkpoint, the
fraction of ladders at or above the target gives P_s, r (eq. (3)) and
TTT = (GPU time so far / L) x r (eq. (5)), as for annealing trials; the
target is 99.9 % of a reference best cut (Table I's rule).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import PT, create_graph, metrics


def tempering_run(dims, weight_seed, betas, n_ladders, sweeps_per_round, n_rounds, checkpoint_rounds, seed=401,
                  log=None):
    import torch

    g = create_graph(list(dims), weight_seed)
    K = len(betas)
    R = K * n_ladders
    pt = PT(g, betas, n_ladders, seed)
    spins = torch.zeros((R, g.n), dtype=torch.int8, device="cuda")
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    best = np.full(n_ladders, np.iinfo(np.int64).min, np.int64)
    checkpoints = []
    gpu_s = 0.0
    q = 0
    while q < n_rounds:
        m = min(checkpoint_rounds, n_rounds - q)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pt.run(spins, m, sweeps_per_round, round_begin=q, init_spins=(q == 0), cut=cut, stream=stream)
        b.record(stream)
        b.synchronize()
        gpu_s += a.elapsed_time(b) / 1e3
        q += m
        c = cut.cpu().numpy().reshape(n_ladders, K)
        best = np.maximum(best, c.max(axis=1))
        checkpoints.append({"rounds": q, "sweeps": q * sweeps_per_round, "gpu_seconds": gpu_s,
                            "ladder_best": best.copy()})
        if log:
            log("round %7d  sweeps %9d  best %d  mean ladder best %.2f  %.3f s" % (
                q, q * sweeps_per_round, best.max(), best.mean(), gpu_s))
    acc = pt.accepted()
    labels = pt.labels().cpu().numpy()
    pt.close()
    out = {"dims": list(dims), "weight_seed": weight_seed, "betas": [float(x) for x in betas],
           "ladders": n_ladders, "replicas": R, "n_sites": g.n, "sweeps_per_round": sweeps_per_round,
           "rounds": n_rounds, "accepted_per_pair": [int(x) for x in acc],
           "exchange_rate_per_pair": [float(x) / (n_ladders * ((n_rounds + (k % 2 == 0)) // 2)) for k, x in
                                      enumerate(acc)],
           "labels_are_permutations": bool(all(sorted(labels[l * K:(l + 1) * K]) == list(range(K))
                                                for l in range(n_ladders))),
           "checkpoints": checkpoints}
    g.close()
    return out


def summarise(run, reference_best, quality=0.999):
    best = max(int(reference_best), int(max(c["ladder_best"].max() for c in run["checkpoints"])))
    target = metrics.target_cut(best, quality)
    L = run["ladders"]
    rows = []
    for c in run["checkpoints"]:
        lb = c["ladder_best"]
        p_s = metrics.success_probability(lb, target)
        t_trial = c["gpu_seconds"] / L
        rows.append({"sweeps": c["sweeps"], "gpu_seconds": c["gpu_seconds"], "best": int(lb.max()),
                     "mean_ladder_best": float(lb.mean()), "P_s": p_s,
                     "r": metrics.repetitions(p_s) if p_s > 0 else None,
                     "TTT_s": t_trial * metrics.repetitions(p_s) if p_s > 0 else None})
    reached = [r for r in rows if r["TTT_s"] is not None]
    fastest = min(reached, key=lambda r: r["TTT_s"]) if reached else None
    return {"best_cut": best, "target": target, "checkpoints": rows, "fastest": fastest}


def main(argv=None):
    ap = argparse.ArgumentParser(description="replica exchange as a trial: best cut and time to target")
    ap.add_argument("--dims", default="100x200")
    ap.add_argument("--weight-seed", type=int, default=81)
    ap.add_argument("--temps", type=int, default=32)
    ap.add_argument("--ladders", type=int, default=32)
    ap.add_argument("--beta-min", type=float, default=0.2)
    ap.add_argument("--beta-max", type=float, default=3.0)
    ap.add_argument("--sweeps-per-round", type=int, default=10)
    ap.add_argument("--rounds", type=int, default=30000)
    ap.add_argument("--checkpoint", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=401)
    ap.add_argument("--reference-best", type=int, default=0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    dims = tuple(int(v) for v in args.dims.split("x"))
    betas = np.geomspace(args.beta_min, args.beta_max, args.temps)
    t0 = time.time()
    run = tempering_run(dims, args.weight_seed, betas, args.ladders, args.sweeps_per_round, args.rounds,
                        args.checkpoint, args.seed, log=lambda m: print(m, flush=True))
    s = summarise(run, args.reference_best)
    for c in run["checkpoints"]:
        c["ladder_best"] = [int(v) for v in c["ladder_best"]]
    out = {"run": run, "summary": s, "wall_seconds": time.time() - t0}
    text = json.dumps(out)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(json.dumps(s))


if __name__ == "__main__":
    sys.exit(main())
