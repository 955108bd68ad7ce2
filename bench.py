"""Benchmark: spin-update attempts per second of replica-parallel checkerboard
Metropolis annealing on one MI355X.

Workload (default): 2-D toroidal grid 100 x 200 (20,000 spins, 40,000 +/-1
edges from weight seed 81: the size of the paper's largest instance, G81),
8,192 replicas, 40,000 sweeps, geometric beta 0.05 -> 4.0, run seed 201.
One step = one whole pass of the hot path over that batch: Philox initial
state, the full sweep schedule with flip counters, exact cut/energy, and the
host readout (best cut, success probability, repetitions r of eq. (3),
sweeps-to-target of eq. (4)).  The library picks the packing (for this
replica count: 32 replicas per LDS word, one block per 32 replicas);
--layout forces another.

Prints one JSON line.  Inputs are synthetic (the paper's Gset instances are
not available); the instance is generated from its seed on the host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    "torus100x100": dict(dims=[100, 100], weight_seed=2, seed=102, R=1024, S=10000, schedule="geometric", beta0=0.05, beta1=4.0,
               name="2-D torus 100x100 (10,000 spins, weight seed 2), 1,024 replicas, 10,000 sweeps, "
                    "geometric beta 0.05->4.0, run seed 102"),
    "torus100x200": dict(dims=[100, 200], weight_seed=81, seed=201, R=8192, S=40000, schedule="geometric", beta0=0.05, beta1=4.0,
               name="2-D torus 100x200 (20,000 spins, weight seed 81), 8,192 replicas, 40,000 sweeps, "
                    "geometric beta 0.05->4.0, run seed 201"),
}
WORKLOADS["batch4tori"] = dict(
    instances=[([50, 100], 11, 111, 256, 5000), ([100, 100], 12, 112, 1024, 10000), ([100, 140], 13, 113, 2048, 15000),
               ([100, 200], 14, 114, 4096, 20000)],
    schedule="geometric", beta0=0.05, beta1=4.0,
    name="batch of 2-D tori 50x100 / 100x100 / 100x140 / 100x200 (weight seeds 11-14) with 256 / 1,024 / 2,048 / "
         "4,096 replicas and 5,000 / 10,000 / 15,000 / 20,000 sweeps in one persistent launch, geometric beta "
         "0.05->4.0, run seeds 111-114")
WORKLOADS["torus1000x1000"] = dict(dims=[1000, 1000], weight_seed=1000, seed=7, R=256, S=2000, schedule="geometric", beta0=0.05,
                       beta1=4.0, name="2-D torus 1000x1000 (1,000,000 spins, weight seed 1000), 256 replicas, 2,000 "
                                        "sweeps streamed from HBM, geometric beta 0.05->4.0, run seed 7")
WORKLOADS["torus64x64x64"] = dict(dims=[64, 64, 64], weight_seed=643, seed=7, R=256, S=2000, schedule="geometric", beta0=0.05,
                          beta1=4.0, name="3-D torus 64^3 (262,144 spins, degree 6, weight seed 643), 256 replicas, "
                                          "2,000 sweeps streamed from HBM, geometric beta 0.05->4.0, run seed 7")
# Time-to-target leg (eq. (3)-(5)): the 20,000-spin instance above, trials long
# enough (10^6 sweeps) for plain annealing to reach 99.9 % of the instance's
# best cut, a ranking every 50,000 sweeps (19 culls), the network trained on
# plain runs of 13 other instances of the same shape (weight seeds 1001-1013)
# by `python -m paper_2505_18508_amd.experiments --replicas 1024 --sweeps 1000000
# --window 50000 --train-replicas 1024 --n-traj 13312 --seeds 5 --long-sweeps
# 3000000 --known-best 13896 --label relative --save-model ...`; best cut known
# for the instance: 13,898 (found by that experiment's learned runs), the
# target 99.9 % of the larger of it and every cut this leg finds.
TTT = dict(dims=[100, 200], weight_seed=81, R=1024, S=1_000_000, window=50_000, seeds=(201, 202, 203),
           beta0=0.05, beta1=4.0, known_best=13898,
           model=os.path.join("paper_2505_18508_amd", "models", "torus100x200_S1e6_relative.npz"),
           name="2-D torus 100x200 (weight seed 81), 1,024 replicas, 10^6 sweeps per trial, geometric beta "
                "0.05->4.0, a ranking every 50,000 sweeps, run seeds 201-203")
HBM_PEAK = 8e12
# streamed layout: per sweep each 32-replica word is read and written once and
# its neighbours' words read once: 12 bytes per word per sweep
STREAM_BYTES_PER_WORD_SWEEP = 12
DEFAULT_WORKLOAD = "torus100x200"
WORKLOAD = WORKLOADS[DEFAULT_WORKLOAD]
# LDS: 256 CUs x 128 bytes per cycle x 2.4 GHz
LDS_PEAK = 256 * 128 * 2.4e9


def lds_bytes_per_attempt(layout, ndim):
    """Algorithmic LDS bytes per attempt of the on-chip packings: bp32 reads
    a site's word and its 2 ndim neighbours' words and writes it back (4 B
    each) per 32 attempts; bs4 (2-D) reads ten 4-byte record entries per
    16-attempt word.  None where no such figure is derived."""
    if layout == "bp32":
        return (2 * ndim + 2) * 4 / 32
    if layout == "bs4" and ndim == 2:
        return 10 * 4 / 16
    return None


# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz of 32-bit integer VALU issue
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# algorithmic VALU lane-ops: one Philox4x32-10 word per attempt that needs a
# uniform (a block = 20 32x32->64 products + 20 three-input xors, 4 words),
# plus the Metropolis decision of every attempt (field lookup, threshold
# compare, conditional flip)
OPS_PER_DRAW = 40 / 4
OPS_PER_ATTEMPT = 3


# the reference copy of --calibrate-copy: a kernel of known HBM traffic
# (this many bytes read and written) that scales the counters of the same run
CALIBRATION_COPY_BYTES = 256 << 20


def traffic_path():
    return os.path.join(ROOT, "profiles", "traffic.json")


def source_closure(src):
    """A kernel source file (repository-relative) and, transitively, every
    header it includes with #include "..." (beside the including file, else
    under include/), in discovery order."""
    import re

    order, seen, todo = [], set(), [src]
    while todo:
        f = todo.pop(0)
        if f in seen:
            continue
        seen.add(f)
        order.append(f)
        for inc in re.findall(r'^#include "([^"]+)"', open(os.path.join(ROOT, f)).read(), re.M):
            path = os.path.normpath(os.path.join(os.path.dirname(f), inc))
            if not os.path.exists(os.path.join(ROOT, path)):
                path = os.path.normpath(os.path.join("include", inc))
            if os.path.exists(os.path.join(ROOT, path)):
                todo.append(path)
    return order


def sources_digest(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter profile, or None when
    there is none or the kernel source changed since it was taken."""
    path = traffic_path()
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("%s/%s" % (kernel, workload))
    if rec is None:
        return None
    # the kernel's source file and every header it includes
    if sources_digest(rec["sources"]) != rec["sources_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def counter_per_dispatch(run_dir, counter, kernel):
    """Per-dispatch values (summed over the device's instances) of one counter
    for the dispatches whose kernel name contains `kernel`, in dispatch order,
    from a rocprofv3 --pmc run written with -o run --output-format csv."""
    import csv

    per, names = {}, {}
    for r in csv.DictReader(open(os.path.join(run_dir, "run_counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            d = int(r["Dispatch_Id"])
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    return [per[d] for d in sorted(per) if kernel in names[d]]


def record_traffic(key, source, kernel, fetch_run, write_run, profile, per_sequence=None):
    """Store a kernel's HBM bytes per launch in profiles/traffic.json from a
    FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled by what
    the counter reads for the run's calibration copy (its largest copy
    dispatch), with the digest of the kernel's source closure.  One launch is
    the last matching dispatch, or with per_sequence = N the mean dispatch
    times N (a launch sequence of N half-sweeps)."""
    kib = CALIBRATION_COPY_BYTES / 1024.0
    sides = {}
    for side, run, counter in (("fetch", fetch_run, "FETCH_SIZE"), ("write", write_run, "WRITE_SIZE")):
        vals = counter_per_dispatch(run, counter, kernel)
        copy = max(counter_per_dispatch(run, counter, "copyBuffer"))
        raw = sum(vals) / len(vals) * per_sequence if per_sequence else vals[-1]
        sides[side] = raw * 1024 * (kib / copy)
    path = traffic_path()
    recs = json.load(open(path)) if os.path.exists(path) else {}
    files = source_closure(source)
    recs[key] = dict(fetch_bytes=sides["fetch"], write_bytes=sides["write"], sources=files,
                     sources_sha256=sources_digest(files), profile=profile)
    json.dump(recs, open(path, "w"), indent=1)
    return recs[key]


def batch_layout(ising, g, run):
    """The packing a batch instance runs in: the requested one, else (AUTO)
    bs4 where it fits, else i8."""
    if run.get("layout", "auto") != "auto":
        return run["layout"]
    try:
        return ising.select_layout(g, run["spins"].shape[0], run["n_sweeps"], "bs4")
    except ising.IsingError:
        return "i8"


def cpu_baseline(budget_s, wl, task_s=None):
    """The oracle on the host's cores: the first replicas of workload wl, one
    replica per task, until the time budget is spent -- each over the whole
    schedule, or over its first sweeps where one replica's whole schedule
    would take longer than task_s (default the budget; about 1e8 attempts
    per core and second).  Runs before the GPU is touched; worker
    processes are spawned fresh."""
    import concurrent.futures
    import multiprocessing

    import oracle

    n = math.prod(wl["dims"])
    w = oracle.random_weights(wl["weight_seed"], len(wl["dims"]) * n)
    cores = min(os.cpu_count() or 1, 16)
    S = wl["S"]
    end = min(S, max(1, int((budget_s if task_s is None else task_s) * 1e8 / n)))

    t0 = time.perf_counter()
    done = []
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        futs = []
        r = 0
        while r < min(cores, wl["R"]):
            futs.append(ex.submit(_oracle_one, r, w, wl, end))
            r += 1
        while futs:
            f = futs.pop(0)
            rr, spins = f.result()
            done.append((rr, spins))
            if time.perf_counter() - t0 < budget_s and r < wl["R"]:
                futs.append(ex.submit(_oracle_one, r, w, wl, end))
                r += 1
    elapsed = time.perf_counter() - t0
    attempts = len(done) * n * end
    what = "full %d-sweep schedule" % S if end == S else "sweeps [0, %d) of the %d-sweep schedule" % (end, S)
    return {"value": attempts / elapsed, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": "%d replicas x %s of %s (%.1f s)" % (len(done), what, wl.get("sample_of", "the same workload"),
                                                          elapsed)}, (done if end == S else None)


def _oracle_one(r, w, wl, end):
    import oracle

    s, _ = oracle.run(wl["dims"], w, wl["seed"], 1, wl["S"], 0, end, schedule=oracle.SCHED_GEOMETRIC,
                      beta0=wl["beta0"], beta1=wl["beta1"], replica_begin=r)
    return r, s[0]


def cpu_workload(name):
    """The single-instance workload the oracle baseline samples: the workload
    itself, or for the batch its largest instance (whose final spins the
    batch returns)."""
    W = WORKLOADS[name]
    if name != "batch4tori":
        return W
    dims, wseed, seed, R, S = W["instances"][-1]
    return dict(dims=dims, weight_seed=wseed, seed=seed, R=R, S=S, schedule=W["schedule"], beta0=W["beta0"],
                beta1=W["beta1"], sample_of="the batch's %dx%d instance" % tuple(dims))


def with_parity(cpu, cpu_spins, final):
    """The baseline record, with whether the oracle's full-schedule replicas
    equal the GPU's final spins (None when it ran a window only)."""
    cpu = dict(cpu)
    cpu["parity_with_gpu"] = None if cpu_spins is None else all(bool((final[rr] == s).all()) for rr, s in cpu_spins)
    return cpu


def ttt_workload(seeds=None):
    """The time-to-target workload, with other run seeds if given."""
    if seeds is None:
        return TTT
    seeds = tuple(int(x) for x in seeds)
    if not seeds:
        raise ValueError("the time-to-target leg needs at least one run seed")
    return dict(TTT, seeds=seeds,
                name=TTT["name"].rsplit(", run seeds", 1)[0] + ", run seeds " + ", ".join(str(x) for x in seeds))


def ttt_leg(log=None, seeds=None):
    """Median time to 99.9 % of the instance's best cut for the plain,
    learned-cull and energy-cull forms (eq. (3)-(5), t_trial = batch time / R)
    on the TTT workload (run seeds: the workload's, or `seeds`); every step
    runs in the library's kernels."""
    from paper_2505_18508_amd import create_graph, learn, metrics

    W = ttt_workload(seeds)
    g = create_graph(W["dims"], W["weight_seed"])
    model = learn.Model.load(os.path.join(ROOT, W["model"]))
    runs = {m: [] for m in learn.METHODS}
    for seed in W["seeds"]:
        for m in learn.METHODS:
            out = learn.anneal(g, W["R"], W["S"], seed, "geometric", W["beta0"], W["beta1"], W["window"], m,
                               model if m == "learned" else None)
            cuts = out["cut"].cpu().numpy()
            runs[m].append((cuts, out["seconds"]))
            if log:
                log("ttt %s seed %d: %.2f s, best %d" % (m, seed, out["seconds"], cuts.max()))
    best = max([W["known_best"]] + [int(c.max()) for m in runs for c, _ in runs[m]])
    target = metrics.target_cut(best)
    per = {m: [learn.time_to_target(c, target, W["S"], t) for c, t in runs[m]] for m in runs}
    med = {m: learn.median([p["TTT"] for p in per[m]]) for m in per}
    g.close()
    ratio = med["learned"] / med["plain"] if math.isfinite(med["plain"]) and med["plain"] > 0 else None
    return {"workload": W["name"], "best_cut": best, "target": target, "median_TTT_s": med,
            "learned_over_plain": ratio,
            "learned_over_energy": med["learned"] / med["energy"] if med["energy"] > 0 else None,
            "median_P_s": {m: learn.median([p["P_s"] for p in per[m]]) for m in per},
            "mean_final_cut": {m: float(sum(c.mean() for c, _ in runs[m]) / len(runs[m])) for m in runs},
            "batch_s": {m: [round(t, 4) for _, t in runs[m]] for m in runs}, "seeds": list(W["seeds"]),
            "model": W["model"],
            "note": "clones are correlated, so eq. (3) flatters the culled forms' P_s; mean_final_cut is not inflated"}


def bench_batch(args, ising, metrics, torch, dev):
    """The uneven-instance batch: one step = one persistent launch over all
    instances, plus the readout of every instance's cuts."""
    W = WORKLOAD
    graphs, runs = [], []
    for dims, wseed, seed, R, S in W["instances"]:
        g = ising.create_graph(dims, wseed)
        graphs.append(g)
        runs.append(dict(seed=seed, n_sweeps=S, schedule=W["schedule"], beta0=W["beta0"], beta1=W["beta1"],
                         spins=torch.zeros((R, g.n), dtype=torch.int8, device=dev),
                         cut=torch.zeros(R, dtype=torch.int64, device=dev)))
    # autotune each instance's packing and tile on short windows (untimed,
    # results checked identical), then time the tuned plan; the default plan's
    # full launch is timed once beside it
    from paper_2505_18508_amd import tune

    picks, table = tune.tune_batch(graphs, runs, log=lambda m: print("tune " + m, file=sys.stderr, flush=True))
    default = ising.Batch(graphs, runs)
    default.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    default.run()
    e1.record()
    e1.synchronize()
    default_ms = e0.elapsed_time(e1)
    default.close()
    runs = [dict(r, layout=l, block_threads=bt) for r, (l, bt) in zip(runs, picks)]
    batch = ising.Batch(graphs, runs)
    stream = torch.cuda.current_stream()
    # algorithmic work: RNG draws of the same trajectories, from instrumented single runs (untimed)
    draws = 0
    for g, run in zip(graphs, runs):
        st = torch.zeros(2, dtype=torch.int64, device=dev)
        tmp = torch.zeros_like(run["spins"])
        ising.run_trials(g, tmp, run["seed"], run["n_sweeps"], schedule=run["schedule"], beta0=run["beta0"],
                         beta1=run["beta1"], layout="i8", stats=st)
        torch.cuda.synchronize()
        draws += int(st[1].item())
        del tmp

    def step(ev):
        ev[0].record(stream)
        batch.run(stream)
        ev[1].record(stream)
        return [int(r["cut"].max().item()) for r in runs]

    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)])
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    bests = [step(ev) for ev in events][-1]
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    kernel_s = sum(e[0].elapsed_time(e[1]) for e in events) / len(events) / 1e3
    attempts = batch.attempts
    ops = OPS_PER_DRAW * draws + OPS_PER_ATTEMPT * attempts
    out = {
        "metric": "spin-update attempts/s on 1 MI355X", "value": attempts * args.steps / total_s,
        "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        # a batch instance takes bs4 wherever that packing fits, else i8
        "config": {"workload": W["name"], "layout": [batch_layout(ising, g, run) for g, run in zip(graphs, runs)],
                   "work_items": batch.n_items, "grid": batch.grid, "block": batch.block,
                   "tuned": [[l, bt] for l, bt in picks], "default_plan_kernel_ms": default_ms,
                   "tuning_window_ms": {"default": table[0][1], "tuned": min(ms for _, ms in table)}},
        "kernel_attempts_per_s": attempts / kernel_s, "kernel_ms": kernel_s * 1e3,
        "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": ops / kernel_s / VALU_PEAK_LANE_OPS,
                     "traffic": measured_traffic("k_sweep_batch", "batch4tori"), "kernel": "k_sweep_batch",
                     "draws": draws, "draw_fraction": draws / attempts},
        "readout": {"best_cut_per_instance": bests},
    }
    final = runs[-1]["spins"].cpu().numpy()  # the largest instance, which the oracle baseline samples
    batch.close()
    return out, final


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--layout", default="auto")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-target leg")
    ap.add_argument("--ttt-only", action="store_true",
                    help="run only the time-to-target leg and print its JSON object")
    ap.add_argument("--ttt-seeds", default=None, help="run seeds of the time-to-target leg, comma-separated")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default=DEFAULT_WORKLOAD)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device-to-device (a reference kernel of known traffic for counters)")
    ap.add_argument("--record-traffic", metavar="KERNEL/WORKLOAD", default=None,
                    help="no GPU: store profiles/traffic.json's record from the rocprofv3 runs named below")
    ap.add_argument("--source", help="with --record-traffic: the kernel's source file")
    ap.add_argument("--kernel", help="with --record-traffic: a substring of the dispatches' kernel name")
    ap.add_argument("--fetch-run", help="with --record-traffic: the FETCH_SIZE run's output folder")
    ap.add_argument("--write-run", help="with --record-traffic: the WRITE_SIZE run's output folder")
    ap.add_argument("--profile", help="with --record-traffic: the summary the record belongs to")
    ap.add_argument("--per-sequence", type=int, default=None,
                    help="with --record-traffic: launches per sequence (mean dispatch x N); else the last dispatch")
    args = ap.parse_args()
    if args.record_traffic:
        missing = [o for o in ("source", "kernel", "fetch_run", "write_run", "profile") if not getattr(args, o)]
        if missing:
            ap.error("--record-traffic needs " + ", ".join("--" + o.replace("_", "-") for o in missing))
        rec = record_traffic(args.record_traffic, args.source, args.kernel, args.fetch_run, args.write_run,
                             args.profile, args.per_sequence)
        print(json.dumps({args.record_traffic: rec}))
        return
    global WORKLOAD
    WORKLOAD = WORKLOADS[args.workload]
    if args.gpus != 1:
        print("bench.py measures one GPU only: the replica-parallel path has no cross-GPU step to time "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    ttt_seeds = [int(x) for x in args.ttt_seeds.split(",")] if args.ttt_seeds else None
    if args.ttt_only:
        print(json.dumps(ttt_leg(log=lambda m: print(m, file=sys.stderr, flush=True), seeds=ttt_seeds)))
        return

    cpu = cpu_spins = None
    if not args.no_cpu:
        cpu, cpu_spins = cpu_baseline(args.cpu_seconds, cpu_workload(args.workload))

    import torch

    import paper_2505_18508_amd as ising
    from paper_2505_18508_amd import metrics

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(CALIBRATION_COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    W = WORKLOAD
    if args.workload == "batch4tori":
        out, final = bench_batch(args, ising, metrics, torch, dev)
        if cpu is not None:
            out["cpu_baseline"] = with_parity(cpu, cpu_spins, final)
        print(json.dumps(out))
        return
    g = ising.create_graph(W["dims"], W["weight_seed"])
    R, S, n = W["R"], W["S"], g.n
    spins = torch.zeros((R, n), dtype=torch.int8, device=dev)
    cut = torch.zeros(R, dtype=torch.int64, device=dev)
    energy = torch.zeros(R, dtype=torch.int64, device=dev)
    flips = torch.zeros(R, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    groups = (R + 31) // 32
    layout = ising.select_layout(g, R, S, args.layout, args.block_threads)  # the packing the library runs
    streamed = layout == "stream"
    kernel_name = {"bp32": "k_sweep_bp32", "i8": "k_sweep_i8", "stream": "k_halfsweep_stream",
                   "bs4": "k_sweep_bs4"}[layout]

    def launch(stats=None):
        ising.run_trials(g, spins, W["seed"], S, 0, S, W["schedule"], W["beta0"], W["beta1"], None, True,
                         args.layout, cut, energy, flips, args.block_threads, 0, stats, stream)

    # RNG consumption of the trajectory (deterministic; an untimed instrumented run)
    stats = torch.zeros(2, dtype=torch.int64, device=dev)
    launch(stats)
    torch.cuda.synchronize()
    blocks, draws = (int(x) for x in stats.cpu().tolist())
    best = int(cut.max().item())
    target = metrics.target_cut(best)

    def step(ev):
        ev[0].record(stream)
        launch()
        ev[1].record(stream)
        c = cut.cpu()  # readout: device -> host, then eq. (3)-(4)
        b = int(c.max())
        return b, metrics.success_probability(c.numpy(), target)

    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)])
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    results = [step(ev) for ev in events]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = [e[0].elapsed_time(e[1]) for e in events]
    total_s = t1 - t0
    attempts = R * n * S
    value = attempts * args.steps / total_s
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    ops = OPS_PER_DRAW * draws + OPS_PER_ATTEMPT * attempts
    achieved = ops / avg_kernel_s
    p_s = results[-1][1]
    r = metrics.repetitions(p_s)

    out = {
        "metric": "spin-update attempts/s on 1 MI355X",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": W["name"], "layout": layout, "replicas": R, "sweeps": S, "spins": n},
        "kernel_attempts_per_s": attempts / avg_kernel_s,
        "kernel_ms": avg_kernel_s * 1e3,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_LANE_OPS,
                     "traffic": measured_traffic(kernel_name, args.workload),
                     "kernel": kernel_name, "philox_blocks": blocks, "draws": draws,
                     "draw_fraction": draws / attempts},
        "readout": {"best_cut": results[-1][0], "target": target, "P_s": p_s, "r": r, "STT_sweeps": S * r},
    }
    lds_b = lds_bytes_per_attempt(layout, len(W["dims"]))
    if lds_b is not None:
        out["lds"] = {"algorithmic_bytes_per_attempt": lds_b, "achieved_TBps": lds_b * attempts / avg_kernel_s / 1e12,
                      "peak_TBps": LDS_PEAK / 1e12, "frac": lds_b * attempts / avg_kernel_s / LDS_PEAK}
    if streamed:
        # kernel_ms covers the whole launch sequence (pack, 2 S half-sweeps, unpack, cut)
        hbm = STREAM_BYTES_PER_WORD_SWEEP * n * groups * S
        out["hbm"] = {"algorithmic_bytes": hbm, "achieved_GBps": hbm / avg_kernel_s / 1e9,
                      "peak_GBps": HBM_PEAK / 1e9, "frac": hbm / avg_kernel_s / HBM_PEAK}
    if cpu is not None:
        out["cpu_baseline"] = with_parity(cpu, cpu_spins, spins.cpu().numpy())
    g.close()
    if not args.no_ttt and args.workload == DEFAULT_WORKLOAD:
        del spins, cut, energy, flips
        out["ttt"] = ttt_leg(log=lambda m: print(m, file=sys.stderr, flush=True), seeds=ttt_seeds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
