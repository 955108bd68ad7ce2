"""Autotuner for the sweep kernels.

For a (torus, replica count) the tuner times every candidate launch shape on
a short window of the real schedule: the packing (4 replicas per block with
maintained fields, 4 replicas x 4 sites bit-sliced, or 32 replicas per block
bit-sliced) and the tile shape
(lines of the colour-split lattice per pass, hence threads per block).
Results never depend on the candidate -- the tuner checks that every
candidate returns bit-identical spins, cuts, energies and flip counts --
so only speed decides.  Choices are cached in a JSON file keyed by device,
torus and replica count (ISING_TUNE_CACHE, default
~/.cache/paper_2505_18508_amd/tune.json).
"""
import json
import os

from . import E_UNSUPPORTED, IsingError, run_trials

MAX_BLOCK = 1024


def _lattice(dims):
    if len(dims) == 2:
        return dict(Lz=1, Ly=dims[0], Lx=dims[1])
    return dict(Lz=dims[0], Ly=dims[1], Lx=dims[2])


def candidates(dims, n_replicas, cus=256):
    """(layout, block_threads) pairs worth timing for a torus and R."""
    L = _lattice(dims)
    hx, lines = L["Lx"] // 2, L["Ly"] * L["Lz"]
    out = []
    if hx > MAX_BLOCK:
        return out
    max_lp = min(MAX_BLOCK // hx, lines)
    lps = sorted({lp for lp in (max_lp, max_lp // 2, max_lp // 4, (max_lp // 2) * 2 if max_lp > 2 else max_lp)
                  if lp >= 1})
    for layout in ("i8", "bp32", "bs4"):
        if layout == "bp32" and (n_replicas + 31) // 32 < cus // 8:
            continue  # fewer than one group per eight CUs: never competitive
        word_lines = (L["Ly"] + 3) // 4 * L["Lz"]  # four rows per word line; Ly = 2 mod 4: a last one of two
        cand_lps = lps if layout != "bs4" else sorted({max(1, min(lp, word_lines)) for lp in lps})
        for lp in cand_lps:
            out.append((layout, lp * hx))
    return out


def cache_path():
    return os.environ.get("ISING_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2505_18508_amd", "tune.json"))


def _key(device_name, dims, n_replicas):
    return "%s|%s|%d" % (device_name, "x".join(str(d) for d in dims), n_replicas)


def load_cache(path=None):
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_cache(cache, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(graph, n_replicas, seed=1, n_sweeps=10000, window=100, schedule="geometric", beta0=0.05, beta1=4.0,
         repeats=3, use_cache=True, path=None, log=None):
    """Best (layout, block_threads) for this torus and R; times each candidate
    on sweeps [0, window) of the schedule and checks they agree bit for bit."""
    import torch

    dev_name = torch.cuda.get_device_name()
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    key = _key(dev_name, graph.dims, n_replicas)
    cache = load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        c = cache[key]
        return c["layout"], c["block_threads"]
    cands = candidates(graph.dims, n_replicas, cus)
    if not cands:
        raise ValueError("no on-chip kernel fits this torus")
    R = n_replicas
    ref = None
    results = []
    for layout, bt in cands:
        spins = torch.zeros((R, graph.n), dtype=torch.int8, device="cuda")
        cut = torch.zeros(R, dtype=torch.int64, device="cuda")
        en = torch.zeros(R, dtype=torch.int64, device="cuda")
        fl = torch.zeros(R, dtype=torch.int32, device="cuda")
        run = lambda: run_trials(graph, spins, seed, n_sweeps, 0, window, schedule, beta0, beta1, None, True,
                                 layout, cut, en, fl, bt)
        try:
            run()  # warm-up, and the candidate's result
        except IsingError as e:
            if e.code == E_UNSUPPORTED:  # does not fit on chip
                continue
            raise
        torch.cuda.synchronize()
        out = (spins.clone(), cut.clone(), en.clone(), fl.clone())
        if ref is None:
            ref = out
        elif not all(bool(torch.equal(a, b)) for a, b in zip(ref, out)):
            raise AssertionError("candidate %s/%d changed the results" % (layout, bt))
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(repeats):
            run()
        end.record()
        end.synchronize()
        ms = start.elapsed_time(end) / repeats
        rate = R * graph.n * window / (ms / 1e3)
        results.append((rate, layout, bt))
        if log:
            log("  %-4s block %4d: %.3f ms, %.3e attempts/s" % (layout, bt, ms, rate))
    if not results:
        raise ValueError("no on-chip kernel fits this torus")
    rate, layout, bt = max(results)
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"layout": layout, "block_threads": bt, "attempts_per_s": rate,
                      "candidates": [[l, b, r] for r, l, b in results]}
        save_cache(cache, path)
    return layout, bt


def tuned_run_trials(graph, spins, seed, n_sweeps, sweep_begin=0, sweep_end=None, schedule="linear", beta0=0.1,
                     beta1=3.0, beta_table=None, init_spins=True, cut=None, energy=None, flips=None, stream=None,
                     path=None):
    """run_trials with the launch shape from the tuning cache (tuned on first use)."""
    layout, bt = tune(graph, spins.shape[0], n_sweeps=n_sweeps, schedule=schedule if schedule != "table" else
                      "geometric", beta0=beta0 if schedule != "table" else 0.05, beta1=beta1 if schedule != "table"
                      else 4.0, path=path)
    run_trials(graph, spins, seed, n_sweeps, sweep_begin, sweep_end, schedule, beta0, beta1, beta_table, init_spins,
               layout, cut, energy, flips, bt, stream=stream)
    return layout, bt



def batch_candidates(dims):
    """(layout, block_threads) pairs for one instance of a persistent batch:
    the four-replica packings at the tile sizes candidates() gives."""
    return [(l, bt) for l, bt in candidates(dims, 4, cus=1 << 30) if l in ("bs4", "i8")]


def tune_batch(graphs, runs, fraction=0.02, repeats=3, log=None):
    """Per-instance (layout, block_threads) of a persistent batch.

    Coordinate descent over the instances, costliest first: each candidate
    for one instance, the others at their current picks, times the whole
    batch on a window of every run's schedule cut to `fraction` of its
    length (so the instances keep their relative costs); every candidate
    plan must return the same spins, cuts, energies and flip counts as the
    default plan (checked).  runs are Batch run dicts (their buffers are not
    touched).  Returns (picks, table): picks[k] = (layout, block_threads)
    with ("auto", 0) the library's default, table = timed plans."""
    import torch

    from . import Batch

    short = []
    for run in runs:
        b = run.get("sweep_begin", 0)
        e = run.get("sweep_end") or run["n_sweeps"]
        w = max(1, int(round((e - b) * fraction)))
        R = run["spins"].shape[0]
        dev = run["spins"].device
        short.append(dict(run, sweep_begin=b, sweep_end=b + w, spins0=run["spins"].clone(),
                          cut=torch.zeros(R, dtype=torch.int64, device=dev),
                          energy=torch.zeros(R, dtype=torch.int64, device=dev),
                          flips=torch.zeros(R, dtype=torch.int32, device=dev)))

    def timed(picks):
        rs = []
        for (layout, bt), s in zip(picks, short):
            r = {k: v for k, v in s.items() if k != "spins0"}
            r.update(layout=layout, block_threads=bt, spins=s["spins0"].clone())
            rs.append(r)
        try:
            batch = Batch(graphs, rs)
        except IsingError as e:
            if e.code == E_UNSUPPORTED:
                return None, None
            raise
        ms = []
        for rep in range(repeats + 1):
            for r, s in zip(rs, short):
                r["spins"].copy_(s["spins0"])
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            batch.run()
            end.record()
            end.synchronize()
            if rep > 0:  # the first run is the warm-up
                ms.append(start.elapsed_time(end))
        out = [t.clone() for r in rs for t in (r["spins"], r["cut"], r["energy"], r["flips"])]
        batch.close()
        return sorted(ms)[len(ms) // 2], out

    picks = [("auto", 0)] * len(graphs)
    best_ms, ref = timed(picks)
    table = [(list(picks), best_ms)]
    if log:
        log("default plan: %.3f ms" % best_ms)
    order = sorted(range(len(graphs)), key=lambda k: -graphs[k].n * runs[k]["spins"].shape[0] * (
        (runs[k].get("sweep_end") or runs[k]["n_sweeps"]) - runs[k].get("sweep_begin", 0)))
    for k in order:
        for cand in batch_candidates(graphs[k].dims):
            trial = list(picks)
            trial[k] = cand
            ms, out = timed(trial)
            if ms is None:
                continue
            if not all(bool(torch.equal(a, b)) for a, b in zip(ref, out)):
                raise AssertionError("batch plan %s changed the results" % (trial,))
            table.append((trial, ms))
            if log:
                log("instance %d %-4s block %4d: %.3f ms" % (k, cand[0], cand[1], ms))
            if ms < best_ms:
                best_ms, picks = ms, trial
    return picks, table


def main(argv=None):
    """Time every candidate launch shape of one torus and replica count and
    print them with the pick and the library's default (AUTO) choice."""
    import argparse

    import torch

    from . import create_graph, select_layout

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--dims", required=True, help="torus, e.g. 100x100 or 16x16x16")
    ap.add_argument("--weight-seed", type=int, default=1)
    ap.add_argument("--replicas", type=int, required=True)
    ap.add_argument("--sweeps", type=int, default=10000, help="schedule length (geometric 0.05 -> 4.0)")
    ap.add_argument("--window", type=int, default=200, help="sweeps [0, window) timed per candidate")
    ap.add_argument("--out", default=None, help="also write the table as JSON")
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the tuner times kernels on a GPU"
    dims = [int(x) for x in args.dims.split("x")]
    g = create_graph(dims, args.weight_seed)
    rows = []
    layout, bt = tune(g, args.replicas, n_sweeps=args.sweeps, window=args.window, use_cache=False,
                      log=lambda s: (print(s, flush=True), rows.append(s.split())))
    auto = select_layout(g, args.replicas, args.sweeps)
    print("pick: %s block %d; default (AUTO): %s" % (layout, bt, auto))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"dims": dims, "replicas": args.replicas, "sweeps": args.sweeps, "window": args.window,
                       "pick": [layout, bt], "auto": auto,
                       "candidates": [[r[0], int(r[2].rstrip(":")), float(r[3]), float(r[5])] for r in rows]},
                      fh, indent=1)
    g.close()


if __name__ == "__main__":
    main()
