"""Persistent batches of uneven instances: every replica bit-identical to a
single-instance run (itself pinned to the oracle), at small and full size,
eagerly and replayed from a captured HIP graph.  Instances take the
bit-sliced 4 x 4 routine (with a two-row last word line per plane where
Ly = 2 mod 4), forced ones the byte-per-replica routine, in the same launch."""
import numpy as np
import pytest

import oracle
from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ising():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as m

    m.lib()
    return m


def make_runs(ising, specs):
    import torch

    graphs, runs = [], []
    for dims, wseed, seed, R, S, b, e, sched, b0, b1 in specs:
        g = ising.create_graph(dims, wseed)
        graphs.append(g)
        runs.append(dict(seed=seed, n_sweeps=S, sweep_begin=b, sweep_end=e, schedule=sched, beta0=b0, beta1=b1,
                         spins=torch.zeros((R, g.n), dtype=torch.int8, device="cuda"),
                         cut=torch.zeros(R, dtype=torch.int64, device="cuda"),
                         energy=torch.zeros(R, dtype=torch.int64, device="cuda"),
                         flips=torch.zeros(R, dtype=torch.int32, device="cuda")))
    return graphs, runs


def single(ising, g, run):
    import torch

    R = run["spins"].shape[0]
    spins = torch.zeros_like(run["spins"])
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    fl = torch.zeros(R, dtype=torch.int32, device="cuda")
    ising.run_trials(g, spins, run["seed"], run["n_sweeps"], run["sweep_begin"], run["sweep_end"], run["schedule"],
                     run["beta0"], run["beta1"], None, True, "i8", cut, en, fl)
    return spins, cut, en, fl


def assert_run_equal(run, ref):
    for name, r in zip(("spins", "cut", "energy", "flips"), ref):
        assert bool((run[name] == r).all()), name


SMALL = [([6, 8], 1, 11, 13, 300, 0, 300, "geometric", 0.05, 4.0),
         ([10, 12], 2, 12, 5, 500, 0, 120, "linear", 0.1, 3.0),
         ([20, 30], 3, 13, 40, 200, 0, 200, "geometric", 0.05, 4.0),
         ([12, 16], 4, 14, 8, 800, 0, 800, "linear", 0.2, 2.5),
         ([2, 4], 5, 15, 3, 100, 0, 100, "geometric", 0.1, 2.0)]


def test_small_uneven_batch_matches_single_runs_and_oracle(ising):
    import torch

    graphs, runs = make_runs(ising, SMALL)
    b = ising.Batch(graphs, runs)
    assert b.n_items == sum((R + 3) // 4 for _, _, _, R, *_ in SMALL)
    b.run()
    torch.cuda.synchronize()
    for g, run in zip(graphs, runs):
        assert_run_equal(run, single(ising, g, run))
    # and the first instance against the oracle directly
    dims, wseed, seed, R, S = SMALL[0][:5]
    n = oracle.n_sites(dims)
    ref, fl = oracle.run(dims, oracle.random_weights(wseed, 2 * n), seed, R, S, schedule=oracle.SCHED_GEOMETRIC,
                         beta0=0.05, beta1=4.0)
    assert (runs[0]["spins"].cpu().numpy() == ref).all()
    assert (runs[0]["flips"].cpu().numpy().astype(np.uint32) == fl).all()
    b.close()


SMALL_3D = [([4, 6, 8], 21, 31, 9, 300, 0, 300, "geometric", 0.05, 4.0),   # Ly = 2 mod 4: short last word line
            ([6, 4, 6], 22, 32, 4, 200, 50, 200, "linear", 0.1, 3.0),
            ([8, 8, 8], 23, 33, 13, 150, 0, 150, "geometric", 0.05, 4.0)]


def test_3d_uneven_batch_matches_single_runs_and_oracle(ising):
    import torch

    graphs, runs = make_runs(ising, SMALL_3D)
    for run in runs[1:2]:  # a window that does not start at sweep 0 takes given spins
        run["spins"].copy_(torch.from_numpy(inputs.random_spins(8, run["spins"].shape[0], run["spins"].shape[1])))
        run["init_spins"] = False
    given = runs[1]["spins"].clone()
    b = ising.Batch(graphs, runs)
    b.run()
    torch.cuda.synchronize()
    for k, (g, run) in enumerate(zip(graphs, runs)):
        if k == 1:
            R = given.shape[0]
            spins = given.clone()
            cut = torch.zeros(R, dtype=torch.int64, device="cuda")
            en = torch.zeros(R, dtype=torch.int64, device="cuda")
            fl = torch.zeros(R, dtype=torch.int32, device="cuda")
            ising.run_trials(g, spins, run["seed"], run["n_sweeps"], run["sweep_begin"], run["sweep_end"],
                             run["schedule"], run["beta0"], run["beta1"], None, False, "i8", cut, en, fl)
            assert_run_equal(run, (spins, cut, en, fl))
        else:
            assert_run_equal(run, single(ising, g, run))
    dims, wseed, seed, R, S = SMALL_3D[0][:5]
    n = oracle.n_sites(dims)
    ref, fl = oracle.run(dims, oracle.random_weights(wseed, 3 * n), seed, R, S, schedule=oracle.SCHED_GEOMETRIC,
                         beta0=0.05, beta1=4.0)
    assert (runs[0]["spins"].cpu().numpy() == ref).all()
    assert (runs[0]["flips"].cpu().numpy().astype(np.uint32) == fl).all()
    b.close()


def test_full_size_uneven_batch_matches_single_runs(ising):
    """The four tori of 5,000-20,000 spins with 256-4,096 replicas and
    5,000-20,000 sweeps in one persistent launch: every replica equal to
    single-instance runs of another packing, and the first and last replica of
    each instance equal to the oracle over its whole schedule."""
    import torch

    specs = [([50, 100], 11, 111, 256, 5000, 0, 5000, "geometric", 0.05, 4.0),
             ([100, 100], 12, 112, 1024, 10000, 0, 10000, "geometric", 0.05, 4.0),
             ([100, 140], 13, 113, 2048, 15000, 0, 15000, "geometric", 0.05, 4.0),
             ([100, 200], 14, 114, 4096, 20000, 0, 20000, "geometric", 0.05, 4.0)]
    graphs, runs = make_runs(ising, specs)
    b = ising.Batch(graphs, runs)
    b.run()
    torch.cuda.synchronize()
    for g, run in zip(graphs, runs):
        assert_run_equal(run, single(ising, g, run))
    b.close()
    # the oracle recomputes the first and the last replica of every instance end to end,
    # one replica per host thread
    import concurrent.futures
    import os

    def orc(task):
        k, r = task
        dims, wseed, seed, R, S = specs[k][:5]
        w = oracle.random_weights(wseed, len(dims) * oracle.n_sites(dims))
        s, fl = oracle.run(dims, w, seed, 1, S, 0, S, oracle.SCHED_GEOMETRIC, 0.05, 4.0, replica_begin=r)
        cut, en = oracle.cut_energy(dims, w, s)
        return task, (s, cut, en, fl)

    tasks = [(k, r) for k, spec in enumerate(specs) for r in (0, spec[3] - 1)]
    print("oracle replicas (instance, replica):", tasks, flush=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        for (k, r), (s, cut, en, fl) in ex.map(orc, tasks):
            run = runs[k]
            assert (run["spins"][r:r + 1].cpu().numpy() == s).all(), (k, r)
            assert run["cut"][r].item() == cut[0] and run["energy"][r].item() == en[0], (k, r)
            assert (run["flips"][r:r + 1].cpu().numpy().astype(np.uint32) == fl).all(), (k, r)


def test_graph_replays_match_eager(ising):
    import torch

    graphs, runs = make_runs(ising, SMALL)
    b = ising.Batch(graphs, runs)
    b.run()
    torch.cuda.synchronize()
    eager = [{k: run[k].clone() for k in ("spins", "cut", "energy", "flips")} for run in runs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run()  # warm-up on the capture stream's side
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run()
    for replay in range(3):
        for run in runs:  # eager work between replays: scramble the outputs
            for k in ("spins", "cut", "energy", "flips"):
                run[k].fill_(replay + 1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for run, ref in zip(runs, eager):
            for k in ref:
                assert bool((run[k] == ref[k]).all()), (replay, k)
    b.close()


def test_batch_argument_errors(ising):
    import torch

    g2 = ising.create_graph([6, 8], 1)
    g3 = ising.create_graph([4, 4, 4], 1)
    s2 = torch.zeros((4, g2.n), dtype=torch.int8, device="cuda")
    s3 = torch.zeros((4, g3.n), dtype=torch.int8, device="cuda")
    run = dict(seed=1, n_sweeps=10)
    with pytest.raises(ising.IsingError) as e:
        ising.Batch([g2, g3], [dict(run, spins=s2), dict(run, spins=s3)])
    assert e.value.code == ising.E_ARG
    with pytest.raises(ising.IsingError) as e:
        ising.Batch([g2], [dict(run, spins=s2, layout="bp32")])
    assert e.value.code == ising.E_UNSUPPORTED
    with pytest.raises(ising.IsingError) as e:
        ising.Batch([g2], [dict(run, spins=s2, sweep_begin=3, sweep_end=2)])
    assert e.value.code == ising.E_ARG


def test_mixed_and_forced_layouts_in_one_batch(ising):
    """Forced i8 and bs4 instances next to AUTO ones (bs4, two-row last word
    lines at 6 and 10 rows): every replica equals its single-instance run."""
    graphs, runs = make_runs(ising, [([8, 6], 6, 21, 9, 300, 0, 300, "geometric", 0.05, 4.0),
                                     ([8, 6], 6, 21, 9, 300, 0, 300, "geometric", 0.05, 4.0),
                                     ([6, 8], 7, 22, 6, 250, 0, 250, "linear", 0.1, 3.0),
                                     ([10, 12], 8, 23, 7, 200, 0, 200, "geometric", 0.05, 4.0)])
    runs[0]["layout"] = "i8"
    runs[1]["layout"] = "bs4"
    b = ising.Batch(graphs, runs)
    b.run()
    import torch

    torch.cuda.synchronize()
    for g, run in zip(graphs, runs):
        assert_run_equal(run, single(ising, g, run))
    b.close()
    g = ising.create_graph([200, 204], 1)  # bit-sliced records beyond a block's LDS
    s = torch.zeros((4, g.n), dtype=torch.int8, device="cuda")
    with pytest.raises(ising.IsingError) as e:
        ising.Batch([g], [dict(seed=1, n_sweeps=10, spins=s, layout="bs4")])
    assert e.value.code == ising.E_UNSUPPORTED



def test_batch_with_replica_thresholds_matches_single_runs(ising):
    """Instances whose replicas run at their own fixed temperatures (the
    replica-exchange sweeps) in one persistent launch: every replica equals
    its single-instance run, and the first instance equals the oracle."""
    import torch

    from oracle import pt as opt

    rng = np.random.default_rng(5)
    specs = [([8, 12], 31, 7, 300), ([6, 10], 32, 6, 250), ([10, 12], 33, 9, 200), ([4, 4, 8], 34, 5, 150)]
    graphs, runs, refs, rep0 = [], [], [], None
    for dims, ws, R, S in specs:
        g = ising.create_graph(dims, ws)
        rep = opt.ladder_thresholds(rng.uniform(0.2, 2.0, R), len(dims))
        if rep0 is None:
            rep0 = rep
        thr = torch.from_numpy(rep.astype(np.int32)).cuda()
        run = dict(seed=40 + ws, n_sweeps=S, sweep_begin=0, sweep_end=S, schedule="linear", beta0=0.0, beta1=0.0,
                   spins=torch.zeros((R, g.n), dtype=torch.int8, device="cuda"),
                   cut=torch.zeros(R, dtype=torch.int64, device="cuda"),
                   energy=torch.zeros(R, dtype=torch.int64, device="cuda"),
                   flips=torch.zeros(R, dtype=torch.int32, device="cuda"), replica_thresholds=thr)
        s2 = torch.zeros_like(run["spins"])
        c2, e2 = torch.zeros_like(run["cut"]), torch.zeros_like(run["energy"])
        f2 = torch.zeros_like(run["flips"])
        ising.run_trials(g, s2, run["seed"], S, 0, S, "linear", 0.0, 0.0, None, True, "auto", c2, e2, f2,
                         replica_thresholds=thr)
        graphs.append(g)
        runs.append(run)
        refs.append((s2, c2, e2, f2))
    b = ising.Batch(graphs[:3], runs[:3])  # one ndim per batch
    b.run()
    b3 = ising.Batch(graphs[3:], runs[3:])
    b3.run()
    torch.cuda.synchronize()
    for run, ref in zip(runs, refs):
        assert_run_equal(run, ref)
    dims, ws, R, S = specs[0]
    w = oracle.random_weights(ws, len(dims) * oracle.n_sites(dims))
    ref, rfl = oracle.run_fixed(dims, w, runs[0]["seed"], rep0, 0, S)
    assert (runs[0]["spins"].cpu().numpy() == ref).all()
    assert (runs[0]["flips"].cpu().numpy().astype(np.uint32) == rfl).all()
    for x in (b, b3):
        x.close()
