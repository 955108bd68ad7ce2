"""Autotuner: candidate launch shapes (CPU) and tuning on the GPU, where every
candidate must give bit-identical results."""
import os

import pytest

from paper_2505_18508_amd import tune


def test_candidates_cover_packings_and_tiles():
    c = tune.candidates([100, 100], 1024)
    layouts = {l for l, _ in c}
    assert layouts == {"i8", "bp32", "bs4"}
    assert all(bt % 50 == 0 and 0 < bt <= 1024 for _, bt in c)  # multiples of Lx/2 = 50
    # bs4 word lines hold 4 rows: at most 100 / 4 = 25 of them per pass
    assert all(bt <= 25 * 50 for l, bt in c if l == "bs4")
    # too few 32-replica groups: the bit-packed layout is not a candidate; 50 rows: 13 word
    # lines, the last of two rows
    c50 = tune.candidates([50, 100], 16)
    assert {l for l, _ in c50} == {"i8", "bs4"}
    assert all(bt <= 13 * 50 for l, bt in c50 if l == "bs4")
    assert {l for l, _ in tune.candidates([48, 100], 16)} == {"i8", "bs4"}
    # 3-D with Ly = 6: two word lines per plane, the second of two rows
    c3 = tune.candidates([4, 6, 8], 16)
    assert {l for l, _ in c3} == {"i8", "bs4"}
    assert all(bt <= 2 * 4 * 4 for l, bt in c3 if l == "bs4")
    assert tune.candidates([2, 4096], 64) == []  # a line wider than a block


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    tune.save_cache({"a|1x2|3": {"layout": "i8", "block_threads": 50}}, path)
    assert tune.load_cache(path)["a|1x2|3"]["block_threads"] == 50
    assert tune.load_cache(str(tmp_path / "missing.json")) == {}


@pytest.mark.gpu
def test_tuning_picks_identical_fastest_shape(tmp_path):
    import torch

    import paper_2505_18508_amd as ising

    path = str(tmp_path / "tune.json")
    g = ising.create_graph([100, 100], 2)
    layout, bt = tune.tune(g, 1024, seed=102, n_sweeps=10000, window=50, path=path, log=print)
    assert layout in ("i8", "bp32", "bs4") and bt > 0
    cache = tune.load_cache(path)
    (entry,) = cache.values()
    assert entry["layout"] == layout and len(entry["candidates"]) >= 2
    # the cache answers the second call; the tuned launch equals the default one
    assert tune.tune(g, 1024, path=path) == (layout, bt)
    R = 64
    a = torch.zeros((R, g.n), dtype=torch.int8, device="cuda")
    b = torch.zeros((R, g.n), dtype=torch.int8, device="cuda")
    ising.run_trials(g, a, 5, 500, schedule="geometric", beta0=0.05, beta1=4.0)
    tune.tuned_run_trials(g, b, 5, 500, schedule="geometric", beta0=0.05, beta1=4.0, path=path)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_batch_candidates_are_four_replica_tiles():
    c = tune.batch_candidates([100, 140])
    assert {l for l, _ in c} == {"i8", "bs4"}
    assert all(bt % 70 == 0 and 0 < bt <= 1024 for _, bt in c)  # multiples of Lx/2 = 70
    assert tune.batch_candidates([2, 4096]) == []


@pytest.mark.gpu
def test_batch_tuning_keeps_results_and_is_used_by_the_plan():
    """The tuner's per-instance picks give the default plan's results bit for
    bit, and a batch built with them equals single runs."""
    import torch

    import paper_2505_18508_amd as ising

    specs = [([20, 30], 3, 11, 16, 400), ([24, 40], 4, 12, 32, 600), ([18, 26], 5, 13, 8, 300)]
    graphs, runs = [], []
    for dims, ws, seed, R, S in specs:
        g = ising.create_graph(dims, ws)
        graphs.append(g)
        runs.append(dict(seed=seed, n_sweeps=S, schedule="geometric", beta0=0.05, beta1=4.0,
                         spins=torch.zeros((R, g.n), dtype=torch.int8, device="cuda"),
                         cut=torch.zeros(R, dtype=torch.int64, device="cuda")))
    picks, table = tune.tune_batch(graphs, runs, fraction=0.5, repeats=1, log=print)
    assert len(picks) == 3 and len(table) > 3
    tuned = [dict(r, layout=l, block_threads=bt) for r, (l, bt) in zip(runs, picks)]
    b = ising.Batch(graphs, tuned)
    b.run()
    torch.cuda.synchronize()
    for g, run in zip(graphs, tuned):
        s = torch.zeros_like(run["spins"])
        c = torch.zeros_like(run["cut"])
        ising.run_trials(g, s, run["seed"], run["n_sweeps"], schedule="geometric", beta0=0.05, beta1=4.0, cut=c)
        torch.cuda.synchronize()
        assert torch.equal(s, run["spins"]) and torch.equal(c, run["cut"])
    b.close()
