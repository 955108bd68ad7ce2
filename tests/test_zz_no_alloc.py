"""GPU tests of ising_run_trials_noalloc (the entry point that allocates
nothing): called through the C ABI, its results equal ising_run_trials' bit
for bit on every layout, on consecutive calls of shrinking size that share
the library's fixed scratch, and runs needing more than that scratch are
refused before anything is enqueued."""
import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ising():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as m

    m.lib()
    return m


def both(ising, dims, R, S, begin=0, end=None, init=True, layout="auto", seed=5, wseed=3, schedule="geometric",
         b0=0.05, b1=4.0, stats=False, rep_thr=None):
    """Outputs of run_trials and of run_trials_noalloc on the same inputs."""
    import torch

    g = ising.create_graph(dims, wseed)
    start = torch.from_numpy(inputs.random_spins(seed + 1, R, g.n)).cuda()
    outs = []
    for fn in (ising.run_trials, ising.run_trials_noalloc):
        spins = start.clone()
        cut = torch.zeros(R, dtype=torch.int64, device="cuda")
        en = torch.zeros(R, dtype=torch.int64, device="cuda")
        fl = torch.zeros(R, dtype=torch.int32, device="cuda")
        st = torch.zeros(2, dtype=torch.int64, device="cuda") if stats else None
        fn(g, spins, seed, S, begin, end, schedule, b0, b1, None, init, layout, cut, energy=en, flips=fl, stats=st,
           replica_thresholds=rep_thr)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (spins, cut, en, fl) + ((st,) if stats else ())])
    g.close()
    return outs


def assert_same(outs):
    (a, b) = outs
    for x, y in zip(a, b):
        assert x.shape == y.shape and (x == y).all()


def test_two_calls_in_a_row_second_smaller(ising):
    print("noalloc: bs4 20x24 R64 S300, then i8 12x16 R16 window [100, 260)", flush=True)
    assert_same(both(ising, [20, 24], 64, 300, layout="bs4"))
    assert_same(both(ising, [12, 16], 16, 500, 100, 260, init=False, layout="i8", seed=9, wseed=4))


@pytest.mark.parametrize("dims,R,S,layout", [([16, 20], 96, 200, "bp32"), ([4, 8, 6], 32, 150, "bs4"),
                                             ([6, 4, 6], 8, 120, "i8"), ([8, 12, 10], 64, 90, "bp32"),
                                             ([100, 200], 8192, 3, "auto")])
def test_layouts_match_run_trials(ising, dims, R, S, layout):
    print("noalloc:", dims, R, S, layout, flush=True)
    assert_same(both(ising, dims, R, S, layout=layout, stats=layout == "bp32"))


def test_streamed_layout_uses_scratch_for_state_and_cut(ising):
    """Streamed 264x264 (69,696 sites: the cut's partial sums go through the
    scratch too), 32 replicas, from given spins over a window."""
    print("noalloc: stream 264x264 R32 window [3, 9)", flush=True)
    assert_same(both(ising, [264, 264], 32, 12, 3, 9, init=False, layout="stream", stats=True))
    print("noalloc: stream 264x264 R32 init", flush=True)
    assert_same(both(ising, [264, 264], 32, 6, layout="stream"))


def test_per_replica_thresholds(ising):
    import torch

    R, K = 16, 2
    thr = ising.thresholds(R, "linear", 0.2, 2.5, degree=4)  # one temperature per replica
    rep = torch.from_numpy(thr.view(np.int32).reshape(R, K).copy()).cuda()
    print("noalloc: bs4 per-replica thresholds 12x16 R16", flush=True)
    assert_same(both(ising, [12, 16], R, 40, layout="bs4", rep_thr=rep))


def test_runs_beyond_the_scratch_are_refused_untouched(ising):
    import torch

    g = ising.create_graph([12, 16], 1)
    spins = torch.ones((4, g.n), dtype=torch.int8, device="cuda")
    # 3,000,000 sweeps x 2 thresholds x 4 B = 24 MB of thresholds
    with pytest.raises(ising.IsingError) as e:
        ising.run_trials_noalloc(g, spins, 1, 3_000_000, 0, None, "geometric", 0.05, 4.0, None, False)
    assert e.value.code == ising.E_UNSUPPORTED and "scratch" in str(e.value)
    # a window inside the same schedule fits
    ising.run_trials_noalloc(g, spins, 1, 3_000_000, 0, 50, "geometric", 0.05, 4.0, None, False)
    g.close()
    big = ising.create_graph([1000, 1000], 1)
    s2 = torch.ones((256, big.n), dtype=torch.int8, device="cuda")
    with pytest.raises(ising.IsingError) as e:  # 32 MB of streamed state
        ising.run_trials_noalloc(big, s2, 1, 10, 0, None, "geometric", 0.05, 4.0, None, False, "stream")
    assert e.value.code == ising.E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((s2 == 1).all())
    big.close()
