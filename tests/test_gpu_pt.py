"""GPU parity of replica exchange against the oracle: per-replica fixed
temperatures in both four-replica layouts, and whole tempering runs (sweeps,
exchange decisions, temperature labels, energies, accepted counts) bit for
bit."""
import numpy as np
import pytest

import oracle
from oracle import pt as opt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ising():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as m

    m.lib()
    return m


@pytest.mark.parametrize("dims,layout", [([8, 12], "bs4"), ([8, 12], "i8"), ([6, 8], "i8"), ([6, 8], "bs4"),
                                         ([2, 10], "bs4"), ([4, 4, 6], "bs4"), ([4, 6, 6], "i8"),
                                         ([4, 6, 6], "bs4")])
def test_replica_thresholds_match_oracle(ising, dims, layout):
    import torch

    n = oracle.n_sites(dims)
    deg = 2 * len(dims)
    rng = np.random.default_rng(len(dims) * 100 + n)
    R = 13
    betas = rng.uniform(0.1, 2.5, R)
    rep = opt.ladder_thresholds(betas, len(dims))
    w = oracle.random_weights(3, len(dims) * n)
    g = ising.create_graph(dims, 3)
    spins = torch.zeros((R, n), dtype=torch.int8, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    fl = torch.zeros(R, dtype=torch.int32, device="cuda")
    thr = torch.from_numpy(rep.astype(np.int32)).cuda()
    ising.run_trials(g, spins, 21, 40, 0, 40, "linear", 0.0, 0.0, None, True, layout, None, en, fl,
                     replica_thresholds=thr)
    ref, rfl = oracle.run_fixed(dims, w, 21, rep, 0, 40)
    _, ren = oracle.cut_energy(dims, w, ref)
    torch.cuda.synchronize()
    assert (spins.cpu().numpy() == ref).all()
    assert (en.cpu().numpy() == ren).all() and (fl.cpu().numpy().astype(np.uint32) == rfl).all()
    assert thr.shape == (R, deg // 2)
    g.close()


def test_replica_thresholds_need_a_four_replica_layout(ising):
    import torch

    g = ising.create_graph([8, 12], 3)
    spins = torch.zeros((8, g.n), dtype=torch.int8, device="cuda")
    thr = torch.zeros((8, 2), dtype=torch.int32, device="cuda")
    for layout in ("bp32", "stream"):
        with pytest.raises(ising.IsingError) as e:
            ising.run_trials(g, spins, 1, 10, layout=layout, replica_thresholds=thr)
        assert e.value.code == ising.E_UNSUPPORTED
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(ising.IsingError) as e:
        ising.run_trials(g, spins, 1, 10, replica_thresholds=thr, stats=st)
    assert e.value.code == ising.E_UNSUPPORTED
    assert ising.select_layout(g, 8) == "bs4"
    g.close()


@pytest.mark.parametrize("dims", [[8, 12], [6, 8], [4, 4, 6]])
def test_tempering_run_matches_oracle(ising, dims):
    import torch

    n = oracle.n_sites(dims)
    betas = list(np.geomspace(0.2, 2.0, 6))
    L, Q, E, seed = 3, 20, 5, 97
    w = oracle.random_weights(5, len(dims) * n)
    g = ising.create_graph(dims, 5)
    p = ising.PT(g, betas, L, seed)
    spins = torch.zeros((L * 6, n), dtype=torch.int8, device="cuda")
    cut = torch.zeros(L * 6, dtype=torch.int64, device="cuda")
    en = torch.zeros(L * 6, dtype=torch.int64, device="cuda")
    p.run(spins, Q, E, init_spins=True, cut=cut, energy=en)
    labels = p.labels().cpu().numpy()
    acc = p.accepted()
    rs, ren, rk, rpos, log = opt.run_pt(dims, w, seed, betas, L, Q, E)
    rcut, _ = oracle.cut_energy(dims, w, rs)
    torch.cuda.synchronize()
    assert (spins.cpu().numpy() == rs).all()
    assert (en.cpu().numpy() == ren).all() and (cut.cpu().numpy() == rcut).all()
    assert (labels == rk).all()
    counts = np.zeros(len(betas) - 1, np.int64)
    for a in log:
        for _, k in a:
            counts[k] += 1
    assert (acc.astype(np.int64) == counts).all() and counts.sum() > 0
    p.close()
    g.close()


def test_tempering_full_shape_matches_oracle(ising):
    """The shape the tempering experiment runs: 100x200 torus, 32 ladders of
    32 temperatures (1,024 replicas, 256 quads), three rounds of 10 sweeps;
    every spin, energy, label and accepted count against the oracle."""
    import torch

    dims = [100, 200]
    n = oracle.n_sites(dims)
    betas = list(np.geomspace(0.5, 3.0, 32))
    L, Q, E, seed = 32, 3, 10, 401
    w = oracle.random_weights(81, 2 * n)
    g = ising.create_graph(dims, 81)
    p = ising.PT(g, betas, L, seed)
    spins = torch.zeros((L * 32, n), dtype=torch.int8, device="cuda")
    en = torch.zeros(L * 32, dtype=torch.int64, device="cuda")
    p.run(spins, Q, E, init_spins=True, energy=en)
    labels = p.labels().cpu().numpy()
    acc = p.accepted()
    rs, ren, rk, rpos, log = opt.run_pt(dims, w, seed, betas, L, Q, E)
    torch.cuda.synchronize()
    assert (spins.cpu().numpy() == rs).all()
    assert (en.cpu().numpy() == ren).all() and (labels == rk).all()
    counts = np.zeros(31, np.int64)
    for a in log:
        for _, k in a:
            counts[k] += 1
    assert (acc.astype(np.int64) == counts).all()
    p.close()
    g.close()


def test_tempering_resumes_and_equal_temperatures_swap(ising):
    import torch

    dims = [8, 12]
    g = ising.create_graph(dims, 6)
    betas = [0.3, 0.5, 0.9, 1.5]
    a = ising.PT(g, betas, 2, 5)
    b = ising.PT(g, betas, 2, 5)
    sa = torch.zeros((8, g.n), dtype=torch.int8, device="cuda")
    sb = torch.zeros_like(sa)
    a.run(sa, 12, 4, init_spins=True)
    b.run(sb, 5, 4, init_spins=True)
    b.run(sb, 7, 4, round_begin=5)
    torch.cuda.synchronize()
    assert torch.equal(sa, sb) and torch.equal(a.labels(), b.labels())
    same = ising.PT(g, [0.8] * 4, 2, 5)
    s = torch.zeros_like(sa)
    same.run(s, 4, 2, init_spins=True)
    acc = same.accepted()
    assert list(acc) == [4, 4, 4]  # pairs (0,1), (2,3) on even rounds, (1,2) on odd, two ladders each
    for h in (a, b, same):
        h.close()
    g.close()


def test_tempering_argument_errors(ising):
    g = ising.create_graph([8, 12], 6)
    for betas, L in (([0.5], 1), ([0.5, 0.4], 1), ([0.5, float("nan")], 1), ([0.5, 0.6], 0),
                     ([0.5, 0.5 + 1e-7], 1)):
        with pytest.raises(ising.IsingError) as e:
            ising.PT(g, betas, L, 1)
        assert e.value.code == ising.E_ARG
    g.close()
