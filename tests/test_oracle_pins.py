"""Pins of the CPU oracle against facts that do not come from the oracle itself:
an outside Philox implementation, the paper's printed cut/energy pairs,
closed forms of the objective, brute force over all states of tiny tori, the
Boltzmann distribution that Metropolis sweeps preserve, and exact invariants
(gauge symmetry, window resume, maintained-field consistency)."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox4x32-10 against PyTorch's engine (independent implementation)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def torch_philox():
    import torch.utils.cpp_extension as ce

    tmp = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(tmp, "philox_ref")
    cmd = ["g++", "-O1", "-std=c++17"] + ["-I" + p for p in ce.include_paths()]
    cmd += [os.path.join(HERE, "philox_torch_ref.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)

    def run(queries):
        text = "".join("%d %d %d %d %d\n" % (k, *c) for k, c in queries)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [tuple(int(x) for x in line.split()) for line in out.strip().splitlines()]

    return run


def test_philox_matches_torch_engine(torch_philox):
    rng = np.random.default_rng(12345)
    queries = [(0, (0, 0, 0, 0)), (2**64 - 1, (2**32 - 1,) * 4), (0xDEADBEEF_00C0FFEE, (1, 2, 3, 4))]
    for _ in range(300):
        key = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        ctr = tuple(int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64))
        queries.append((key, ctr))
    # counters shaped like the method's: (site, sweep, replica quad, tag)
    for site in (0, 1, 4999, 19999):
        for t in (0, 1, 39999):
            for q in (0, 7, 2047):
                for tag in range(4):
                    queries.append((101, (site, t, q, tag)))
    ref = torch_philox(queries)
    for (key, ctr), want in zip(queries, ref):
        got = tuple(int(x) for x in oracle.philox(key, ctr))
        assert got == want, (key, ctr)


@pytest.fixture(scope="module")
def metropolis_words():
    """2^20 Metropolis words: Philox blocks of (site, sweep, quad, tag 0) for
    4,096 sites x 16 sweeps x 4 quads; column r = the word of replica 4q + r."""
    out = np.zeros((4096 * 16 * 4, 4), np.uint32)
    i = 0
    for q in range(4):
        for t in range(16):
            for site in range(4096):
                out[i] = oracle.philox(2024, (site, t, q, oracle.TAG_METROPOLIS))
                i += 1
    return out


def test_philox_words_uniform(metropolis_words):
    # 2^18 words per output position: chi^2 of the top and the bottom byte
    # against uniform (256 bins, 1,024 expected per bin)
    for j in range(4):
        col = metropolis_words[:, j]
        for byte in (col >> 24, col & 0xFF):
            assert stats.chisquare(np.bincount(byte.astype(np.int64), minlength=256)).pvalue > 1e-4


@pytest.mark.parametrize("beta", [0.05, 0.2, 0.5])
def test_metropolis_acceptance_frequency(metropolis_words, beta):
    """The fraction of Metropolis words below T_k(beta) is exp(-4 k beta), the
    Metropolis acceptance of dE = 4k (binomial z-test over 2^20 words)."""
    u = metropolis_words.reshape(-1).astype(np.uint64)
    N = u.size
    for k in (1, 2, 3):
        p = math.exp(-4 * k * beta)
        hits = int(np.count_nonzero(u < oracle.threshold(beta, k)))
        z = (hits - N * p) / math.sqrt(N * p * (1 - p))
        assert abs(z) < 5, (beta, k, hits, N * p)


# --------------------------------------------------------------------------
# Torus structure (Section I, Appendix A: toroidal grid, 4 neighbours, periodic)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [[2, 2], [2, 4], [4, 6], [6, 4], [50, 100], [2, 2, 2], [4, 2, 6], [6, 6, 6]])
def test_torus_edges_follow_coordinates(dims):
    a, b = oracle.torus_edges(dims)
    nd = len(dims)
    n = int(np.prod(dims))
    assert len(a) == nd * n
    # expected endpoints from coordinate arithmetic: edge nd*i + d steps the
    # d-th fastest axis forward by one, periodically
    strides = [int(np.prod(dims[k + 1:])) for k in range(nd)]
    for i in range(n):
        coords = [(i // strides[k]) % dims[k] for k in range(nd)]
        for d in range(nd):
            axis = nd - 1 - d
            nb = list(coords)
            nb[axis] = (nb[axis] + 1) % dims[axis]
            j = sum(nb[k] * strides[k] for k in range(nd))
            assert a[nd * i + d] == i and b[nd * i + d] == j
    deg = np.bincount(np.concatenate([a, b]), minlength=n)
    assert (deg == 2 * nd).all()


@pytest.mark.parametrize("dims", [[2, 2], [4, 6], [50, 100], [2, 2, 2], [4, 6, 2]])
def test_checkerboard_colouring_is_proper(dims):
    a, b = oracle.torus_edges(dims)
    col = oracle.colours(dims)
    assert (col[a] != col[b]).all()
    assert col.sum() * 2 == len(col)


def test_random_weights_balanced_and_seeded():
    w = oracle.random_weights(81, 40000)
    assert set(np.unique(w)) == {-1, 1}
    assert abs(int(w.sum())) < 5 * math.sqrt(40000)
    assert (w == oracle.random_weights(81, 40000)).all()
    assert (w != oracle.random_weights(82, 40000)).any()


def test_init_spins_balanced_and_seeded():
    s = oracle.init_spins(101, 16, 5000)
    assert set(np.unique(s)) == {-1, 1}
    assert abs(int(s.sum())) < 5 * math.sqrt(s.size)
    # replica offset selects the same streams
    assert (oracle.init_spins(101, 4, 5000, replica_begin=12) == s[12:]).all()


# --------------------------------------------------------------------------
# Objective: eq. (1) and eq. (2) with J = -w, h = 0
# --------------------------------------------------------------------------
def _dense_weights(dims, w):
    """Symmetric coupling matrix with parallel edges summed."""
    a, b = oracle.torus_edges(dims)
    n = oracle.n_sites(dims)
    W = np.zeros((n, n), np.int64)
    for e in range(len(a)):
        W[a[e], b[e]] += int(w[e])
        W[b[e], a[e]] += int(w[e])
    return W


@pytest.mark.parametrize("dims", [[2, 2], [4, 6], [8, 10], [2, 2, 2], [4, 2, 4]])
def test_cut_matches_eq1_and_energy_identity(dims):
    rng = np.random.default_rng(len(dims) * 100 + dims[0])
    n = oracle.n_sites(dims)
    w = oracle.random_weights(int(rng.integers(1, 1000)), len(dims) * n)
    W = _dense_weights(dims, w)
    iu = np.triu_indices(n, 1)
    spins = (2 * rng.integers(0, 2, size=(20, n)) - 1).astype(np.int8)
    cut, en = oracle.cut_energy(dims, w, spins)
    for r in range(20):
        x = spins[r].astype(np.int64)
        outer = np.outer(x, x)
        eq1 = 0.5 * np.sum(W[iu] * (1 - outer[iu]))
        ising = np.sum(W[iu] * outer[iu])  # -sum J s s with J = -w
        assert cut[r] == eq1
        assert en[r] == ising
        assert en[r] == int(w.sum()) - 2 * cut[r]


@pytest.mark.parametrize("dims", [[2, 2], [6, 4], [50, 100], [2, 4, 2]])
def test_cut_closed_forms(dims):
    n = oracle.n_sites(dims)
    ne = len(dims) * n
    ones = np.ones(ne, np.int8)
    board = np.where(oracle.colours(dims) == 0, 1, -1).astype(np.int8)
    cut, en = oracle.cut_energy(dims, ones, board)
    assert cut[0] == ne and en[0] == -ne
    cut, en = oracle.cut_energy(dims, ones, np.ones(n, np.int8))
    assert cut[0] == 0 and en[0] == ne
    w = oracle.random_weights(5, ne)
    cut, en = oracle.cut_energy(dims, w, -np.ones(n, np.int8))
    assert cut[0] == 0 and en[0] == int(w.sum())


def test_paper_pairs_fix_single_count_energy():
    """The paper's printed (cut, energy) pairs are consistent with H = W - 2 cut
    for an integer edge-weight sum W of the right parity and size, and not with
    an energy that counts each edge twice."""
    rows = []
    with open(os.path.join(HERE, "golden", "paper_cut_energy_pairs.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, ne, cut, en = line.split()
                rows.append((name, int(ne), int(cut), int(en)))
    double_count_ok = 0
    for name, ne, cut, en in rows:
        w_total = en + 2 * cut
        assert abs(w_total) <= 5 * math.sqrt(ne), name  # sum of ne random +/-1
        assert (w_total - ne) % 2 == 0, name
        if en % 2 == 0:
            w_double = en // 2 + 2 * cut
            double_count_ok += (w_double - ne) % 2 == 0 and abs(w_double) <= 5 * math.sqrt(ne)
    assert double_count_ok == 0
    # and the oracle's energy/cut satisfy that same relation
    dims = [10, 20]
    w = oracle.random_weights(9, 400)
    s = oracle.init_spins(3, 8, 200)
    cut, en = oracle.cut_energy(dims, w, s)
    assert (en == int(w.sum()) - 2 * cut).all()


# --------------------------------------------------------------------------
# Brute force and its closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [[2, 2], [2, 4], [4, 4], [2, 8], [2, 2, 2], [2, 2, 4]])
def test_bruteforce_closed_forms(dims):
    ne = len(dims) * oracle.n_sites(dims)
    best, state = oracle.maxcut_bruteforce(dims, np.ones(ne, np.int8))
    assert best == ne  # bipartite: every edge can be cut
    best, _ = oracle.maxcut_bruteforce(dims, -np.ones(ne, np.int8))
    assert best == 0


def test_bruteforce_2x2_is_doubled_four_cycle():
    """The 2x2 torus is the 4-cycle 0-1-3-2-0 with every edge doubled; the cut
    edges of a cycle form an even subset, so the max cut is the best even
    subset of the four summed weights."""
    import itertools

    for seed in range(1, 21):
        w = oracle.random_weights(seed, 8).astype(int)
        # edges: 2i + 0 -> right neighbour, 2i + 1 -> down neighbour
        a, b = oracle.torus_edges([2, 2])
        pair_w = {}
        for e in range(8):
            key = tuple(sorted((int(a[e]), int(b[e]))))
            pair_w[key] = pair_w.get(key, 0) + w[e]
        cycle = [pair_w[(0, 1)], pair_w[(1, 3)], pair_w[(2, 3)], pair_w[(0, 2)]]
        want = max(sum(c for c, m in zip(cycle, mask) if m)
                   for mask in itertools.product([0, 1], repeat=4) if sum(mask) % 2 == 0)
        best, state = oracle.maxcut_bruteforce([2, 2], w.astype(np.int8))
        assert best == want
        assert oracle.cut_energy([2, 2], w.astype(np.int8), state)[0][0] == best


@pytest.mark.parametrize("dims", [[2, 2], [2, 4], [4, 2], [4, 4], [2, 6], [2, 8], [2, 2, 2], [2, 2, 4]])
def test_annealer_reaches_bruteforce_max(dims):
    ne = len(dims) * oracle.n_sites(dims)
    for seed in range(1, 21):
        w = oracle.random_weights(seed, ne)
        best, _ = oracle.maxcut_bruteforce(dims, w)
        s, _ = oracle.run(dims, w, 1000 + seed, 16, 1000, schedule=oracle.SCHED_LINEAR, beta0=0.1, beta1=3.0)
        cut, _ = oracle.cut_energy(dims, w, s)
        assert cut.max() == best, (dims, seed)
        assert cut.max() <= best


def test_bipartite_all_positive_reaches_all_edges():
    dims = [50, 100]
    ne = 10000
    s, _ = oracle.run(dims, np.ones(ne, np.int8), 7, 16, 1000, schedule=oracle.SCHED_LINEAR, beta0=0.1, beta1=3.0)
    cut, _ = oracle.cut_energy(dims, np.ones(ne, np.int8), s)
    assert cut.max() == ne
    s, _ = oracle.run(dims, -np.ones(ne, np.int8), 7, 4, 200, schedule=oracle.SCHED_LINEAR, beta0=0.1, beta1=3.0)
    cut, _ = oracle.cut_energy(dims, -np.ones(ne, np.int8), s)
    assert cut.max() == 0


# --------------------------------------------------------------------------
# Metropolis at fixed beta samples exp(-beta H) / Z
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims,beta,wseed", [([2, 4], 0.35, 4), ([2, 2, 2], 0.25, 6), ([4, 2], 0.6, 8)])
def test_fixed_beta_samples_boltzmann(dims, beta, wseed):
    n = oracle.n_sites(dims)
    w = oracle.random_weights(wseed, len(dims) * n)
    S = 40
    R = 24000
    s, _ = oracle.run(dims, w, 4242, R, S, schedule=oracle.SCHED_TABLE, table=np.full(S, beta))
    idx = ((s > 0).astype(np.int64) << np.arange(n)).sum(axis=1)
    observed = np.bincount(idx, minlength=2**n)
    states = np.array([[1 if (k >> i) & 1 else -1 for i in range(n)] for k in range(2**n)], np.int8)
    _, en = oracle.cut_energy(dims, w, states)
    p = np.exp(-beta * (en - en.min()))
    p /= p.sum()
    expected = p * R
    # pool states with small expectation so the chi^2 approximation holds
    order = np.argsort(expected)
    obs_b, exp_b, acc_o, acc_e = [], [], 0, 0.0
    for k in order:
        acc_o += observed[k]
        acc_e += expected[k]
        if acc_e >= 20:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o, acc_e = 0, 0.0
    obs_b[-1] += acc_o
    exp_b[-1] += acc_e
    assert stats.chisquare(obs_b, exp_b).pvalue > 1e-3


def test_thresholds_closed_form():
    assert oracle.threshold(0.0, 1) == 0xFFFFFFFF
    for beta in (0.01, 0.05, 0.1, 0.5, 1.0, 2.0, 3.0, 4.0):
        prev = None
        for k in (1, 2, 3):
            t = oracle.threshold(beta, k)
            exact = 2.0**32 * math.exp(-4 * k * beta)
            assert abs(t - exact) <= 1.0
            if prev is not None:
                assert t <= prev
            prev = t
    # exp(-4 ln2 / 4) = 1/2 -> threshold at 2^31 up to rounding of ln 2
    assert abs(oracle.threshold(math.log(2) / 4, 1) - 2**31) <= 2
    # large beta: acceptance underflows to zero
    assert oracle.threshold(6.0, 1) == 0


def test_schedules():
    S = 1000
    lin = [oracle.beta(oracle.SCHED_LINEAR, 0.1, 3.0, S, t) for t in range(S)]
    assert lin[0] == 0.1 and abs(lin[-1] - 3.0) < 1e-15
    assert np.allclose(np.diff(lin), 2.9 / (S - 1), rtol=1e-9)
    geo = [oracle.beta(oracle.SCHED_GEOMETRIC, 0.05, 4.0, S, t) for t in range(S)]
    assert geo[0] == 0.05 and abs(geo[-1] - 4.0) < 1e-14
    ratios = np.array(geo[1:]) / np.array(geo[:-1])
    assert np.allclose(ratios, (4.0 / 0.05) ** (1.0 / (S - 1)), rtol=1e-12)
    assert oracle.beta(oracle.SCHED_GEOMETRIC, 0.05, 4.0, 1, 0) == 0.05


# --------------------------------------------------------------------------
# Exact invariants of the trajectory
# --------------------------------------------------------------------------
def test_gauge_transformation_commutes_with_sweeps():
    """w'_ab = g_a g_b w_ab and s' = g * s leave every energy change, hence
    every decision and draw, unchanged: trajectory(w', g*s0) = g * trajectory(w, s0)."""
    dims = [10, 12]
    n = 120
    rng = np.random.default_rng(77)
    w = oracle.random_weights(31, 2 * n)
    g = (2 * rng.integers(0, 2, size=n) - 1).astype(np.int8)
    a, b = oracle.torus_edges(dims)
    wg = (g[a] * g[b] * w).astype(np.int8)
    s0 = oracle.init_spins(5, 8, n)
    s1, f1 = oracle.run(dims, w, 99, 8, 300, spins=s0, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    s2, f2 = oracle.run(dims, wg, 99, 8, 300, spins=s0 * g, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    assert (s2 == s1 * g).all()
    assert (f1 == f2).all()
    assert (s1 != s0).any()


def test_planted_gauge_instance_reaches_its_bound():
    """w_ab = g_a g_b (a gauge of the all-positive torus): the state
    x = g * checkerboard satisfies every bond, so H(x) = -|E| is the minimum
    and cut(x) = number of +1 edges, the upper bound of any cut."""
    dims = [20, 30]
    n = 600
    rng = np.random.default_rng(5)
    g = (2 * rng.integers(0, 2, size=n) - 1).astype(np.int8)
    a, b = oracle.torus_edges(dims)
    board = np.where(oracle.colours(dims) == 0, 1, -1).astype(np.int8)
    w = (g[a].astype(np.int16) * g[b]).astype(np.int8)
    x = g * board
    positive = int((w > 0).sum())
    cut, en = oracle.cut_energy(dims, w, x)
    assert cut[0] == positive and en[0] == -2 * n
    s, _ = oracle.run(dims, w, 3, 8, 1000, schedule=oracle.SCHED_LINEAR, beta0=0.1, beta1=3.0)
    cut, en = oracle.cut_energy(dims, w, s)
    assert cut.max() == positive and en.min() == -2 * n


def test_window_resume_equals_one_run():
    dims = [20, 10]
    w = oracle.random_weights(2, 400)
    full, ff = oracle.run(dims, w, 17, 8, 500, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    a, fa = oracle.run(dims, w, 17, 8, 500, 0, 123, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    b, fb = oracle.run(dims, w, 17, 8, 500, 123, 500, spins=a, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    assert (b == full).all()
    assert (fa + fb == ff).all()


def test_replica_subsets_are_independent_streams():
    dims = [6, 8]
    w = oracle.random_weights(2, 96)
    full, _ = oracle.run(dims, w, 17, 12, 50)
    part, _ = oracle.run(dims, w, 17, 5, 50, replica_begin=6)
    assert (part == full[6:11]).all()


@pytest.mark.parametrize("dims", [[8, 6], [2, 4], [4, 4, 2]])
def test_maintained_fields_equal_recomputed(dims):
    n = oracle.n_sites(dims)
    w = oracle.random_weights(13, len(dims) * n)
    s, _, fo = oracle.run(dims, w, 21, 6, 77, schedule=oracle.SCHED_LINEAR, beta0=0.2, beta1=1.5, return_fields=True)
    a, b = oracle.torus_edges(dims)
    for r in range(6):
        f = np.zeros(n, np.int64)
        np.add.at(f, a, w.astype(np.int64) * s[r][b])
        np.add.at(f, b, w.astype(np.int64) * s[r][a])
        assert (fo[r] == f).all()


def test_flip_count_matches_changed_spins_at_infinite_temperature():
    # beta = 0: every proposal accepted (thresholds 2^32 - 1 reject with p 2^-32),
    # so each sweep flips every spin once: n flips per sweep and, over an even
    # number of sweeps, the initial state again.
    dims = [4, 6]
    w = oracle.random_weights(1, 48)
    s0 = oracle.init_spins(9, 4, 24)
    s, fl = oracle.run(dims, w, 3, 4, 10, spins=s0, schedule=oracle.SCHED_TABLE, table=np.zeros(10))
    assert (fl == 240).all()
    assert (s == s0).all()


def test_run_rejects_bad_arguments():
    w = oracle.random_weights(1, 30)
    with pytest.raises(ValueError):
        oracle.run([3, 5], w, 1, 2, 10)
    with pytest.raises(ValueError):
        oracle.run([4, 4], oracle.random_weights(1, 32), 1, 2, 10, begin=2, end=5)
