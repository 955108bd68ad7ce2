"""Pins of the replica-exchange oracle against what the method fixes: the
exchange acceptance frequency equals exp((beta_k - beta_{k+1})(H_a - H_b)),
the K-temperature chain samples the product of the Boltzmann distributions
(brute force over all states of a tiny torus), equal temperatures always
swap, every decision follows the energies, labels stay permutations, and
rounds resume exactly."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import pt


def test_exchange_acceptance_frequency_is_boltzmann_ratio():
    """For fixed energy gap 4m the fraction of draws below X(m) is
    exp(-(beta_hi - beta_lo) 4m) (binomial test over Philox exchange words)."""
    lo, hi = 0.5, 0.6
    N = 60000
    words = np.array([int(oracle.philox(77, (k % 7, q, k // 7, pt.TAG_EXCHANGE))[0])
                      for q in range(N // 60) for k in range(60)], np.uint64)
    for m in (1, 3, 7):
        x = pt.exchange_threshold(lo, hi, m)
        p = math.exp(-(hi - lo) * 4 * m)
        hits = int(np.count_nonzero(words < x))
        z = (hits - N * p) / math.sqrt(N * p * (1 - p))
        assert abs(z) < 5, (m, hits, N * p)
    xs = [pt.exchange_threshold(lo, hi, m) for m in range(1, 200)]
    assert all(a >= b for a, b in zip(xs, xs[1:])) and xs[-1] < xs[0]


@pytest.mark.parametrize("dims,betas", [([2, 4], (0.4, 1.0)), ([4, 2], (0.2, 0.6, 1.2))])
def test_ladders_sample_product_of_boltzmann(dims, betas):
    """Many independent ladders after 30 rounds of one sweep plus one exchange
    pass: the states found at each temperature follow exp(-beta H)/Z of that
    temperature (every state of the 8-spin torus enumerated)."""
    n = oracle.n_sites(dims)
    w = oracle.random_weights(31, len(dims) * n)
    L = 12000
    spins, energy, kidx, pos, log = pt.run_pt(dims, w, 5150, list(betas), L, 30, 1)
    assert sum(len(a) for a in log) > 0.05 * L * 30 * (len(betas) - 1) / 2  # exchanges do happen
    states = np.array([[1 if (k >> i) & 1 else -1 for i in range(n)] for k in range(2**n)], np.int8)
    _, en = oracle.cut_energy(dims, w, states)
    for k, beta in enumerate(betas):
        slots = pos[:, k]
        idx = ((spins[slots] > 0).astype(np.int64) << np.arange(n)).sum(axis=1)
        observed = np.bincount(idx, minlength=2**n)
        p = np.exp(-beta * (en - en.min()))
        p /= p.sum()
        expected = p * L
        order = np.argsort(expected)
        obs_b, exp_b, acc_o, acc_e = [], [], 0, 0.0
        for s in order:
            acc_o += observed[s]
            acc_e += expected[s]
            if acc_e >= 20:
                obs_b.append(acc_o)
                exp_b.append(acc_e)
                acc_o, acc_e = 0, 0.0
        obs_b[-1] += acc_o
        exp_b[-1] += acc_e
        assert stats.chisquare(obs_b, exp_b).pvalue > 1e-3, (k, beta)


def test_equal_temperatures_always_swap_and_leave_sweeps_unchanged():
    dims = [4, 6]
    n = 24
    w = oracle.random_weights(8, 2 * n)
    betas = [0.7] * 4
    L, Q, E = 2, 6, 3
    spins, energy, kidx, pos, log = pt.run_pt(dims, w, 9, betas, L, Q, E)
    for q, acc in enumerate(log):
        assert sorted(acc) == sorted((l, k) for l in range(L) for k in range(q % 2, 3, 2))
    # temperature labels do not change any threshold: the spins are those of fixed-beta runs
    rep = pt.ladder_thresholds(betas, 2)[np.zeros(L * 4, np.int64)]
    ref, _ = oracle.run_fixed(dims, w, 9, rep, 0, Q * E)
    assert (spins == ref).all()


def test_decisions_follow_energies_and_labels_stay_permutations():
    dims = [4, 6]
    n = 24
    w = oracle.random_weights(12, 2 * n)
    betas = [0.2, 0.35, 0.6, 1.0, 1.6]
    L, E = 3, 2
    kidx, pos = pt.new_labels(L, len(betas))
    spins = None
    metro = pt.ladder_thresholds(betas, 2)
    accepted_any = rejected_any = 0
    for q in range(25):
        spins, _ = oracle.run_fixed(dims, w, 4, metro[kidx], q * E, (q + 1) * E, spins=spins)
        _, energy = oracle.cut_energy(dims, w, spins)
        before = pos.copy()
        acc = set(pt.exchange(q, 4, energy, kidx, pos, betas))
        for l in range(L):
            assert sorted(pos[l]) == list(range(l * len(betas), (l + 1) * len(betas)))
            for k in range(len(betas)):
                assert kidx[pos[l, k]] == k
            for k in range(q % 2, len(betas) - 1, 2):
                a, b = before[l, k], before[l, k + 1]
                d = int(energy[a]) - int(energy[b])
                if d <= 0:
                    assert (l, k) in acc
                else:
                    u = int(oracle.philox(4, (k, q, l, pt.TAG_EXCHANGE))[0])
                    assert ((l, k) in acc) == (u < pt.exchange_threshold(betas[k], betas[k + 1], d // 4))
                    accepted_any += (l, k) in acc
                    rejected_any += (l, k) not in acc
    assert accepted_any and rejected_any


def test_rounds_resume_exactly():
    dims = [6, 4]
    n = 24
    w = oracle.random_weights(2, 2 * n)
    betas = [0.3, 0.5, 0.9, 1.4]
    full = pt.run_pt(dims, w, 17, betas, 2, 12, 3)
    a = pt.run_pt(dims, w, 17, betas, 2, 5, 3)
    b = pt.run_pt(dims, w, 17, betas, 2, 7, 3, round_begin=5, spins=a[0], kidx=a[2], pos=a[3])
    assert (b[0] == full[0]).all() and (b[1] == full[1]).all()
    assert (b[2] == full[2]).all() and (b[3] == full[3]).all()
