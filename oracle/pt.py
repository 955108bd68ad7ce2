"""Oracle of replica exchange (parallel tempering) over the sweep oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

L ladders of K inverse temperatures beta_0 <= ... <= beta_{K-1}; replica slot
r = l K + i of ladder l starts at temperature index i.  A round q runs sweeps
[qE, (q+1)E) with every replica at its own temperature (its Metropolis
thresholds T_k(beta), as in the annealing schedule), then one exchange pass
over the adjacent pairs (k, k+1) with k = q mod 2, q mod 2 + 2, ... of every
ladder: the replicas a (at beta_k) and b (at beta_{k+1}) swap temperatures
with probability min(1, exp((beta_k - beta_{k+1}) (H_a - H_b))) (the replica
exchange of Swendsen & Wang, 1986, and Hukushima & Nemoto, 1996), which
keeps the product of the K Boltzmann distributions stationary.

Integer decision, as for the sweeps: on a torus of even degree any two
energies differ by a multiple of 4, H_a - H_b = 4m.  m <= 0, or equal
temperatures, accept without a draw; otherwise accept iff u < X_k(m) =
min(2^32 - 1, floor(2^32 exp(-(beta_{k+1} - beta_k) 4m))), u = word 0 of
Philox(seed, (k, q, l, tag 4)).
"""
import math

import numpy as np

from . import cut_energy, philox, run_fixed, threshold

TAG_EXCHANGE = 4


def ladder_thresholds(betas, ndim):
    """Metropolis thresholds T_k(beta_i), k = 1..ndim: uint32 [K][ndim]."""
    return np.array([[threshold(b, k) for k in range(1, ndim + 1)] for b in betas], np.uint32)


def exchange_threshold(beta_lo, beta_hi, m):
    """X(m) for the pair (beta_lo, beta_hi), m >= 1."""
    x = (beta_hi - beta_lo) * (4.0 * m)
    return min(2**32 - 1, math.floor(math.ldexp(math.exp(-x), 32)))


def new_labels(n_ladders, K):
    """kidx[r] = temperature index of slot r; pos[l][k] = slot holding k."""
    kidx = np.array([r % K for r in range(n_ladders * K)], np.int64)
    pos = np.array([[l * K + k for k in range(K)] for l in range(n_ladders)], np.int64)
    return kidx, pos


def exchange(q, seed, energy, kidx, pos, betas):
    """One exchange pass of round q (in place); returns the accepted pairs [(l, k)]."""
    n_ladders, K = pos.shape
    accepted = []
    for l in range(n_ladders):
        for k in range(q % 2, K - 1, 2):
            a, b = int(pos[l, k]), int(pos[l, k + 1])
            d = int(energy[a]) - int(energy[b])
            assert d % 4 == 0
            if d <= 0 or betas[k + 1] == betas[k]:
                ok = True
            else:
                u = int(philox(seed, (k, q, l, TAG_EXCHANGE))[0])
                ok = u < exchange_threshold(betas[k], betas[k + 1], d // 4)
            if ok:
                pos[l, k], pos[l, k + 1] = b, a
                kidx[a], kidx[b] = k + 1, k
                accepted.append((l, k))
    return accepted


def run_pt(dims, w, seed, betas, n_ladders, n_rounds, sweeps_per_round, round_begin=0, spins=None, kidx=None,
           pos=None):
    """Rounds [round_begin, round_begin + n_rounds); spins=None: Philox initial
    state (round_begin must be 0).  Returns (spins, energy, kidx, pos, accepted
    pairs per round)."""
    K = len(betas)
    metro = ladder_thresholds(betas, len(dims))
    if kidx is None:
        kidx, pos = new_labels(n_ladders, K)
    kidx, pos = np.array(kidx, np.int64), np.array(pos, np.int64)
    E = sweeps_per_round
    log = []
    energy = None
    for q in range(round_begin, round_begin + n_rounds):
        spins, _ = run_fixed(dims, w, seed, metro[kidx], q * E, (q + 1) * E, spins=spins)
        _, energy = cut_energy(dims, w, spins)
        log.append(exchange(q, seed, energy, kidx, pos, betas))
    return spins, energy, kidx, pos, log
