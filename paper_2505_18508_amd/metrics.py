"""Readout of a campaign of trials (paper, Section III): success probability
against a target cut, repetitions r for 99% confidence (eq. (3)),
sweeps-to-target (eq. (4)) and time-to-target (eq. (5)); the 99.9% target
rule of Table I; and the solution-bitstring format of Appendices C-E.
Host-side arithmetic on results the GPU has produced."""
import math

import numpy as np


def target_cut(best, quality=0.999):
    """Smallest integer cut reaching `quality` of the best cut (Table I prints
    the 99.9% targets as 0.999 * best, e.g. >= 14045.94 for 14060)."""
    return int(math.ceil(quality * best - 1e-9))


def success_probability(cuts, target):
    """Fraction of trials whose end-of-trial cut reaches the target (solutions
    are read out at the end of each trial)."""
    cuts = np.asarray(cuts)
    if cuts.size == 0:
        raise ValueError("no trials")
    return float(np.count_nonzero(cuts >= target)) / cuts.size


def repetitions(p_s, confidence=0.99):
    """eq. (3): r = max(1, log(1 - confidence) / log(1 - P_s)); infinite when
    no trial reached the target."""
    if not 0.0 <= p_s <= 1.0:
        raise ValueError("P_s must be in [0, 1]")
    if p_s == 0.0:
        return math.inf
    if p_s == 1.0:
        return 1.0
    return max(1.0, math.log(1.0 - confidence) / math.log(1.0 - p_s))


def sweeps_to_target(sweeps_per_trial, p_s):
    """eq. (4): STT = S_trial * r."""
    return sweeps_per_trial * repetitions(p_s)


def time_to_target(seconds_per_trial, p_s):
    """eq. (5): TTT = t_trial * r, t_trial the average time of one trial."""
    return seconds_per_trial * repetitions(p_s)


def decode_hex_solution(text, n):
    """Spins of a solution bitstring: hexadecimal digits expand to bits for
    variables 1..n, bit 0 -> spin -1 and bit 1 -> +1 (Appendices C-E).  The
    most significant bit of each digit is taken first (the paper does not
    state the order within a digit).  Whitespace is ignored; the string must
    hold exactly ceil(n / 4) digits and any padding bits must be zero."""
    digits = "".join(text.split()).lower()
    need = (n + 3) // 4
    if len(digits) != need:
        raise ValueError("expected %d hex digits for %d variables, got %d" % (need, n, len(digits)))
    try:
        vals = [int(c, 16) for c in digits]
    except ValueError:
        raise ValueError("not a hexadecimal string")
    bits = np.zeros(4 * need, np.int8)
    for k, v in enumerate(vals):
        for b in range(4):
            bits[4 * k + b] = (v >> (3 - b)) & 1
    if bits[n:].any():
        raise ValueError("nonzero padding bits")
    return (2 * bits[:n] - 1).astype(np.int8)


def encode_hex_solution(spins):
    """Inverse of decode_hex_solution."""
    s = np.asarray(spins)
    n = s.size
    bits = np.zeros(4 * ((n + 3) // 4), np.int8)
    bits[:n] = (s > 0).astype(np.int8)
    out = []
    for k in range(0, bits.size, 4):
        out.append("%x" % (bits[k] << 3 | bits[k + 1] << 2 | bits[k + 2] << 1 | bits[k + 3]))
    return "".join(out)
