"""The bit-sliced kernels' threshold compare chains on given words, against
plain numpy: bit j of a result is (word j < its threshold), strictly, each
word's threshold picked by its level bits (the paper's acceptance rule,
Section III, with the library's integer thresholds).  Words equal to, one
below and one above a threshold, 0 and 2^32 - 1 are planted; one wave of 64
sets holds only words above every threshold, so the screened forms skip
their chains there, and the next holds a single word below one, so they run
it for the whole wave."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# replica q's thresholds in the 16-word results, as indices into (T1, T2, T3)
A_PAT, B_PAT, C_PAT = (0, 1, 2, 0), (1, 0, 1, 2), (2, 2, 0, 1)
M32 = 0xFFFFFFFF


def pack(mask):
    """[n][32] booleans -> uint32 with bit j = mask[:, j]."""
    return (mask.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def reference(u, sel2, sel3, T):
    j = np.arange(32, dtype=np.uint64)
    b2 = ((sel2.astype(np.uint64)[:, None] >> j) & 1).astype(bool)
    b3 = ((sel3.astype(np.uint64)[:, None] >> j) & 1).astype(bool)
    T = np.array(T, dtype=np.int64)
    w = u.astype(np.int64)
    q = np.arange(32) & 3
    A, B, C = (T[list(p)][q] for p in (A_PAT, B_PAT, C_PAT))
    low = np.arange(32) < 16
    out = np.zeros((u.shape[0], 8), dtype=np.uint32)
    out[:, 0] = pack(w < np.where(b2, T[1], T[0]))
    out[:, 1] = pack(w < np.where(b3, T[2], np.where(b2, T[1], T[0])))
    out[:, 2] = pack((w < A) & low)
    out[:, 3], out[:, 4], out[:, 5] = (pack(w < T[k]) for k in range(3))
    out[:, 6] = pack((w < np.where(b2, B, A)) & low)
    out[:, 7] = pack((w < np.where(b3, C, np.where(b2, B, A))) & low)
    return out


def make_sets(seed, n, T):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, 2**32, size=(n, 32), dtype=np.uint64)
    level = rng.integers(0, 3, size=(n, 32))  # 0: T1, 1: T2, 2: T3 (disjoint selector bits)
    sel2 = pack(level == 1)
    sel3 = pack(level == 2)
    # planted edges: a threshold itself, one below, one above, and the extremes
    plant = rng.random((n, 32)) < 0.4
    k = rng.integers(0, 3, size=(n, 32))
    d = rng.integers(-1, 2, size=(n, 32))
    edge = np.clip(np.array(T, dtype=np.int64)[k] + d, 0, M32)
    edge = np.where(rng.random((n, 32)) < 0.15, rng.choice([0, M32], size=(n, 32)), edge)
    u = np.where(plant, edge, u).astype(np.uint64)
    # wave 1 (sets 64..127): every word above every threshold; wave 2: the same but one word below T3's
    # (or T1's) threshold, so each screen runs for the whole wave
    top = max(T)
    if n >= 192 and top < M32:
        high = rng.integers(top + 1, 2**32, size=(128, 32), dtype=np.uint64)
        u[64:192] = high
        lowest = min(t for t in T if t > 0) if any(T) else 0
        if lowest > 0:
            u[150, 7] = lowest - 1
    return u.astype(np.uint32), sel2, sel3


@pytest.mark.parametrize("T", [(M32, M32, M32), (3_000_000_000, 1_000_000_000, 5), (2**31, 2**31 - 1, 0),
                               (0, 0, 0), (123456, 1000, 7), (5, 1_000_000_000, 3_000_000_000),
                               (1 << 21, (1 << 21) - 1, 1), (M32 - 1, 2**16, 2**16)])
def test_compare_chains_match_numpy(T):
    import torch

    assert torch.cuda.is_available()
    import paper_2505_18508_amd as ising

    n = 64 * 5 + 17  # a ragged last wave
    u, sel2, sel3 = make_sets(sum(T) % 1000 + 7, n, T)
    dev = "cuda"
    out = torch.zeros((n, 8), dtype=torch.int32, device=dev)
    ising.compare_chains(torch.from_numpy(u.view(np.int32)).to(dev), torch.from_numpy(sel2.view(np.int32)).to(dev),
                         torch.from_numpy(sel3.view(np.int32)).to(dev), T[0], T[1], T[2], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = reference(u, sel2, sel3, T)
    bad = np.argwhere(got != want)
    assert len(bad) == 0, "set, result: %s" % bad[:8].tolist()
    if max(T) < M32 and any(T):
        # the all-high wave really produced zeros (every screen skipped) and the next did not
        assert (got[64:128, 3:6] == 0).all()
        assert got[150, 3:6].any()


def test_compare_chains_argument_errors():
    import torch

    assert torch.cuda.is_available()
    import paper_2505_18508_amd as ising

    L = ising.lib()
    assert L.ising_compare_chains(-1, None, None, None, 0, 0, 0, None, None) == ising.E_ARG
    assert L.ising_compare_chains(4, None, None, None, 0, 0, 0, None, None) == ising.E_ARG
    assert L.ising_compare_chains(0, None, None, None, 0, 0, 0, None, None) == ising.OK
