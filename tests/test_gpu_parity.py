"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs.  Spins, cuts, energies, flip counts and Philox
streams must agree bit for bit (integer work)."""
import numpy as np
import pytest

import oracle
from tests import inputs

pytestmark = pytest.mark.gpu

SCHED = {"linear": oracle.SCHED_LINEAR, "geometric": oracle.SCHED_GEOMETRIC, "table": oracle.SCHED_TABLE}
LAYOUTS = ["i8", "bp32", "stream", "bs4"]


def bs4_ok(dims):
    """The 4 x 4 bit-sliced layout takes every even torus (Ly = 2 mod 4: the
    last word line of each plane holds two rows)."""
    return True


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as ising

    ising.lib()
    return torch.device("cuda:0")


def _ising():
    import paper_2505_18508_amd as ising

    return ising


def run_gpu(dims, weight_seed, seed, R, S, begin=0, end=None, schedule="linear", beta0=0.1, beta1=3.0,
            table=None, spins0=None, layout="auto", block_threads=0, replica_offset=0, weights=None):
    import torch

    ising = _ising()
    g = ising.create_graph(dims, weight_seed, weights)
    n = g.n
    if spins0 is None:
        spins = torch.zeros((R, n), dtype=torch.int8, device="cuda")
    else:
        spins = torch.from_numpy(np.ascontiguousarray(spins0)).cuda()
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    fl = torch.zeros(R, dtype=torch.int32, device="cuda")
    ising.run_trials(g, spins, seed, S, begin, end, schedule, beta0, beta1, table, spins0 is None, layout,
                     cut, en, fl, block_threads, replica_offset)
    torch.cuda.synchronize()
    out = (spins.cpu().numpy(), cut.cpu().numpy(), en.cpu().numpy(), fl.cpu().numpy().astype(np.uint32))
    g.close()
    return out


def run_oracle(dims, weight_seed, seed, R, S, begin=0, end=None, schedule="linear", beta0=0.1, beta1=3.0,
               table=None, spins0=None, replica_begin=0, weights=None):
    n = oracle.n_sites(dims)
    w = oracle.random_weights(weight_seed, len(dims) * n) if weights is None else weights
    s, fl = oracle.run(dims, w, seed, R, S, begin, end, SCHED[schedule], beta0, beta1, table, spins0,
                       replica_begin=replica_begin)
    cut, en = oracle.cut_energy(dims, w, s)
    return s, cut, en, fl


def run_oracle_blocks(dims, weight_seed, seed, starts, width, S, begin=0, end=None, schedule="linear", beta0=0.1,
                      beta1=3.0, spins0=None):
    """Oracle outputs of the replica blocks [start, start + width), computed
    side by side on host threads (the C oracle keeps no global state and
    ctypes releases the interpreter lock during the call): {start: outputs}."""
    import concurrent.futures
    import os

    def one(start):
        sp = None if spins0 is None else spins0[start:start + width]
        return start, run_oracle(dims, weight_seed, seed, width, S, begin, end, schedule, beta0, beta1, spins0=sp,
                                 replica_begin=start)

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return dict(ex.map(one, list(starts)))


def assert_same(gpu, orc, rows=None):
    gs, gc, ge, gf = gpu
    if rows is not None:
        gs, gc, ge, gf = gs[rows], gc[rows], ge[rows], gf[rows]
    os_, oc, oe, of = orc
    assert gs.shape == os_.shape
    mism = np.nonzero((gs != os_).any(axis=1))[0]
    assert len(mism) == 0, "replicas differ: %s" % mism[:10]
    assert (gc == oc).all() and (ge == oe).all()
    assert (gf == of).all()


# --------------------------------------------------------------------------
def test_philox_stream_matches_oracle(dev):
    import torch

    rng = np.random.default_rng(1)
    m = 4096
    ctr = rng.integers(0, 2**32, size=(m, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:16] = [[i, t, q, tag] for i in range(2) for t in range(2) for q in range(2) for tag in range(2)]
    key = 0x0123456789ABCDEF
    c = torch.from_numpy(ctr.view(np.int32)).cuda()
    out = torch.zeros((m, 4), dtype=torch.int32, device="cuda")
    _ising().philox_dump(key, c, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    for k in list(range(64)) + list(rng.integers(0, m, size=200)):
        assert (got[k] == oracle.philox(key, ctr[k])).all(), k


@pytest.mark.parametrize("layout", LAYOUTS)
def test_torus50x100_full_run_bit_exact(dev, layout):
    c = inputs.TORUS_50x100_R16
    dims = c["dims"]  # 50 rows: the bit-sliced layout's last word line holds two
    gpu = run_gpu(dims, c["weight_seed"], c["seed"], c["R"], c["S"], schedule=c["schedule"],
                  beta0=c["beta0"], beta1=c["beta1"], layout=layout)
    orc = run_oracle(dims, c["weight_seed"], c["seed"], c["R"], c["S"], schedule=c["schedule"],
                     beta0=c["beta0"], beta1=c["beta1"])
    assert_same(gpu, orc)


_C2_ORACLE = {}


@pytest.mark.parametrize("layout", LAYOUTS)
def test_torus100x100_first_200_sweeps_every_replica(dev, layout):
    """All 1,024 replicas for sweeps [0, 200) of the 10,000-sweep schedule,
    every one recomputed by the oracle (once, shared by the layouts)."""
    c = inputs.TORUS_100x100_R1024
    gpu = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, 200, c["schedule"], c["beta0"], c["beta1"],
                  layout=layout)
    if not _C2_ORACLE:
        print("oracle: 1,024 replicas x 200 sweeps", flush=True)
        _C2_ORACLE.update(run_oracle_blocks(c["dims"], c["weight_seed"], c["seed"], range(0, c["R"], 16), 16, c["S"],
                                            0, 200, c["schedule"], c["beta0"], c["beta1"]))
    for start, orc in sorted(_C2_ORACLE.items()):
        assert_same(gpu, orc, rows=slice(start, start + 16))


def test_torus100x100_full_schedule_in_bench_launch_sampled(dev):
    """The configuration of the 10,000-spin benchmark: all 1,024 replicas
    through the whole 10,000-sweep schedule in one launch of the
    automatically chosen packing; the oracle recomputes 16 replica quads
    spread over the run end to end (64 replicas)."""
    c = inputs.TORUS_100x100_R1024
    gpu = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, c["S"], c["schedule"], c["beta0"],
                  c["beta1"], layout="auto")
    starts = [4 * (k * (c["R"] // 4 - 1) // 15) for k in range(16)]
    assert starts[0] == 0 and starts[-1] == c["R"] - 4
    print("oracle quads", starts, flush=True)
    for start, orc in run_oracle_blocks(c["dims"], c["weight_seed"], c["seed"], starts, 4, c["S"], 0, c["S"],
                                        c["schedule"], c["beta0"], c["beta1"]).items():
        assert_same(gpu, orc, rows=slice(start, start + 4))


def test_torus100x100_layouts_agree_on_every_replica(dev):
    """i8, bp32 and bs4 packings give identical spins, cuts, energies and
    flip counts on all 1,024 replicas of sweeps [0, 200)."""
    c = inputs.TORUS_100x100_R1024
    a = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, 200, c["schedule"], c["beta0"], c["beta1"],
                layout="i8")
    for other in ("bp32", "bs4"):
        b = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, 200, c["schedule"], c["beta0"],
                    c["beta1"], layout=other)
        for x, y in zip(a, b):
            assert (x == y).all()


def test_torus100x200_full_schedule_in_bench_launch_sampled(dev):
    """The 20,000-spin workload as timed: all 8,192 replicas through the whole
    40,000-sweep schedule in one launch of the automatically chosen packing
    (32 replicas per word, flip counters flushed every few sweeps); the oracle
    recomputes four replica quads end to end: the first, two in the middle
    (in the first and the last of the 256 32-replica groups' halves) and the
    last."""
    c = inputs.TORUS_100x200_R8192
    gpu = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, c["S"], c["schedule"], c["beta0"],
                  c["beta1"], layout="auto")
    starts = [0, 2732, 4100, c["R"] - 4]
    print("oracle quads", starts, flush=True)
    # one replica per task: a replica's whole schedule is 8e8 attempts
    reps = run_oracle_blocks(c["dims"], c["weight_seed"], c["seed"], [q + b for q in starts for b in range(4)], 1,
                             c["S"], 0, c["S"], c["schedule"], c["beta0"], c["beta1"])
    for r, orc in reps.items():
        assert_same(gpu, orc, rows=slice(r, r + 1))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_torus100x200_short_window_sampled(dev, layout):
    """The 20,000-spin torus with 8,192 replicas (full launch shape), 30 sweeps."""
    c = inputs.TORUS_100x200_R8192
    gpu = run_gpu(c["dims"], c["weight_seed"], c["seed"], c["R"], c["S"], 0, 30, c["schedule"], c["beta0"], c["beta1"],
                  layout=layout)
    for start in (0, 4096, 8188):
        orc = run_oracle(c["dims"], c["weight_seed"], c["seed"], 4, c["S"], 0, 30, c["schedule"], c["beta0"],
                         c["beta1"], replica_begin=start)
        assert_same(gpu, orc, rows=slice(start, start + 4))


@pytest.mark.parametrize("dims,R", [([2, 2], 5), ([2, 4], 3), ([4, 2], 8), ([4, 6], 13), ([6, 8], 1), ([2, 6], 7),
                                    ([2, 2, 2], 6), ([4, 4, 6], 9), ([6, 8, 10], 4), ([2, 4, 2], 2),
                                    ([34, 18], 11), ([10, 1000], 3), ([6, 4], 37), ([8, 6, 4], 33),
                                    ([8, 6], 6), ([12, 10], 17), ([4, 1000], 5), ([2, 8, 6], 3), ([20, 34], 9),
                                    ([14, 600], 6)])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_small_and_ragged_tori(dev, dims, R, layout):
    if layout == "bs4" and not bs4_ok(dims):
        pytest.skip("bs4 needs the second-fastest axis divisible by 4")
    gpu = run_gpu(dims, 7, 55, R, 300, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout)
    orc = run_oracle(dims, 7, 55, R, 300, schedule="geometric", beta0=0.05, beta1=4.0)
    assert_same(gpu, orc)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_3d_degree6_torus(dev, layout):
    dims = [16, 16, 16]
    gpu = run_gpu(dims, 643, 9, 40, 120, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout)
    orc = run_oracle(dims, 643, 9, 40, 120, schedule="geometric", beta0=0.05, beta1=4.0)
    assert_same(gpu, orc)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_given_spins_and_weights_and_table_schedule(dev, layout):
    dims = [20, 30]
    n = 600
    w = inputs.random_weights(5, 2 * n)
    s0 = inputs.random_spins(6, 42, n)
    table = np.linspace(0.3, 2.5, 150)
    table[:5] = 0.0  # beta = 0: every proposal accepted except with probability 2^-32
    gpu = run_gpu(dims, 0, 77, 42, 150, schedule="table", table=table, spins0=s0, weights=w, layout=layout)
    orc = run_oracle(dims, 0, 77, 42, 150, schedule="table", table=table, spins0=s0, weights=w)
    assert_same(gpu, orc)


# beta at which thresholds vanish: T_k = 0 once 4 k beta > 32 ln 2 (k = 3: 1.85, k = 2: 2.77,
# k = 1: 5.55); past the last, only dE <= 0 flips remain and no draw is taken
LEVEL_TABLE = [0.0, 0.4, 1.0, 1.8, 1.9, 2.7, 2.8, 3.5, 5.5, 5.6, 7.0, 12.0]


@pytest.mark.parametrize("dims", [[20, 30], [6, 8, 10], [6, 10]])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_threshold_levels_vanishing_and_zero_temperature(dev, layout, dims):
    n = oracle.n_sites(dims)
    table = np.array(LEVEL_TABLE * 6)  # back and forth between hot and zero-temperature sweeps
    s0 = inputs.random_spins(12, 19, n)
    w = inputs.random_weights(13, len(dims) * n)
    gpu = run_gpu(dims, 0, 91, 19, len(table), schedule="table", table=table, spins0=s0, weights=w, layout=layout)
    orc = run_oracle(dims, 0, 91, 19, len(table), schedule="table", table=table, spins0=s0, weights=w)
    assert_same(gpu, orc)
    assert oracle.threshold(12.0, 1) == 0 and oracle.threshold(1.9, 3) == 0 and oracle.threshold(1.8, 3) > 0


# beta on either side of where the smallest nonzero threshold crosses 2^21, the bound below
# which the 32-replica kernels screen their compares per wave: T_2 at 0.953 / 0.9531 (2-D),
# T_3 at 0.6353 / 0.6356 (3-D); hot and cold sweeps between them
SCREEN_TABLE = [0.953, 0.9531, 0.953, 0.9532, 0.6353, 0.6356, 0.6353, 0.3, 2.0, 0.6356, 0.9531, 0.953]


@pytest.mark.parametrize("dims", [[20, 30], [6, 8, 10]])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_sweeps_alternating_across_the_compare_screen_bound(dev, layout, dims):
    n = oracle.n_sites(dims)
    table = np.array(SCREEN_TABLE * 5)
    s0 = inputs.random_spins(14, 45, n)
    w = inputs.random_weights(15, len(dims) * n)
    gpu = run_gpu(dims, 0, 93, 45, len(table), schedule="table", table=table, spins0=s0, weights=w, layout=layout)
    orc = run_oracle(dims, 0, 93, 45, len(table), schedule="table", table=table, spins0=s0, weights=w)
    assert_same(gpu, orc)
    assert oracle.threshold(0.953, 2) >= 2**21 > oracle.threshold(0.9531, 2)
    assert oracle.threshold(0.6353, 3) >= 2**21 > oracle.threshold(0.6356, 3)


@pytest.mark.parametrize("dims", [[20, 30], [6, 8, 10], [6, 10]])
@pytest.mark.parametrize("layout", ["bs4", "i8"])
def test_replica_thresholds_mixing_zero_and_hot_replicas(dev, layout, dims):
    """Per-replica temperatures where some quads are entirely at zero
    temperature, some mix vanishing levels, some are hot."""
    import torch

    from oracle import pt as opt

    ising = _ising()
    n = oracle.n_sites(dims)
    betas = [12.0, 12.0, 12.0, 12.0, 0.0, 12.0, 2.8, 1.9, 5.6, 5.5, 0.4, 12.0, 1.0, 1.0, 3.5, 7.0, 0.3]
    R = len(betas)
    rep = opt.ladder_thresholds(betas, len(dims))
    s0 = inputs.random_spins(14, R, n)
    w = inputs.random_weights(15, len(dims) * n)
    g = ising.create_graph(dims, 0, w)
    spins = torch.from_numpy(s0.copy()).cuda()
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    fl = torch.zeros(R, dtype=torch.int32, device="cuda")
    ising.run_trials(g, spins, 23, 60, 0, 60, "linear", 0.0, 0.0, None, False, layout, cut, en, fl,
                     replica_thresholds=torch.from_numpy(rep.astype(np.int32)).cuda())
    torch.cuda.synchronize()
    ref, rfl = oracle.run_fixed(dims, w, 23, rep, 0, 60, spins=s0)
    rc, re_ = oracle.cut_energy(dims, w, ref)
    assert (spins.cpu().numpy() == ref).all()
    assert (fl.cpu().numpy().astype(np.uint32) == rfl).all()
    assert (cut.cpu().numpy() == rc).all() and (en.cpu().numpy() == re_).all()
    g.close()


@pytest.mark.parametrize("dims", [[10, 12], [4, 6, 8]])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_64bit_seeds_and_large_replica_offsets(dev, layout, dims):
    """Both key words of Philox come from the run and weight seeds, and the
    replica quad counter from offsets far beyond the replicas of the run."""
    seed, wseed, off = 0xFEDCBA9876543210, 0x8000000100000003, 2**30 + 4
    gpu = run_gpu(dims, wseed, seed, 7, 50, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout,
                  replica_offset=off)
    orc = run_oracle(dims, wseed, seed, 7, 50, schedule="geometric", beta0=0.05, beta1=4.0, replica_begin=off)
    assert_same(gpu, orc)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_window_resume_equals_single_run(dev, layout):
    dims = [40, 50]
    full = run_gpu(dims, 3, 8, 40, 400, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout)
    a = run_gpu(dims, 3, 8, 40, 400, 0, 170, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout)
    b = run_gpu(dims, 3, 8, 40, 400, 170, 400, schedule="geometric", beta0=0.05, beta1=4.0, spins0=a[0],
                layout=layout)
    assert (b[0] == full[0]).all() and (b[1] == full[1]).all()
    assert (a[3] + b[3] == full[3]).all()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_replica_offset_selects_streams(dev, layout):
    dims = [12, 10]
    full = run_gpu(dims, 3, 8, 80, 100, layout=layout)
    part = run_gpu(dims, 3, 8, 40, 100, replica_offset=12, layout=layout)
    assert (part[0] == full[0][12:52]).all()


@pytest.mark.parametrize("rows", [50, 48])
@pytest.mark.parametrize("bt", [1, 100, 300, 512, 1000])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_block_size_does_not_change_results(dev, bt, layout, rows):
    """Every block size walks a thread's lines differently (one word line per
    pass up to whole blocks; bp32 pairs of middle lines with an odd one left
    over; bs4 on 48 rows takes the 2-D walk with per-thread wrap offsets, on
    50 the general one): results equal the i8 layout's."""
    c = inputs.TORUS_50x100_R16
    dims = [rows, c["dims"][1]]
    ref = run_gpu(dims, c["weight_seed"], c["seed"], 36, 200, schedule="linear", layout="i8")
    got = run_gpu(dims, c["weight_seed"], c["seed"], 36, 200, schedule="linear", block_threads=bt, layout=layout)
    for x, y in zip(ref, got):
        assert (x == y).all()
    if rows == 48 and bt == 1000:
        orc = run_oracle(dims, c["weight_seed"], c["seed"], 36, 200, schedule="linear")
        assert_same(got, orc)


@pytest.mark.parametrize("dims", [[48, 100], [80, 80]])
def test_bs4_default_block_with_many_quads_per_cu(dev, dims):
    """4,096 replicas (four quads per CU): the default bs4 block shrinks to at
    most 512 threads; results equal the largest block's and the oracle's."""
    R, S = 4096, 20
    hx = dims[1] // 2
    full = min(1024 // hx, (dims[0] + 3) // 4) * hx
    got = run_gpu(dims, 3, 17, R, S, schedule="geometric", beta0=0.05, beta1=4.0, layout="bs4")
    ref = run_gpu(dims, 3, 17, R, S, schedule="geometric", beta0=0.05, beta1=4.0, layout="bs4", block_threads=full)
    for x, y in zip(ref, got):
        assert (x == y).all()
    for r0 in (0, 1000, 4088):
        orc = run_oracle(dims, 3, 17, 8, S, schedule="geometric", beta0=0.05, beta1=4.0, replica_begin=r0)
        assert_same(got, orc, rows=slice(r0, r0 + 8))


@pytest.mark.parametrize("layout,dims", [("i8", [200, 202]), ("bp32", [180, 180]), ("bs4", [172, 172]),
                                          ("bs4", [170, 172]), ("bs4", [12, 30, 56])])
def test_largest_on_chip_torus(dev, layout, dims):
    # i8: 40,400 sites = 161,600 B of state + 272 B of tables per block; bp32: 32,400 sites = 162,448 B;
    # bs4: 29,584 sites = 3,698 records of 44 B = 162,712 B + 64 B; 170 rows (2 mod 4) fill 43 word lines
    # of 86 records as well, the last of each plane holding two rows; 3-D 12 x 30 x 56: 2,688 records of 60 B
    gpu = run_gpu(dims, 4, 4, 5, 20, schedule="geometric", beta0=0.05, beta1=4.0, layout=layout)
    orc = run_oracle(dims, 4, 4, 5, 20, schedule="geometric", beta0=0.05, beta1=4.0)
    assert_same(gpu, orc)


def test_too_large_torus_is_rejected(dev):
    import torch

    ising = _ising()
    g = ising.create_graph([256, 256], 1)
    s = torch.zeros((4, g.n), dtype=torch.int8, device="cuda")
    for layout in ("i8", "bp32"):  # AUTO streams it from HBM instead
        with pytest.raises(ising.IsingError) as e:
            ising.run_trials(g, s, 1, 10, layout=layout)
        assert e.value.code == ising.E_UNSUPPORTED
    g2 = ising.create_graph([200, 202], 1)
    s2 = torch.zeros((4, g2.n), dtype=torch.int8, device="cuda")
    for layout in ("bp32", "bs4"):
        with pytest.raises(ising.IsingError) as e:
            ising.run_trials(g2, s2, 1, 10, layout=layout)
        assert e.value.code == ising.E_UNSUPPORTED


@pytest.mark.parametrize("entry", ["run_trials", "run_trials_noalloc"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_degenerate_windows_and_zero_replicas_are_rejected(dev, layout, entry):
    """An empty window, one past the schedule's end, one running backwards and
    a call with no replicas are argument errors that leave the spins as they
    were; a one-sweep schedule runs (its single beta is beta0)."""
    import torch

    ising = _ising()
    run = getattr(ising, entry)
    dims = [8, 12]
    g = ising.create_graph(dims, 3)
    s = torch.ones((8, g.n), dtype=torch.int8, device="cuda")
    for begin, end in ((5, 5), (0, 11), (6, 4)):
        with pytest.raises(ising.IsingError) as e:
            run(g, s, 1, 10, begin, end, layout=layout, init_spins=False)
        assert e.value.code == ising.E_ARG
    torch.cuda.synchronize()
    assert (s == 1).all()
    empty = torch.zeros((0, g.n), dtype=torch.int8, device="cuda")
    with pytest.raises(ising.IsingError) as e:
        run(g, empty, 1, 10, layout=layout)
    assert e.value.code == ising.E_ARG
    g.close()
    gpu = run_gpu(dims, 3, 5, 8, 1, layout=layout)
    orc = run_oracle(dims, 3, 5, 8, 1)
    assert_same(gpu, orc)


@pytest.mark.parametrize("dims", [[200, 204], [40, 40, 40]])
def test_bs4_rejects_lattices_too_large_for_lds(dev, dims):
    """A forced bit-sliced packing of a lattice whose records exceed a block's LDS."""
    import torch

    ising = _ising()
    g = ising.create_graph(dims, 1)
    s = torch.zeros((4, g.n), dtype=torch.int8, device="cuda")
    with pytest.raises(ising.IsingError) as e:
        ising.run_trials(g, s, 1, 10, layout="bs4")
    assert e.value.code == ising.E_UNSUPPORTED


@pytest.mark.parametrize("layout", LAYOUTS)
def test_invalid_input_spins_flagged(dev, layout):
    import torch

    ising = _ising()
    g = ising.create_graph([8, 6], 2)
    s0 = inputs.random_spins(1, 8, g.n)
    s0[3, 7] = 0
    s0[5, 0] = 3
    s = torch.from_numpy(s0).cuda()
    cut = torch.zeros(8, dtype=torch.int64, device="cuda")
    en = torch.zeros(8, dtype=torch.int64, device="cuda")
    ising.run_trials(g, s, 1, 10, init_spins=False, cut=cut, energy=en, layout=layout)
    torch.cuda.synchronize()
    c = cut.cpu().numpy()
    assert c[3] == ising.INVALID_VALUE and c[5] == ising.INVALID_VALUE
    assert (np.delete(c, [3, 5]) != ising.INVALID_VALUE).all()


def test_argument_errors(dev):
    import torch

    ising = _ising()
    g = ising.create_graph([6, 8], 2)
    s = torch.zeros((4, g.n), dtype=torch.int8, device="cuda")
    cases = [dict(n_sweeps=10, sweep_begin=5, sweep_end=5), dict(n_sweeps=10, sweep_begin=0, sweep_end=11),
             dict(n_sweeps=10, sweep_begin=2, sweep_end=5, init_spins=True), dict(n_sweeps=10, schedule="geometric", beta0=0.0),
             dict(n_sweeps=10, replica_offset=2)]
    for kw in cases:
        n_sweeps = kw.pop("n_sweeps")
        with pytest.raises(ising.IsingError) as e:
            ising.run_trials(g, s, 1, n_sweeps, **kw)
        assert e.value.code == ising.E_ARG, kw
    # short or mistyped output buffers never reach a kernel
    short = torch.zeros(3, dtype=torch.int64, device="cuda")
    for kw in (dict(cut=short), dict(energy=short), dict(flips=torch.zeros(4, dtype=torch.int64, device="cuda"))):
        with pytest.raises(ValueError):
            ising.run_trials(g, s, 1, 10, **kw)
    with pytest.raises(ValueError):
        ising.eval_cut(g, s, short, None)
    with pytest.raises(ValueError):
        ising.run_trials(g, s.to(torch.int32), 1, 10)


# --------------------------------------------------------------------------
# eval_cut
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [[50, 100], [2, 2], [4, 6], [100, 200], [6, 4, 8], [64, 64, 64]])
def test_eval_cut_matches_oracle(dev, dims):
    import torch

    ising = _ising()
    g = ising.create_graph(dims, 11)
    n = g.n
    R = 9
    s0 = inputs.random_spins(2, R, n)
    s0[1] = 1
    s0[2] = -1
    s0[3] = np.where(oracle.colours(dims) == 0, 1, -1) if n <= 50000 else s0[3]
    s = torch.from_numpy(s0).cuda()
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    ising.eval_cut(g, s, cut, en)
    torch.cuda.synchronize()
    w = oracle.random_weights(11, len(dims) * n)
    oc, oe = oracle.cut_energy(dims, w, s0)
    assert (cut.cpu().numpy() == oc).all() and (en.cpu().numpy() == oe).all()
    assert (g.weights() == w).all()


def test_eval_cut_flags_invalid_values(dev):
    import torch

    ising = _ising()
    g = ising.create_graph([4, 6], 1)
    s0 = inputs.random_spins(3, 4, g.n)
    s0[2, 5] = 0
    s = torch.from_numpy(s0).cuda()
    cut = torch.zeros(4, dtype=torch.int64, device="cuda")
    ising.eval_cut(g, s, cut, None)
    torch.cuda.synchronize()
    c = cut.cpu().numpy()
    assert c[2] == ising.INVALID_VALUE and (np.delete(c, 2) != ising.INVALID_VALUE).all()


def test_eval_cut_empty(dev):
    import torch

    ising = _ising()
    g = ising.create_graph([4, 6], 1)
    s = torch.zeros((0, g.n), dtype=torch.int8, device="cuda")
    ising.eval_cut(g, s, None, None)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dims", [[1000, 1000], [64, 64, 64]])
def test_streamed_stress_tori_sampled(dev, dims):
    """Lattices larger than a block's LDS run from HBM (AUTO picks it); 64
    replicas, sweeps [0, 6) of a 2,000-sweep schedule; the oracle recomputes
    the first and last replica quads."""
    wseed = 1000 if len(dims) == 2 else 643
    gpu = run_gpu(dims, wseed, 77, 64, 2000, 0, 6, schedule="geometric", beta0=0.05, beta1=4.0, layout="auto")
    for start in (0, 60):
        orc = run_oracle(dims, wseed, 77, 4, 2000, 0, 6, "geometric", 0.05, 4.0, replica_begin=start)
        assert_same(gpu, orc, rows=slice(start, start + 4))


@pytest.mark.parametrize("dims", [[1000, 1000], [64, 64, 64]])
def test_streamed_stress_tori_cold_end_every_replica(dev, dims):
    """The full streamed launch shape (256 replicas) at the cold end of the
    2,000-sweep schedule: sweeps [1990, 2000) from a seeded state, where the
    second threshold level has vanished and almost every draw is rejected;
    all 256 replicas recomputed by the oracle from the same state."""
    wseed = 1000 if len(dims) == 2 else 643
    R = 256
    n = int(np.prod(dims))
    start = inputs.random_spins(4242, R, n)
    gpu = run_gpu(dims, wseed, 7, R, 2000, 1990, 2000, schedule="geometric", beta0=0.05, beta1=4.0, spins0=start,
                  layout="auto")
    print("oracle: 256 replicas x 10 sweeps", flush=True)
    for b, orc in run_oracle_blocks(dims, wseed, 7, range(0, R, 16), 16, 2000, 1990, 2000, "geometric", 0.05, 4.0,
                                    spins0=start).items():
        assert_same(gpu, orc, rows=slice(b, b + 16))


def test_streamed_matches_on_chip_layouts(dev):
    dims = [40, 60]
    a = run_gpu(dims, 9, 3, 70, 300, schedule="geometric", beta0=0.05, beta1=4.0, layout="stream")
    b = run_gpu(dims, 9, 3, 70, 300, schedule="geometric", beta0=0.05, beta1=4.0, layout="bp32")
    c = run_gpu(dims, 9, 3, 70, 300, schedule="geometric", beta0=0.05, beta1=4.0, layout="i8")
    for x, y, z in zip(a, b, c):
        assert (x == y).all() and (x == z).all()


@pytest.mark.parametrize("dims,R,want", [([100, 100], 1024, "bs4"), ([100, 200], 8192, "bp32"), ([50, 100], 16, "bs4"),
                                         ([1000, 1000], 256, "stream"), ([200, 202], 4, "i8"),
                                         ([64, 64, 64], 256, "stream"), ([16, 16, 16], 40, "bs4"),
                                         ([8, 6, 8], 8, "bs4")])
def test_select_layout_reports_the_auto_choice(dev, dims, R, want):
    ising = _ising()
    g = ising.create_graph(dims, 1)
    assert ising.select_layout(g, R) == want
    assert ising.select_layout(g, R, layout="stream") == "stream"
    g.close()
