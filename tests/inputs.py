"""Seeded synthetic inputs shared by the GPU-path tests and the oracle side.

Holds none of the method's arithmetic: only random +/-1 arrays and the
instance shapes used by the tests."""
import numpy as np

# Torus shapes of the workloads (2-D {rows, cols}, 3-D {Lz, Ly, Lx}): the
# paper's toroidal grids of 5,000 / 10,000 / 14,000 / 20,000 spins
# (Table I, Appendix A), and the 3-D degree-6 torus.
TORUS_50x100_R16 = dict(dims=[50, 100], weight_seed=1, seed=101, R=16, S=1000, schedule="linear", beta0=0.1, beta1=3.0)
TORUS_100x100_R1024 = dict(dims=[100, 100], weight_seed=2, seed=102, R=1024, S=10000, schedule="geometric", beta0=0.05, beta1=4.0)
TORUS_100x200_R8192 = dict(dims=[100, 200], weight_seed=81, seed=201, R=8192, S=40000, schedule="geometric", beta0=0.05, beta1=4.0)
# lattices too large for a block's LDS, streamed from HBM
TORUS_1000x1000_R256 = dict(dims=[1000, 1000], weight_seed=1000, seed=7, R=256, S=2000, schedule="geometric", beta0=0.05,
                            beta1=4.0)
TORUS_64x64x64_R256 = dict(dims=[64, 64, 64], weight_seed=643, seed=7, R=256, S=2000, schedule="geometric", beta0=0.05,
                           beta1=4.0)


def random_spins(seed, n_replicas, n):
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, size=(n_replicas, n)) - 1).astype(np.int8)


def random_weights(seed, n_edges):
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, size=n_edges) - 1).astype(np.int8)
