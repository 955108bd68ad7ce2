"""CPU oracle for checkerboard Metropolis annealing on +/-1 toroidal Ising /
Max-Cut instances.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product (the HIP library and its
Python binding) never does.  The arithmetic lives in plain C (oracle.c) and in
plain numpy float64 (mlp.py); this module only marshals numpy arrays.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

TAG_METROPOLIS, TAG_INIT, TAG_WEIGHT, TAG_MLP = 0, 1, 2, 3
SCHED_LINEAR, SCHED_GEOMETRIC, SCHED_TABLE = 0, 1, 2

_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        c_i64, c_i32, c_u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [c_u64, _u32p, _u32p]
        L.orc_n_sites.argtypes = [ctypes.c_int, _i32p]
        L.orc_n_sites.restype = c_i64
        L.orc_n_edges.argtypes = [ctypes.c_int, _i32p]
        L.orc_n_edges.restype = c_i64
        L.orc_torus_edges.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p]
        L.orc_site_colour.argtypes = [ctypes.c_int, _i32p, c_i64]
        L.orc_site_colour.restype = ctypes.c_int
        L.orc_random_weights.argtypes = [c_u64, c_i64, _i8p]
        L.orc_beta.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, c_i32, c_i32]
        L.orc_beta.restype = ctypes.c_double
        L.orc_threshold.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_threshold.restype = ctypes.c_uint32
        L.orc_init_spins.argtypes = [c_u64, c_i32, c_i32, c_i64, _i8p]
        L.orc_cut_energy.argtypes = [c_i64, c_i64, _i32p, _i32p, _i8p, c_i32, _i8p, _i64p, _i64p]
        L.orc_fields.argtypes = [ctypes.c_int, _i32p, _i8p, _i8p, _i32p]
        L.orc_run.argtypes = [ctypes.c_int, _i32p, _i8p, c_u64, c_i32, c_i32, c_i32, c_i32, c_i32,
                              ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                              ctypes.c_int, _i8p, _u32p, ctypes.c_void_p]
        L.orc_run.restype = ctypes.c_int
        L.orc_run_fixed.argtypes = [ctypes.c_int, _i32p, _i8p, c_u64, c_i32, c_i32, c_i32, c_i32, _u32p,
                                    ctypes.c_int, _i8p, _u32p]
        L.orc_run_fixed.restype = ctypes.c_int
        L.orc_maxcut_bruteforce.argtypes = [c_i64, c_i64, _i32p, _i32p, _i8p, ctypes.POINTER(ctypes.c_uint64)]
        L.orc_maxcut_bruteforce.restype = c_i64
        _lib = L
    return _lib


def _dims(dims):
    return np.ascontiguousarray(dims, dtype=np.int32)


def philox(key, ctr):
    """Philox4x32-10 block for 64-bit key and 4-word counter; returns uint32[4]."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(int(key), c, out)
    return out


def n_sites(dims):
    d = _dims(dims)
    return int(lib().orc_n_sites(len(d), d))


def torus_edges(dims):
    d = _dims(dims)
    ne = int(lib().orc_n_edges(len(d), d))
    a = np.zeros(ne, np.int32)
    b = np.zeros(ne, np.int32)
    lib().orc_torus_edges(len(d), d, a, b)
    return a, b


def colours(dims):
    d = _dims(dims)
    return np.array([lib().orc_site_colour(len(d), d, i) for i in range(n_sites(dims))], np.int32)


def random_weights(seed, n_edges):
    w = np.zeros(int(n_edges), np.int8)
    lib().orc_random_weights(int(seed), int(n_edges), w)
    return w


def beta(schedule, beta0, beta1, n_sweeps, t, table=None):
    tab = None if table is None else np.ascontiguousarray(table, np.float64)
    ptr = None if tab is None else tab.ctypes.data
    return float(lib().orc_beta(int(schedule), float(beta0), float(beta1), ptr, int(n_sweeps), int(t)))


def threshold(beta_value, k):
    return int(lib().orc_threshold(float(beta_value), int(k)))


def thresholds(schedule, beta0, beta1, n_sweeps, degree, table=None):
    """[S][degree/2] uint32 table of T_k(t), k = 1..degree/2."""
    out = np.zeros((n_sweeps, degree // 2), np.uint32)
    for t in range(n_sweeps):
        b = beta(schedule, beta0, beta1, n_sweeps, t, table)
        for k in range(1, degree // 2 + 1):
            out[t, k - 1] = threshold(b, k)
    return out


def init_spins(seed, n_replicas, n, replica_begin=0):
    s = np.zeros((n_replicas, n), np.int8)
    lib().orc_init_spins(int(seed), int(replica_begin), int(n_replicas), int(n), s)
    return s


def cut_energy(dims, w, spins):
    a, b = torus_edges(dims)
    spins = np.ascontiguousarray(spins, np.int8)
    if spins.ndim == 1:
        spins = spins[None, :]
    R, n = spins.shape
    cut = np.zeros(R, np.int64)
    en = np.zeros(R, np.int64)
    lib().orc_cut_energy(n, len(a), a, b, np.ascontiguousarray(w, np.int8), R, spins, cut, en)
    return cut, en


def fields(dims, w, spins_row):
    d = _dims(dims)
    f = np.zeros(n_sites(dims), np.int32)
    lib().orc_fields(len(d), d, np.ascontiguousarray(w, np.int8), np.ascontiguousarray(spins_row, np.int8), f)
    return f


def run(dims, w, seed, n_replicas, n_sweeps, begin=0, end=None, schedule=SCHED_LINEAR,
        beta0=0.1, beta1=3.0, table=None, spins=None, replica_begin=0, return_fields=False):
    """Run sweeps [begin, end); spins=None means Philox initial state (begin must be 0).

    Returns (spins [R][n] int8, flips [R] uint32) and, with return_fields, the
    maintained local fields [R][n] int32 at the end of the window."""
    d = _dims(dims)
    n = n_sites(dims)
    end = n_sweeps if end is None else end
    init = spins is None
    s = np.zeros((n_replicas, n), np.int8) if init else np.array(spins, dtype=np.int8, copy=True, order="C")
    fl = np.zeros(n_replicas, np.uint32)
    tab = None if table is None else np.ascontiguousarray(table, np.float64)
    ptr = None if tab is None else tab.ctypes.data
    fo = np.zeros((n_replicas, n), np.int32) if return_fields else None
    rc = lib().orc_run(len(d), d, np.ascontiguousarray(w, np.int8), int(seed), int(replica_begin),
                       int(n_replicas), int(n_sweeps), int(begin), int(end), int(schedule),
                       float(beta0), float(beta1), ptr, int(init), s, fl,
                       None if fo is None else fo.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the run arguments")
    return (s, fl, fo) if return_fields else (s, fl)


def run_fixed(dims, w, seed, rep_thr, begin, end, spins=None, replica_begin=0):
    """Sweeps [begin, end) with replica r at its own fixed thresholds
    rep_thr[r] (uint32 [R][deg/2]); spins=None: Philox initial state (begin
    must be 0).  Returns (spins, flips)."""
    d = _dims(dims)
    n = n_sites(dims)
    th = np.ascontiguousarray(rep_thr, np.uint32)
    R = th.shape[0]
    init = spins is None
    s = np.zeros((R, n), np.int8) if init else np.array(spins, dtype=np.int8, copy=True, order="C")
    fl = np.zeros(R, np.uint32)
    rc = lib().orc_run_fixed(len(d), d, np.ascontiguousarray(w, np.int8), int(seed), int(replica_begin), R,
                             int(begin), int(end), th, int(init), s, fl)
    if rc != 0:
        raise ValueError("oracle rejected the run arguments")
    return s, fl


def maxcut_bruteforce(dims, w):
    a, b = torus_edges(dims)
    n = n_sites(dims)
    st = ctypes.c_uint64(0)
    best = lib().orc_maxcut_bruteforce(n, len(a), a, b, np.ascontiguousarray(w, np.int8), ctypes.byref(st))
    bits = np.array([(st.value >> i) & 1 for i in range(n)], np.int8)
    return int(best), (2 * bits - 1).astype(np.int8)
