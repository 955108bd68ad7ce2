"""Python binding of libising.so, the MI355X (gfx950) library for
replica-parallel checkerboard Metropolis annealing on +/-1 toroidal Ising /
Max-Cut instances (paper: maximise eq. (1); Ising form eq. (2) with J = -w,
h = 0; trial length in sweeps, Section III).

This module only marshals arguments to the C ABI declared in
include/ising.h; every step of the computation runs in the library's HIP
kernels.  torch is used for device memory and streams only.  If the library
has not been built the import of the binding fails loudly: there is no CPU
fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libising.so")

OK, E_ARG, E_TOPOLOGY, E_NOMEM, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
SCHED_LINEAR, SCHED_GEOMETRIC, SCHED_TABLE = 0, 1, 2
LAYOUT_AUTO, LAYOUT_I8, LAYOUT_BP32, LAYOUT_STREAM, LAYOUT_BS4 = 0, 1, 2, 3, 4
INVALID_VALUE = -(2**63)

SCHEDULES = {"linear": SCHED_LINEAR, "geometric": SCHED_GEOMETRIC, "table": SCHED_TABLE}
LAYOUTS = {"auto": LAYOUT_AUTO, "i8": LAYOUT_I8, "bp32": LAYOUT_BP32, "stream": LAYOUT_STREAM, "bs4": LAYOUT_BS4}

EXPORTED = [
    "ising_create_graph", "ising_destroy_graph", "ising_graph_info", "ising_graph_weights",
    "ising_generate_weights", "ising_run_trials", "ising_run_trials_noalloc", "ising_select_layout", "ising_eval_cut", "ising_thresholds",
    "ising_philox_dump", "ising_last_error",
    "ising_features", "ising_mlp_init", "ising_mlp_forward", "ising_mlp_workspace_floats", "ising_mlp_loss_grad",
    "ising_adam_step", "ising_feature_stats", "ising_cull_clone", "ising_energy_score", "ising_schedule_beta",
    "ising_batch_create", "ising_batch_run", "ising_batch_info", "ising_batch_destroy", "ising_final_cut_score",
    "ising_pt_create", "ising_pt_run", "ising_pt_state", "ising_pt_destroy", "ising_standardize_groups",
    "ising_cut_labels", "ising_compare_chains",
]
N_FEATURES, MLP_HIDDEN, MLP_PARAMS = 16, 64, 5313
TRACK_WORDS = 4  # ising_track = 32 bytes: held as int64 [R][4]


class IsingError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("ising error %d: %s" % (code, message))
        self.code = code


class RunParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("layout", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("n_replicas", ctypes.c_int32),
        ("n_sweeps", ctypes.c_int32),
        ("sweep_begin", ctypes.c_int32),
        ("sweep_end", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("init_spins", ctypes.c_int32),
        ("beta0", ctypes.c_double),
        ("beta1", ctypes.c_double),
        ("beta_table", ctypes.c_void_p),
        ("block_threads", ctypes.c_int32),
        ("replica_offset", ctypes.c_int32),
        ("stats_out", ctypes.c_void_p),
        ("replica_thresholds", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libising.so is not built (run paper_2505_18508_amd/build.py): %s" % LIB_PATH)
        # torch ships its own HIP runtime under the same soname as the system
        # one this library links against; whichever is loaded first serves the
        # whole process, and torch works only with its own.  Loading torch
        # first makes torch's streams, its allocations and this library's
        # launches share that one runtime.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.ising_create_graph.argtypes = [i32, vp, u64, vp, ctypes.POINTER(vp)]
        L.ising_destroy_graph.argtypes = [vp]
        L.ising_destroy_graph.restype = None
        L.ising_graph_info.argtypes = [vp, vp, vp, vp, vp]
        L.ising_graph_weights.argtypes = [vp, vp]
        L.ising_generate_weights.argtypes = [i32, vp, u64, vp]
        L.ising_run_trials.argtypes = [vp, ctypes.POINTER(RunParams), vp, vp, vp, vp, vp]
        L.ising_run_trials_noalloc.argtypes = [vp, ctypes.POINTER(RunParams), vp, vp, vp, vp, vp]
        L.ising_eval_cut.argtypes = [vp, vp, i64, vp, vp, vp]
        L.ising_thresholds.argtypes = [ctypes.POINTER(RunParams), i32, vp]
        L.ising_philox_dump.argtypes = [u64, vp, i64, vp, vp]
        u32 = ctypes.c_uint32
        L.ising_compare_chains.argtypes = [i64, vp, vp, vp, u32, u32, u32, vp, vp]
        L.ising_last_error.argtypes = []
        L.ising_last_error.restype = ctypes.c_char_p
        f32 = ctypes.c_float
        L.ising_features.argtypes = [vp, vp, vp, vp, i64, vp, i32, i32, i32, ctypes.c_double, i32, vp, vp]
        L.ising_mlp_init.argtypes = [u64, vp, vp]
        L.ising_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, vp]
        L.ising_mlp_workspace_floats.argtypes = [i64]
        L.ising_mlp_loss_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp]
        L.ising_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]
        L.ising_feature_stats.argtypes = [vp, i64, vp, vp, vp]
        L.ising_cull_clone.argtypes = [vp, i64, i64, vp, vp, vp, vp]
        L.ising_energy_score.argtypes = [vp, i64, vp, vp]
        L.ising_cut_labels.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp]
        L.ising_schedule_beta.argtypes = [ctypes.POINTER(RunParams), i32, ctypes.POINTER(ctypes.c_double)]
        L.ising_batch_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.ising_batch_run.argtypes = [vp, vp]
        L.ising_batch_info.argtypes = [vp, vp, vp, vp, vp]
        L.ising_batch_destroy.argtypes = [vp]
        L.ising_batch_destroy.restype = None
        L.ising_final_cut_score.argtypes = [vp, vp, vp, i64, vp, vp]
        L.ising_pt_create.argtypes = [vp, i32, vp, i32, u64, ctypes.POINTER(vp)]
        L.ising_pt_run.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp]
        L.ising_pt_state.argtypes = [vp, vp, vp, vp]
        L.ising_standardize_groups.argtypes = [vp, i64, i64, i32, vp]
        L.ising_pt_destroy.argtypes = [vp]
        L.ising_pt_destroy.restype = None
        for name in EXPORTED:
            if name not in ("ising_destroy_graph", "ising_last_error", "ising_mlp_workspace_floats",
                            "ising_batch_destroy", "ising_pt_destroy"):
                getattr(L, name).restype = ctypes.c_int
        L.ising_mlp_workspace_floats.restype = i64
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise IsingError(rc, lib().ising_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _want(t, name, dtypes, numel=None):
    """Check that t (or None) has one of dtypes (torch dtype names) and at
    least numel elements: the kernels index these buffers by the sizes the
    call states, so a short or mistyped buffer is refused here."""
    if t is None:
        return
    import torch

    if t.dtype not in tuple(getattr(torch, d) for d in dtypes):
        raise ValueError("%s must be %s, got %s" % (name, " or ".join(dtypes), str(t.dtype).replace("torch.", "")))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))


def _dev(t, name, dtypes, numel=None):
    """_ptr after _want's checks."""
    _want(t, name, dtypes, numel)
    return _ptr(t)


def _devs(*specs):
    """Device pointers of several (tensor, name, dtypes, numel) buffers, every
    one checked before any is converted."""
    for spec in specs:
        _want(*spec)
    return [_ptr(spec[0]) for spec in specs]


I32 = ("int32", "uint32")


def _stream(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _dims_arr(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    return d, d.ctypes.data


class Graph:
    """A torus instance (handle of ising_create_graph) on the current device."""

    def __init__(self, dims, weight_seed=0, weights=None):
        d, dp = _dims_arr(dims)
        self.dims = [int(x) for x in d]
        h = ctypes.c_void_p()
        wp = None
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.int8)
            wp = w.ctypes.data
        _check(lib().ising_create_graph(len(d), dp, int(weight_seed), wp, ctypes.byref(h)))
        self._h = h
        n, ne, wt, deg = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().ising_graph_info(h, ctypes.byref(n), ctypes.byref(ne), ctypes.byref(wt), ctypes.byref(deg)))
        self.n, self.n_edges, self.w_total, self.degree = n.value, ne.value, wt.value, deg.value

    @property
    def handle(self):
        return self._h

    def weights(self):
        out = np.zeros(self.n_edges, np.int8)
        _check(lib().ising_graph_weights(self._h, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ising_destroy_graph(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_graph(dims, weight_seed=0, weights=None):
    return Graph(dims, weight_seed, weights)


def generate_weights(dims, weight_seed):
    d, dp = _dims_arr(dims)
    out = np.zeros(len(d) * int(np.prod(d)), np.int8)
    _check(lib().ising_generate_weights(len(d), dp, int(weight_seed), out.ctypes.data))
    return out


def make_params(seed, n_replicas, n_sweeps, sweep_begin=0, sweep_end=None, schedule="linear", beta0=0.1,
                beta1=3.0, beta_table=None, init_spins=True, layout="auto", block_threads=0, replica_offset=0,
                stats=None, replica_thresholds=None):
    """RunParams plus the objects whose memory it points to (keep both alive)."""
    p = RunParams()
    p.struct_size = ctypes.sizeof(RunParams)
    p.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    p.seed = int(seed)
    p.n_replicas = int(n_replicas)
    p.n_sweeps = int(n_sweeps)
    p.sweep_begin = int(sweep_begin)
    p.sweep_end = int(n_sweeps if sweep_end is None else sweep_end)
    p.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    p.init_spins = 1 if init_spins else 0
    p.beta0 = float(beta0)
    p.beta1 = float(beta1)
    keep = None
    if beta_table is not None:
        keep = np.ascontiguousarray(beta_table, dtype=np.float64)
        p.beta_table = keep.ctypes.data
    p.block_threads = int(block_threads)
    p.replica_offset = int(replica_offset)
    p.stats_out = None if stats is None else _dev(stats, "stats", ("int64",), 2).value
    p.replica_thresholds = None if replica_thresholds is None else _dev(
        replica_thresholds, "replica_thresholds", I32).value
    return p, keep


def select_layout(graph, n_replicas, n_sweeps=1, layout="auto", block_threads=0):
    """Name of the packing ising_run_trials would use for R replicas (AUTO resolved)."""
    p, _ = make_params(0, n_replicas, n_sweeps, layout=layout, block_threads=block_threads)
    out = ctypes.c_int32(0)
    _check(lib().ising_select_layout(graph.handle, ctypes.byref(p), ctypes.byref(out)))
    return {v: k for k, v in LAYOUTS.items()}[out.value]


def run_trials(graph, spins, seed, n_sweeps, sweep_begin=0, sweep_end=None, schedule="linear", beta0=0.1,
               beta1=3.0, beta_table=None, init_spins=True, layout="auto", cut=None, energy=None, flips=None,
               block_threads=0, replica_offset=0, stats=None, stream=None, replica_thresholds=None):
    """ising_run_trials on device tensors: spins int8 [R][n] (in/out); cut,
    energy int64 [R], flips uint32/int32 [R], stats int64 [2] optional;
    replica_thresholds uint32/int32 [R][degree/2] (each replica at its own
    fixed temperature) optional.  Asynchronous."""
    _run(lib().ising_run_trials, graph, spins, seed, n_sweeps, sweep_begin, sweep_end, schedule, beta0, beta1,
         beta_table, init_spins, layout, cut, energy, flips, block_threads, replica_offset, stats, stream,
         replica_thresholds)


def run_trials_noalloc(graph, spins, seed, n_sweeps, sweep_begin=0, sweep_end=None, schedule="linear", beta0=0.1,
                       beta1=3.0, beta_table=None, init_spins=True, layout="auto", cut=None, energy=None, flips=None,
                       block_threads=0, replica_offset=0, stats=None, stream=None, replica_thresholds=None):
    """ising_run_trials_noalloc: run_trials without any allocation (the
    library's fixed per-GPU scratch; calls overlapping on one GPU race)."""
    _run(lib().ising_run_trials_noalloc, graph, spins, seed, n_sweeps, sweep_begin, sweep_end, schedule, beta0,
         beta1, beta_table, init_spins, layout, cut, energy, flips, block_threads, replica_offset, stats, stream,
         replica_thresholds)


def _run(fn, graph, spins, seed, n_sweeps, sweep_begin, sweep_end, schedule, beta0, beta1, beta_table, init_spins,
         layout, cut, energy, flips, block_threads, replica_offset, stats, stream, replica_thresholds):
    R = spins.shape[0]
    if spins.dim() != 2 or spins.shape[1] != graph.n:
        raise ValueError("spins must be [R][%d]" % graph.n)
    if replica_thresholds is not None and tuple(replica_thresholds.shape) != (R, graph.degree // 2):
        raise ValueError("replica_thresholds must be [R][%d]" % (graph.degree // 2))
    p, keep = make_params(seed, R, n_sweeps, sweep_begin, sweep_end, schedule, beta0, beta1, beta_table,
                          init_spins, layout, block_threads, replica_offset, stats, replica_thresholds)
    _check(fn(graph.handle, ctypes.byref(p), _dev(spins, "spins", ("int8",)), _dev(cut, "cut", ("int64",), R),
              _dev(energy, "energy", ("int64",), R), _dev(flips, "flips", I32, R), _stream(stream)))
    del keep


def eval_cut(graph, spins, cut=None, energy=None, stream=None):
    if spins.dim() != 2 or spins.shape[1] != graph.n:
        raise ValueError("spins must be [R][%d]" % graph.n)
    R = spins.shape[0]
    _check(lib().ising_eval_cut(graph.handle, _dev(spins, "spins", ("int8",)), R, _dev(cut, "cut", ("int64",), R),
                                _dev(energy, "energy", ("int64",), R), _stream(stream)))


def thresholds(n_sweeps, schedule="linear", beta0=0.1, beta1=3.0, beta_table=None, degree=4):
    """Acceptance thresholds T_k(t) of a whole schedule: uint32 [S][degree/2]."""
    p, keep = make_params(0, 1, n_sweeps, 0, None, schedule, beta0, beta1, beta_table)
    out = np.zeros((n_sweeps, degree // 2), np.uint32)
    _check(lib().ising_thresholds(ctypes.byref(p), int(degree), out.ctypes.data))
    del keep
    return out


def schedule_beta(n_sweeps, t, schedule="linear", beta0=0.1, beta1=3.0, beta_table=None):
    """beta_t of sweep t of an n_sweeps schedule (the library's own schedule)."""
    p, keep = make_params(0, 1, n_sweeps, 0, None, schedule, beta0, beta1, beta_table)
    out = ctypes.c_double()
    _check(lib().ising_schedule_beta(ctypes.byref(p), int(t), ctypes.byref(out)))
    del keep
    return out.value


def philox_dump(key, ctr, out, stream=None):
    """Philox4x32-10 blocks on the GPU: ctr, out uint32/int32 device [m][4]."""
    m = ctr.shape[0]
    if ctr.dim() != 2 or ctr.shape[1] != 4:
        raise ValueError("ctr must be [m][4]")
    _check(lib().ising_philox_dump(int(key), _dev(ctr, "ctr", I32), m, _dev(out, "out", I32, 4 * m),
                                   _stream(stream)))


def compare_chains(u, sel2, sel3, T1, T2, T3, out, stream=None):
    """ising_compare_chains: the kernels' threshold compare chains on u
    uint32/int32 device [n][32] with level bits sel2, sel3 [n]; out [n][8]."""
    n = u.shape[0]
    if u.dim() != 2 or u.shape[1] != 32:
        raise ValueError("u must be [n][32]")
    _check(lib().ising_compare_chains(n, *_devs((u, "u", I32, 32 * n), (sel2, "sel2", I32, n),
                                               (sel3, "sel3", I32, n)),
                                      int(T1) & 0xFFFFFFFF, int(T2) & 0xFFFFFFFF, int(T3) & 0xFFFFFFFF,
                                      _dev(out, "out", I32, 8 * n), _stream(stream)))


# ---------------------------------------------------------------------------
# Learned culling
# ---------------------------------------------------------------------------
def new_track(n_replicas, device=None):
    """Zeroed per-replica trajectory records (ising_track [R])."""
    import torch

    return torch.zeros((n_replicas, TRACK_WORDS), dtype=torch.int64, device=device or "cuda")


def features(graph, spins, energy, window_flips, track, sweeps_done, window, n_sweeps, beta, n_checkpoints, out,
             stream=None):
    """ising_features: out float32 [R][16]; track updated in place."""
    R = spins.shape[0]
    if spins.dim() != 2 or spins.shape[1] != graph.n:
        raise ValueError("spins must be [R][%d]" % graph.n)
    _check(lib().ising_features(graph.handle, _dev(spins, "spins", ("int8",)), _dev(energy, "energy", ("int64",), R),
                                _dev(window_flips, "window_flips", I32, R),
                                R, _dev(track, "track", ("int64",), R * TRACK_WORDS), int(sweeps_done), int(window),
                                int(n_sweeps), float(beta), int(n_checkpoints),
                                _dev(out, "features", ("float32",), R * N_FEATURES), _stream(stream)))


F32 = ("float32",)


def _rows16(x, name="x"):
    """Rows of a float32 [rows][16] feature table."""
    if x.dim() != 2 or x.shape[1] != N_FEATURES:
        raise ValueError("%s must be [rows][%d]" % (name, N_FEATURES))
    return x.shape[0]


def _batch(x, idx, batch, mean, std):
    """Rows of x and samples B of a forward/backward call.  idx is int32
    [>= B]; without idx the batch must lie within x.  Index values outside
    x are the kernels' concern (they read nothing and give NaN)."""
    rows = _rows16(x)
    B = (idx.shape[0] if idx is not None else rows) if batch is None else int(batch)
    if B < 0:
        raise ValueError("batch must be >= 0")
    if idx is None and B > rows:
        raise ValueError("batch %d exceeds the %d rows of x" % (B, rows))
    if (mean is None) != (std is None):
        raise ValueError("mean and std must both be given or both be None")
    return rows, B


def mlp_init(seed, params, stream=None):
    """Kaiming-uniform parameters from Philox: params float32 [5313]."""
    (pp,) = _devs((params, "params", F32, MLP_PARAMS))
    _check(lib().ising_mlp_init(int(seed), pp, _stream(stream)))


def mlp_forward(params, x, y, idx=None, mean=None, std=None, batch=None, stream=None):
    """y[b] = network(x[idx[b]]) (or x[b]): x float32 [rows][16], y float32 [B]."""
    rows, B = _batch(x, idx, batch, mean, std)
    pp, xp, ip, mp, sp, yp = _devs((params, "params", F32, MLP_PARAMS), (x, "x", F32), (idx, "idx", ("int32",), B),
                                   (mean, "mean", F32, N_FEATURES), (std, "std", F32, N_FEATURES), (y, "y", F32, B))
    _check(lib().ising_mlp_forward(pp, xp, rows, ip, mp, sp, B, yp, _stream(stream)))


def mlp_workspace_floats(batch):
    return int(lib().ising_mlp_workspace_floats(int(batch)))


def mlp_loss_grad(params, x, target, grad, workspace, loss=None, idx=None, mean=None, std=None, batch=None,
                  stream=None):
    """Mean squared error of the batch and its gradient: target float32
    [rows] (read at idx) or [B]; grad float32 [5313]; loss float32 [1] or
    None; workspace float32 [mlp_workspace_floats(B)]."""
    rows, B = _batch(x, idx, batch, mean, std)
    pp, xp, ip, mp, sp, tp, gp, lp, wp = _devs(
        (params, "params", F32, MLP_PARAMS), (x, "x", F32), (idx, "idx", ("int32",), B),
        (mean, "mean", F32, N_FEATURES), (std, "std", F32, N_FEATURES),
        (target, "target", F32, rows if idx is not None else B), (grad, "grad", F32, MLP_PARAMS),
        (loss, "loss", F32, 1), (workspace, "workspace", F32, mlp_workspace_floats(B)))
    _check(lib().ising_mlp_loss_grad(pp, xp, rows, ip, mp, sp, tp, B, gp, lp, wp, _stream(stream)))


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step on every element of params (float32); grad, m, v alike."""
    n = params.numel()
    pp, gp, mp, vp = _devs((params, "params", F32), (grad, "grad", F32, n), (m, "m", F32, n), (v, "v", F32, n))
    _check(lib().ising_adam_step(pp, gp, mp, vp, n, int(step), float(lr), float(beta1), float(beta2), float(eps),
                                 _stream(stream)))


def feature_stats(x, mean, std, rows=None, stream=None):
    """Column means and deviations of x float32 [rows][16] into mean, std float32 [16]."""
    n = _rows16(x) if rows is None else int(rows)
    if n > x.shape[0]:
        raise ValueError("rows %d exceeds the %d rows of x" % (n, x.shape[0]))
    xp, mp, sp = _devs((x, "x", F32), (mean, "mean", F32, N_FEATURES), (std, "std", F32, N_FEATURES))
    _check(lib().ising_feature_stats(xp, n, mp, sp, _stream(stream)))


def cull_clone(score, spins, track=None, order=None, stream=None):
    R, n = spins.shape
    _check(lib().ising_cull_clone(_dev(score, "score", ("float32",), R), R, n, _dev(spins, "spins", ("int8",)),
                                  _dev(track, "track", ("int64",), R * TRACK_WORDS), _dev(order, "order", I32, R),
                                  _stream(stream)))


def final_cut_score(graph, gain, feats, score, stream=None):
    """score = predicted final cut / |E| from the network's gain prediction."""
    R = gain.shape[0]
    _check(lib().ising_final_cut_score(graph.handle, _dev(gain, "gain", ("float32",)),
                                       _dev(feats, "features", ("float32",), R * N_FEATURES), R,
                                       _dev(score, "score", ("float32",), R), _stream(stream)))


def standardize_groups(x, n_groups, rows, cols, stream=None):
    """In place: every column of every group of rows of a float32 [n_groups][rows][cols]
    table to zero mean and unit (population) deviation within the group."""
    _check(lib().ising_standardize_groups(_dev(x, "x", ("float32",), int(n_groups) * int(rows) * int(cols)),
                                          int(n_groups), int(rows), int(cols), _stream(stream)))


def cut_labels(final_cut, out, now_cut=None, scale=1.0, stream=None):
    """out = (final_cut - now_cut) * scale (now_cut None: 0): int64 [R] -> float32 [R]."""
    R = final_cut.shape[0]
    fp, np_, op = _devs((final_cut, "final_cut", ("int64",), R), (now_cut, "now_cut", ("int64",), R),
                        (out, "out", F32, R))
    _check(lib().ising_cut_labels(fp, np_, R, float(scale), op, _stream(stream)))


def energy_score(energy, score, stream=None):
    R = energy.shape[0]
    _check(lib().ising_energy_score(_dev(energy, "energy", ("int64",)), R, _dev(score, "score", ("float32",), R),
                                    _stream(stream)))


# ---------------------------------------------------------------------------
# Batches of uneven instances
# ---------------------------------------------------------------------------
class Batch:
    """A prepared persistent launch over several (graph, run) pairs.  Each run
    is a dict of run_trials keyword arguments (replica_thresholds included)
    plus `spins` (device int8 [R][n]) and optional `cut`, `energy`, `flips`
    device tensors."""

    def __init__(self, graphs, runs):
        k = len(graphs)
        if k != len(runs) or k == 0:
            raise ValueError("need one run per graph")
        self._keep = []
        params = (RunParams * k)()
        ptrs = {name: (ctypes.c_void_p * k)() for name in ("spins", "cut", "energy", "flips")}
        gh = (ctypes.c_void_p * k)(*[g.handle.value for g in graphs])
        for i, (g, run) in enumerate(zip(graphs, runs)):
            spins = run["spins"]
            if spins.dim() != 2 or spins.shape[1] != g.n:
                raise ValueError("spins of instance %d must be [R][%d]" % (i, g.n))
            rt = run.get("replica_thresholds")
            if rt is not None and tuple(rt.shape) != (spins.shape[0], g.degree // 2):
                raise ValueError("replica_thresholds of instance %d must be [R][%d]" % (i, g.degree // 2))
            p, keep = make_params(run["seed"], spins.shape[0], run["n_sweeps"], run.get("sweep_begin", 0),
                                  run.get("sweep_end"), run.get("schedule", "geometric"), run.get("beta0", 0.05),
                                  run.get("beta1", 4.0), run.get("beta_table"), run.get("init_spins", True),
                                  run.get("layout", "auto"), run.get("block_threads", 0), run.get("replica_offset", 0),
                                  replica_thresholds=rt)
            params[i] = p
            self._keep.append(keep)
            R = spins.shape[0]
            kinds = {"spins": (("int8",), None), "cut": (("int64",), R), "energy": (("int64",), R), "flips": (I32, R)}
            for name in ptrs:
                t = run.get(name)
                ptrs[name][i] = None if t is None else _dev(t, name, *kinds[name]).value
        h = ctypes.c_void_p()
        _check(lib().ising_batch_create(k, gh, params, ptrs["spins"], ptrs["cut"], ptrs["energy"], ptrs["flips"],
                                        ctypes.byref(h)))
        self._h = h
        self.graphs, self.runs = graphs, runs
        n, a, gr, bl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ising_batch_info(h, ctypes.byref(n), ctypes.byref(a), ctypes.byref(gr), ctypes.byref(bl)))
        self.n_items, self.attempts, self.grid, self.block = n.value, a.value, gr.value, bl.value

    def run(self, stream=None):
        _check(lib().ising_batch_run(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ising_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PT:
    """Replica exchange (ising_pt_*): L ladders of K inverse temperatures on
    one graph, L K replica slots.  run() advances rounds of sweeps plus one
    exchange pass each; labels() gives every slot's temperature index."""

    def __init__(self, graph, betas, n_ladders, seed):
        b = np.ascontiguousarray(betas, np.float64)
        h = ctypes.c_void_p()
        _check(lib().ising_pt_create(graph.handle, len(b), b.ctypes.data, int(n_ladders), int(seed), ctypes.byref(h)))
        self._h = h
        self.graph, self.betas, self.n_ladders = graph, b, int(n_ladders)
        self.n_replicas = len(b) * self.n_ladders

    def run(self, spins, n_rounds, sweeps_per_round, round_begin=0, init_spins=False, cut=None, energy=None,
            stream=None):
        if spins.dim() != 2 or spins.shape != (self.n_replicas, self.graph.n):
            raise ValueError("spins must be [%d][%d]" % (self.n_replicas, self.graph.n))
        R = self.n_replicas
        _check(lib().ising_pt_run(self._h, _dev(spins, "spins", ("int8",)), 1 if init_spins else 0, int(round_begin),
                                  int(n_rounds), int(sweeps_per_round), _dev(cut, "cut", ("int64",), R),
                                  _dev(energy, "energy", ("int64",), R), _stream(stream)))

    def labels(self, out=None, stream=None):
        """Temperature index of every slot (device int32 [L K])."""
        import torch

        if out is None:
            out = torch.zeros(self.n_replicas, dtype=torch.int32, device="cuda")
        _check(lib().ising_pt_state(self._h, _dev(out, "out", I32, self.n_replicas), None, _stream(stream)))
        return out

    def accepted(self):
        """Exchanges accepted per adjacent pair since creation (host uint64 [K-1]); synchronises."""
        acc = np.zeros(len(self.betas) - 1, np.uint64)
        _check(lib().ising_pt_state(self._h, None, acc.ctypes.data, None))
        return acc

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ising_pt_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

