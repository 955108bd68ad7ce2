"""CPU tests of the product's host side: the C ABI loads and exports every
declared symbol, host-only entry points agree with the oracle, argument
errors are reported.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2505_18508_amd as ising

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert "ising_run_trials" in names and "ising_eval_cut" in names and "ising_create_graph" in names
    L = ising.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(ising.EXPORTED)


@pytest.mark.parametrize("sched,b0,b1,S", [("linear", 0.1, 3.0, 1000), ("geometric", 0.05, 4.0, 10000),
                                           ("linear", 0.0, 0.0, 7), ("geometric", 0.3, 0.3, 1),
                                           ("linear", 2.5, 0.2, 333), ("geometric", 4.0, 0.05, 2)])
@pytest.mark.parametrize("degree", [4, 6])
def test_thresholds_match_oracle_bit_for_bit(sched, b0, b1, S, degree):
    lib_t = ising.thresholds(S, sched, b0, b1, degree=degree)
    code = oracle.SCHED_LINEAR if sched == "linear" else oracle.SCHED_GEOMETRIC
    orc_t = oracle.thresholds(code, b0, b1, S, degree)
    assert lib_t.dtype == np.uint32 and (lib_t == orc_t).all()


def test_table_schedule_thresholds_match_oracle():
    rng = np.random.default_rng(3)
    table = rng.uniform(0.0, 5.0, size=500)
    table[:3] = [0.0, 1e-300, 100.0]
    lib_t = ising.thresholds(500, "table", beta_table=table, degree=6)
    orc_t = oracle.thresholds(oracle.SCHED_TABLE, 0, 0, 500, 6, table=table)
    assert (lib_t == orc_t).all()


@pytest.mark.parametrize("dims,seed", [([2, 2], 1), ([50, 100], 1), ([100, 100], 2), ([100, 200], 81),
                                       ([2, 4, 6], 5), ([8, 8, 8], 643), ([6, 10], 2**63 + 11)])
def test_generated_weights_match_oracle(dims, seed):
    w = ising.generate_weights(dims, seed)
    ne = len(dims) * int(np.prod(dims))
    assert (w == oracle.random_weights(seed, ne)).all()


def test_host_argument_errors():
    with pytest.raises(ising.IsingError) as e:
        ising.generate_weights([3, 4], 1)
    assert e.value.code == ising.E_TOPOLOGY
    with pytest.raises(ising.IsingError) as e:
        ising.generate_weights([4, 4, 4, 4], 1)
    assert e.value.code == ising.E_TOPOLOGY
    with pytest.raises(ising.IsingError) as e:
        ising.generate_weights([0, 4], 1)
    assert e.value.code == ising.E_TOPOLOGY
    with pytest.raises(ising.IsingError) as e:
        ising.thresholds(10, "geometric", 0.0, 1.0)
    assert e.value.code == ising.E_ARG
    with pytest.raises(ising.IsingError) as e:
        ising.thresholds(10, "linear", -0.5, 1.0)
    assert e.value.code == ising.E_ARG
    with pytest.raises(ising.IsingError) as e:
        ising.thresholds(3, "table", beta_table=[0.1, float("nan"), 0.3])
    assert e.value.code == ising.E_ARG
    with pytest.raises(ising.IsingError) as e:
        ising.thresholds(0, "linear", 0.1, 1.0)
    assert e.value.code == ising.E_ARG
    p, keep = ising.make_params(1, 1, 10)
    p.struct_size = 8
    rc = ising.lib().ising_thresholds(ctypes.byref(p), 4, ctypes.c_void_p(np.zeros(40, np.uint32).ctypes.data))
    assert rc == ising.E_ARG
    assert b"struct_size" in ising.lib().ising_last_error()
    # graph creation rejects odd tori before touching the device
    h = ctypes.c_void_p()
    d = np.array([5, 4], np.int32)
    assert ising.lib().ising_create_graph(2, d.ctypes.data, 1, None, ctypes.byref(h)) == ising.E_TOPOLOGY
    assert ising.lib().ising_create_graph(2, None, 1, None, ctypes.byref(h)) == ising.E_ARG
    ising.lib().ising_destroy_graph(None)  # NULL-safe
    # sizes beyond a launch's grid are rejected before any device work
    L, big = ising.lib(), 2**31
    fake = ctypes.c_void_p(16)  # never dereferenced: the size check comes first
    assert L.ising_adam_step(fake, fake, fake, fake, big, 1, 1e-3, 0.9, 0.999, 1e-8, None) == ising.E_ARG
    assert L.ising_energy_score(fake, big, fake, None) == ising.E_ARG
    assert L.ising_adam_step(fake, fake, fake, fake, -1, 1, 1e-3, 0.9, 0.999, 1e-8, None) == ising.E_ARG


def test_one_hip_runtime_in_the_process():
    """Loading the library first (before any torch import) still leaves a
    single HIP runtime mapped: torch's, which the library then shares."""
    import subprocess
    import sys

    code = ("import paper_2505_18508_amd as p; p.lib(); "
            "m = open('/proc/self/maps').read(); "
            "print(len(set(l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_binding_refuses_mistyped_or_short_buffers():
    """The binding checks dtype and length of every sized buffer before any
    pointer reaches the library (host tensors: no device is needed)."""
    import torch

    import paper_2505_18508_amd as ising

    with pytest.raises(ValueError, match="must be int64"):
        ising._dev(torch.zeros(4, dtype=torch.int32), "cut", ("int64",), 4)
    with pytest.raises(ValueError, match="holds 3 elements, needs 4"):
        ising._dev(torch.zeros(3, dtype=torch.int64), "cut", ("int64",), 4)
    with pytest.raises(ValueError, match="device tensor"):
        ising._dev(torch.zeros(4, dtype=torch.int64), "cut", ("int64",), 4)
    with pytest.raises(ValueError, match="must be int32 or uint32"):
        ising._dev(torch.zeros(4, dtype=torch.float32), "flips", ising.I32, 4)
    assert ising._dev(None, "cut", ("int64",), 4) is None


def test_learned_part_wrappers_check_every_buffer():
    """mlp_init, mlp_forward, mlp_loss_grad, adam_step and feature_stats
    refuse a short or mistyped buffer (host tensors here: each check fires
    before the device-pointer check, so no GPU is needed)."""
    import torch

    f32 = torch.float32
    P = ising.MLP_PARAMS
    with pytest.raises(ValueError, match="params holds 5312 elements, needs 5313"):
        ising.mlp_init(1, torch.zeros(P - 1, dtype=f32))
    with pytest.raises(ValueError, match="params must be float32"):
        ising.mlp_init(1, torch.zeros(P, dtype=torch.float64))
    p = torch.zeros(P, dtype=f32)
    x = torch.zeros((8, 16), dtype=f32)
    with pytest.raises(ValueError, match=r"x must be \[rows\]\[16\]"):
        ising.mlp_forward(p, torch.zeros((8, 15), dtype=f32), torch.zeros(8, dtype=f32))
    with pytest.raises(ValueError, match="batch 9 exceeds the 8 rows"):
        ising.mlp_forward(p, x, torch.zeros(9, dtype=f32), batch=9)
    with pytest.raises(ValueError, match="idx must be int32"):
        ising.mlp_forward(p, x, torch.zeros(4, dtype=f32), idx=torch.zeros(4, dtype=torch.int64))
    with pytest.raises(ValueError, match="mean and std"):
        ising.mlp_forward(p, x, torch.zeros(8, dtype=f32), mean=torch.zeros(16, dtype=f32))
    with pytest.raises(ValueError, match="std holds 15"):
        ising.mlp_forward(p, x, torch.zeros(8, dtype=f32), mean=torch.zeros(16, dtype=f32),
                          std=torch.zeros(15, dtype=f32))
    with pytest.raises(ValueError, match="params holds"):
        ising.mlp_forward(torch.zeros(100, dtype=f32), x, torch.zeros(8, dtype=f32))
    with pytest.raises(ValueError, match="y holds 7 elements, needs 8"):
        ising.mlp_forward(p, x, torch.zeros(7, dtype=f32))
    ws = torch.zeros(ising.mlp_workspace_floats(8), dtype=f32)
    g = torch.zeros(P, dtype=f32)
    # with idx the target is read at the gathered rows: it must cover x
    with pytest.raises(ValueError, match="target holds 4 elements, needs 8"):
        ising.mlp_loss_grad(p, x, torch.zeros(4, dtype=f32), g, ws, idx=torch.zeros(4, dtype=torch.int32))
    with pytest.raises(ValueError, match="grad holds"):
        ising.mlp_loss_grad(p, x, torch.zeros(8, dtype=f32), torch.zeros(10, dtype=f32), ws)
    with pytest.raises(ValueError, match="workspace holds"):
        ising.mlp_loss_grad(p, x, torch.zeros(8, dtype=f32), g, ws[:10])
    with pytest.raises(ValueError, match="loss must be float32"):
        ising.mlp_loss_grad(p, x, torch.zeros(8, dtype=f32), g, ws, loss=torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError, match="m holds 10 elements"):
        ising.adam_step(p, g, torch.zeros(10, dtype=f32), torch.zeros(P, dtype=f32), 1)
    with pytest.raises(ValueError, match="grad must be float32"):
        ising.adam_step(p, g.double(), torch.zeros(P, dtype=f32), torch.zeros(P, dtype=f32), 1)
    with pytest.raises(ValueError, match="mean holds 3"):
        ising.feature_stats(x, torch.zeros(3, dtype=f32), torch.zeros(16, dtype=f32))
    with pytest.raises(ValueError, match="rows 9 exceeds"):
        ising.feature_stats(x, torch.zeros(16, dtype=f32), torch.zeros(16, dtype=f32), rows=9)
    # every check passed: the last one is the device-pointer check
    with pytest.raises(ValueError, match="device tensor"):
        ising.mlp_forward(p, x, torch.zeros(8, dtype=f32))


def test_mlp_entry_points_reject_a_batch_beyond_x():
    """Without idx the C entry points refuse a batch larger than x_rows
    before any launch (pointers never dereferenced)."""
    L = ising.lib()
    fake = ctypes.c_void_p(16)
    assert L.ising_mlp_forward(fake, fake, 8, None, None, None, 9, fake, None) == ising.E_ARG
    assert b"x_rows" in L.ising_last_error()
    assert L.ising_mlp_loss_grad(fake, fake, 8, None, None, None, fake, 9, fake, None, fake, None) == ising.E_ARG
    assert L.ising_mlp_forward(fake, fake, -1, fake, None, None, 4, fake, None) == ising.E_ARG
