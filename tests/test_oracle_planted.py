"""Planted mistakes in the oracle, caught by its pins.

Each case copies one oracle source, plants one plausible mistake in the copy
(a dropped or doubled term, a wrong sign, a wrong index or axis, a transposed
operand, a wrong constant), loads the copy in place of the oracle, and checks
that at least one of the named pins fails on it.  The control cases run every
pin named here on unmodified copies loaded the same way, so each failure comes
from the planted mistake alone.  Everything here runs on the CPU.
"""
import os
import subprocess
import types

import pytest

import oracle
from tests import test_oracle_learn as learn_pins
from tests import test_oracle_pins as pins
from tests import test_oracle_pt as pt_pins
from tests.test_oracle_pins import torch_philox  # noqa: F401  (fixture)

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))

# (case, planted text replaced, replacement, pins as (module, test, args))
C_CASES = [
    ("philox_multiplier", "mult_a = 0xD2511F53u", "mult_a = 0xD2511F57u",
     [(pins, "test_philox_matches_torch_engine", "philox")]),
    ("philox_xor_operand", "^ x1 ^ k0", "^ x3 ^ k0",
     [(pins, "test_philox_matches_torch_engine", "philox")]),
    ("philox_key_schedule", "k1 += weyl_b;", "k1 += weyl_a;",
     [(pins, "test_philox_matches_torch_engine", "philox")]),
    ("torus_axis_length", "nb[axis] = (c[axis] + 1) % dims[axis];", "nb[axis] = (c[axis] + 1) % dims[d];",
     [(pins, "test_torus_edges_follow_coordinates", ([4, 6],)),
      (pins, "test_torus_edges_follow_coordinates", ([4, 2, 6],))]),
    ("colour_parity_bit", "return (int)(s & 1);", "return (int)((s >> 1) & 1);",
     [(pins, "test_checkerboard_colouring_is_proper", ([4, 6],))]),
    ("cut_counts_uncut_edges", "if (sa != sb) c += w[e];", "if (sa == sb) c += w[e];",
     [(pins, "test_cut_matches_eq1_and_energy_identity", ([4, 6],))]),
    ("energy_counts_edges_twice", "h += (int64_t)w[e] * sa * sb;", "h += 2 * (int64_t)w[e] * sa * sb;",
     [(pins, "test_cut_matches_eq1_and_energy_identity", ([4, 6],)),
      (pins, "test_paper_pairs_fix_single_count_energy", ())]),
    ("energy_sign", "h += (int64_t)w[e] * sa * sb;", "h -= (int64_t)w[e] * sa * sb;",
     [(pins, "test_cut_matches_eq1_and_energy_identity", ([4, 6],))]),
    ("threshold_energy_step", "exp(-(double)(4 * k) * beta)", "exp(-(double)(2 * k) * beta)",
     [(pins, "test_thresholds_closed_form", ()),
      (pins, "test_fixed_beta_samples_boltzmann", ([2, 4], 0.35, 4))]),
    ("threshold_sign", "exp(-(double)(4 * k) * beta)", "exp((double)(4 * k) * beta)",
     [(pins, "test_thresholds_closed_form", ())]),
    ("delta_energy_sign", "int dE = -2 * s[i] * f[i];", "int dE = 2 * s[i] * f[i];",
     [(pins, "test_annealer_reaches_bruteforce_max", ([2, 4],)),
      (pins, "test_fixed_beta_samples_boltzmann", ([2, 4], 0.35, 4))]),
    ("threshold_index", "accept = u < thr[dE / 4];", "accept = u < thr[1];",
     [(pins, "test_fixed_beta_samples_boltzmann", ([2, 4], 0.35, 4)),
      (pins, "test_fixed_beta_samples_boltzmann", ([2, 2, 2], 0.25, 6))]),
    ("field_update_sign", "-= 2 * adj.wt[i * deg + k] * old;", "+= 2 * adj.wt[i * deg + k] * old;",
     [(pins, "test_maintained_fields_equal_recomputed", ([8, 6],))]),
    ("field_update_factor", "-= 2 * adj.wt[i * deg + k] * old;", "-= adj.wt[i * deg + k] * old;",
     [(pins, "test_maintained_fields_equal_recomputed", ([8, 6],))]),
    ("field_update_target", "f[adj.nb[i * deg + k]] -= 2", "f[i] -= 2",
     [(pins, "test_maintained_fields_equal_recomputed", ([8, 6],))]),
    ("initial_field_operand", "acc += adj.wt[i * deg + k] * s[adj.nb[i * deg + k]];",
     "acc += adj.wt[i * deg + k] * s[i];",
     [(pins, "test_maintained_fields_equal_recomputed", ([8, 6],))]),
    ("half_sweep_ignores_colour", "if (colour[i] != c) continue;", "if (colour[i] == 2) continue;",
     [(pins, "test_flip_count_matches_changed_spins_at_infinite_temperature", ())]),
    ("schedule_endpoint", "(double)t / (double)(n_sweeps - 1)", "(double)t / (double)n_sweeps",
     [(pins, "test_schedules", ())]),
    ("geometric_schedule_reversed", "beta0 * pow(beta1 / beta0, frac)", "beta0 * pow(beta1 / beta0, 1.0 - frac)",
     [(pins, "test_schedules", ())]),
    ("bruteforce_skips_states", "state < ((uint64_t)1 << n)", "state < ((uint64_t)1 << (n - 2))",
     [(pins, "test_bruteforce_closed_forms", ([2, 2],)),
      (pins, "test_bruteforce_2x2_is_doubled_four_cycle", ())]),
    ("replica_thresholds_of_replica_0", "thr[k] = rep_thr[(int64_t)rr * (deg / 2) + k - 1];", "thr[k] = rep_thr[k - 1];",
     [(pt_pins, "test_ladders_sample_product_of_boltzmann", ([2, 4], (0.4, 1.0)))]),
    ("bruteforce_counts_uncut_edges", "if (xa != xb) c += w[e];", "if (xa == xb) c += w[e];",
     [(pins, "test_bruteforce_closed_forms", ([2, 2],)),
      (pins, "test_bruteforce_2x2_is_doubled_four_cycle", ())]),
]

PY_CASES = [
    ("learn", "backprop_transposed_weight", 'd1 = (d2 @ p["W2"]) * (a1 > 0)', 'd1 = (d2 @ p["W2"].T) * (a1 > 0)',
     [(learn_pins, "test_gradient_matches_central_differences", ())]),
    ("learn", "backprop_wrong_mask", 'd2 = np.outer(dy, p["W3"]) * (a2 > 0)', 'd2 = np.outer(dy, p["W3"]) * (a1 > 0)',
     [(learn_pins, "test_gradient_matches_central_differences", ())]),
    ("learn", "loss_gradient_factor", "dy = 2.0 * err / B", "dy = err / B",
     [(learn_pins, "test_gradient_matches_central_differences", ())]),
    ("learn", "bias_gradient_operand", 'g["b1"] = d1.sum(axis=0)', 'g["b1"] = d2.sum(axis=0)',
     [(learn_pins, "test_gradient_matches_central_differences", ())]),
    ("learn", "forward_drops_relu", "h1 = np.maximum(a1, 0.0)", "h1 = a1",
     [(learn_pins, "test_forward_closed_form", ()),
      (learn_pins, "test_gradient_matches_central_differences", ())]),
    ("learn", "adam_no_bias_correction", "m_hat = m / (1.0 - beta1**step)", "m_hat = m",
     [(learn_pins, "test_adam_constant_gradient_moves_lr_per_step", ())]),
    ("learn", "adam_ascends", "theta - lr * m_hat", "theta + lr * m_hat",
     [(learn_pins, "test_adam_constant_gradient_moves_lr_per_step", ())]),
    ("learn", "standardize_wrong_axis", "sd = np.sqrt(((a - mu) ** 2).mean(axis=1, keepdims=True))",
     "sd = np.sqrt(((a - mu) ** 2).mean(axis=2, keepdims=True))",
     [(learn_pins, "test_standardize_groups_closed_form_and_invariants", ())]),
    ("learn", "histogram_reversed", "for v in (-6, -4, -2, 0, 2, 4, 6)", "for v in (6, 4, 2, 0, -2, -4, -6)",
     [(learn_pins, "test_features_identities", ([6, 8],)),
      (learn_pins, "test_features_bipartite_closed_form", ())]),
    ("learn", "energy_change_sign", "(H - h_prev) / E", "(h_prev - H) / E",
     [(learn_pins, "test_features_identities", ([6, 8],))]),
    ("learn", "init_fan_in_of_rows", 'fan_in = shape[-1] if name != "W3" else NH', 'fan_in = shape[0] if name != "W3" else NH',
     [(learn_pins, "test_init_bound_of_each_layer_follows_its_own_fan_in", (5,))]),
    ("learn", "init_last_layer_fan_in", 'fan_in = shape[-1] if name != "W3" else NH', 'fan_in = shape[-1] if name != "W3" else NF',
     [(learn_pins, "test_init_bound_of_each_layer_follows_its_own_fan_in", (5,))]),
    ("learn", "final_score_energy_sign", "0.5 * (w_total / n_edges - np.asarray", "0.5 * (w_total / n_edges + np.asarray",
     [(learn_pins, "test_final_cut_score_is_eq1_cut_plus_gain", ([6, 8],))]),
    ("learn", "final_score_drops_half", "return 0.5 * (w_total / n_edges", "return 1.0 * (w_total / n_edges",
     [(learn_pins, "test_final_cut_score_is_eq1_cut_plus_gain", ([6, 8],))]),
    ("learn", "final_score_gain_sign", "[:, 0]) + np.asarray(gain", "[:, 0]) - np.asarray(gain",
     [(learn_pins, "test_final_cut_score_is_eq1_cut_plus_gain", ([6, 8],))]),
    ("learn", "cull_ranks_worst_first", "(0, -s)", "(0, s)",
     [(learn_pins, "test_cull_order_and_clone", ())]),
    ("learn", "clone_direction", "spins[dst] = spins[src]", "spins[src] = spins[dst]",
     [(learn_pins, "test_cull_order_and_clone", ())]),
    ("pt", "exchange_direction", "if d <= 0 or", "if d >= 0 or",
     [(pt_pins, "test_decisions_follow_energies_and_labels_stay_permutations", ())]),
    ("pt", "exchange_threshold_sign", "math.exp(-x)", "math.exp(x)",
     [(pt_pins, "test_exchange_acceptance_frequency_is_boltzmann_ratio", ())]),
    ("pt", "exchange_drops_factor", "x = (beta_hi - beta_lo) * (4.0 * m)", "x = (beta_hi - beta_lo) * m",
     [(pt_pins, "test_exchange_acceptance_frequency_is_boltzmann_ratio", ())]),
    ("pt", "labels_not_swapped", "kidx[a], kidx[b] = k + 1, k", "kidx[a], kidx[b] = k, k + 1",
     [(pt_pins, "test_decisions_follow_energies_and_labels_stay_permutations", ())]),
    ("pt", "pairs_ignore_round_parity", "for k in range(q % 2, K - 1, 2)", "for k in range(0, K - 1, 2)",
     [(pt_pins, "test_decisions_follow_energies_and_labels_stay_permutations", ()),
      (pt_pins, "test_equal_temperatures_always_swap_and_leave_sweeps_unchanged", ())]),
]


def _planted_c(tmp_path, name, old, new):
    src = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    assert src.count(old) == 1, old
    path = tmp_path / ("oracle_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = str(tmp_path / ("liboracle_%s.so" % name))
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I", ORACLE_DIR, "-o", so, str(path), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return so


def _planted_py(module, old, new):
    path = os.path.join(ORACLE_DIR, module + ".py")
    src = open(path).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("oracle." + module)
    mod.__package__ = "oracle"
    mod.__file__ = path
    exec(compile(src.replace(old, new, 1), path, "exec"), mod.__dict__)
    return mod


def _failing(request, pin_list):
    """The pins of `pin_list` that fail (raise AssertionError)."""
    failed = []
    for module, test, args in pin_list:
        if args == "philox":
            args = (request.getfixturevalue("torch_philox"),)
        try:
            getattr(module, test)(*args)
        except AssertionError:
            failed.append(test)
    return failed


def _use_c_library(monkeypatch, so):
    monkeypatch.setattr(oracle._build, "build", lambda force=False: so)
    monkeypatch.setattr(oracle, "_lib", None)


@pytest.mark.parametrize("name,old,new,pin_list", C_CASES, ids=[c[0] for c in C_CASES])
def test_c_oracle_pins_catch_planted_mistake(request, monkeypatch, tmp_path, name, old, new, pin_list):
    _use_c_library(monkeypatch, _planted_c(tmp_path, name, old, new))
    assert _failing(request, pin_list), "no pin caught " + name


def test_c_oracle_control_copy_passes_every_pin(request, monkeypatch, tmp_path):
    _use_c_library(monkeypatch, _planted_c(tmp_path, "control", "int dE = -2", "int dE = -2"))
    every = {(t, repr(a)): (m, t, a) for _, _, _, pl in C_CASES for m, t, a in pl}
    assert _failing(request, [every[k] for k in sorted(every)]) == []


@pytest.mark.parametrize("module,name,old,new,pin_list", PY_CASES, ids=[c[1] for c in PY_CASES])
def test_python_oracle_pins_catch_planted_mistake(request, monkeypatch, module, name, old, new, pin_list):
    holder = learn_pins if module == "learn" else pt_pins
    monkeypatch.setattr(holder, module, _planted_py(module, old, new))
    assert _failing(request, pin_list), "no pin caught " + name


@pytest.mark.parametrize("module", ["learn", "pt"])
def test_python_oracle_control_copy_passes_every_pin(request, monkeypatch, module):
    holder = learn_pins if module == "learn" else pt_pins
    monkeypatch.setattr(holder, module, _planted_py(module, "import math", "import math"))
    every = {(t, repr(a)): (m, t, a) for mod, _, _, _, pl in PY_CASES if mod == module for m, t, a in pl}
    assert _failing(request, [every[k] for k in sorted(every)]) == []
