"""Pins of the learned-culling oracle: gradients against central finite
differences, networks whose output is known in closed form, Adam's
constant-gradient behaviour, the initialiser's range and uniformity, feature
identities (the s f histogram against eq. (2)), and the cull ranking."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import learn


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = learn.init_params(11) + 0.05 * rng.standard_normal(learn.N_PARAMS)
    z = rng.standard_normal((7, 16))
    t = rng.standard_normal(7)
    _, g = learn.loss_grad(theta, z, t)
    h = 1e-6
    num = np.zeros_like(theta)
    for i in range(learn.N_PARAMS):
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = learn.loss_grad(theta + e, z, t)
        lm, _ = learn.loss_grad(theta - e, z, t)
        num[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g - num) / np.linalg.norm(num) < 1e-7
    # the loss is the mean squared error of forward()
    loss, _ = learn.loss_grad(theta, z, t)
    assert loss == pytest.approx(np.mean((learn.forward(theta, z) - t) ** 2), rel=1e-12)


def test_forward_closed_form():
    """W1 copies the inputs into hidden units 0..15, W2's first row sums them,
    W3 reads that unit: y = sum_k relu(z_k) + b3."""
    theta = np.zeros(learn.N_PARAMS)
    p = learn.unpack(theta)
    p["W1"][:16, :16] = np.eye(16)
    p["W2"][0, :16] = 1.0
    p["W3"][0] = 1.0
    p["b3"][0] = 0.5
    z = np.random.default_rng(1).standard_normal((50, 16))
    assert np.allclose(learn.forward(theta, z), np.maximum(z, 0).sum(axis=1) + 0.5, rtol=0, atol=1e-12)
    # a negative first-layer bias shifts every ReLU
    p["b1"][:16] = -0.25
    assert np.allclose(learn.forward(theta, z), np.maximum(z - 0.25, 0).sum(axis=1) + 0.5, atol=1e-12)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2, so every step moves lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for step in range(1, 6):
        new, m, v = learn.adam_step(theta, g, m, v, step, lr=0.01)
        assert np.allclose(new - theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
        theta = new


def test_init_range_and_uniformity():
    theta = learn.init_params(5)
    p = learn.unpack(theta)
    for name, fan_in in (("W1", 16), ("W2", 64), ("W3", 64)):
        a = math.sqrt(6.0 / fan_in)
        assert np.abs(p[name]).max() <= a
    for name in ("b1", "b2", "b3"):
        assert (p[name] == 0).all()
    u = (p["W2"].reshape(-1) / math.sqrt(6.0 / 64) + 1) / 2
    assert stats.chisquare(np.histogram(u, bins=16, range=(0, 1))[0]).pvalue > 1e-4
    assert (learn.init_params(5) == theta).all() and (learn.init_params(6) != theta).any()


@pytest.mark.parametrize("seed", [5, 17, 2024])
def test_init_bound_of_each_layer_follows_its_own_fan_in(seed):
    """Kaiming-uniform: every weight of a layer with fan-in F is uniform on
    [-a, a], a = sqrt(6/F) (W1: F = 16, W2 and W3: F = 64).  The largest |w|
    of m such draws falls below a (1 - d) with probability (1 - d)^m, and the
    mean |w| is a/2 with standard error a / sqrt(12 m); so a layer drawn with
    another layer's fan-in misses both bounds by a factor of two."""
    p = learn.unpack(learn.init_params(seed))
    for name, fan_in, slack in (("W1", 16, 0.02), ("W2", 64, 0.01), ("W3", 64, 0.15)):
        a = math.sqrt(6.0 / fan_in)
        x = np.abs(p[name].reshape(-1))
        m = x.size
        assert a * (1 - slack) < x.max() <= a, name
        assert abs(x.mean() - a / 2) < 5 * a / math.sqrt(12 * m), name


def _eq1_cut_and_energy(dims, w, spins):
    """eq. (1) and eq. (2) by the double sum over i < j of the dense coupling
    matrix (parallel edges summed)."""
    a, b = oracle.torus_edges(dims)
    n = oracle.n_sites(dims)
    W = np.zeros((n, n), np.int64)
    for e in range(len(a)):
        W[a[e], b[e]] += int(w[e])
        W[b[e], a[e]] += int(w[e])
    iu = np.triu_indices(n, 1)
    cuts, ens = [], []
    for x in spins.astype(np.int64):
        outer = np.outer(x, x)[iu]
        cuts.append(0.5 * np.sum(W[iu] * (1 - outer)))
        ens.append(np.sum(W[iu] * outer))
    return np.array(cuts), np.array(ens)


@pytest.mark.parametrize("dims", [[6, 8], [4, 4, 6]])
def test_final_cut_score_is_eq1_cut_plus_gain(dims):
    """The score of the "gain" label is the predicted end-of-trial cut / |E|:
    with zero gain it is the replica's eq. (1) cut now / |E| (read from
    feature 0 = H/|E| through H = W_total - 2 cut), and a gain adds to it
    unchanged."""
    rng = np.random.default_rng(len(dims))
    n = oracle.n_sites(dims)
    E = len(dims) * n
    w = oracle.random_weights(int(rng.integers(1, 1000)), E)
    spins = (2 * rng.integers(0, 2, size=(9, n)) - 1).astype(np.int8)
    cut, en = _eq1_cut_and_energy(dims, w, spins)
    f = learn.features(dims, w, spins, en, np.zeros(9, np.uint32), learn.new_track(9), 10, 10, 20, 0.5, 2)
    zero = learn.final_cut_score(int(w.sum()), E, np.zeros(9), f)
    assert np.allclose(zero, cut / E, rtol=0, atol=1e-12)
    gain = rng.standard_normal(9)
    assert np.allclose(learn.final_cut_score(int(w.sum()), E, gain, f), cut / E + gain, rtol=0, atol=1e-12)
    # the all-positive torus in its checkerboard state cuts every edge: score 1
    ones = np.ones(E, np.int8)
    board = np.where(oracle.colours(dims) == 0, 1, -1).astype(np.int8)[None, :]
    _, hb = _eq1_cut_and_energy(dims, ones, board)
    fb = learn.features(dims, ones, board, hb, np.zeros(1, np.uint32), learn.new_track(1), 10, 10, 10, 1.0, 1)
    assert learn.final_cut_score(E, E, np.zeros(1), fb)[0] == 1.0


@pytest.mark.parametrize("dims", [[6, 8], [4, 4, 6]])
def test_features_identities(dims):
    n = oracle.n_sites(dims)
    E = len(dims) * n
    w = oracle.random_weights(3, E)
    spins = oracle.init_spins(8, 5, n)
    spins, fl = oracle.run(dims, w, 8, 5, 200, 0, 50, schedule=oracle.SCHED_GEOMETRIC, beta0=0.05, beta1=4.0)
    _, en = oracle.cut_energy(dims, w, spins)
    tr = learn.new_track(5)
    f = learn.features(dims, w, spins, en, fl, tr, 50, 50, 200, 0.7, 4)
    vals = np.array([-6, -4, -2, 0, 2, 4, 6])
    # sum_i s_i f_i = 2 H: the histogram against eq. (2)
    assert np.allclose(n * (f[:, 7:14] * vals).sum(axis=1), 2 * en)
    assert np.allclose(f[:, 7:14].sum(axis=1), 1.0)
    assert np.allclose(f[:, 0], en / E) and np.allclose(f[:, 1], en / E) and np.allclose(f[:, 2], en / E)
    assert np.allclose(f[:, 3], fl / (n * 50)) and np.allclose(f[:, 15], 0.0)
    assert np.allclose(f[:, 5], 0.7) and np.allclose(f[:, 14], math.log(0.7)) and np.allclose(f[:, 6], 0.25)
    # a second checkpoint at the infinite-temperature state: energy rises
    hot = oracle.init_spins(99, 5, n)
    _, en2 = oracle.cut_energy(dims, w, hot)
    fl2 = np.full(5, 7, np.uint32)
    f2 = learn.features(dims, w, hot, en2, fl2, tr, 100, 50, 200, 0.9, 4)
    worse = en2 > en
    assert np.allclose(f2[worse, 1], (en / E)[worse]) and np.allclose(f2[worse, 15], 0.25)
    assert np.allclose(f2[:, 2], (en2 - en) / E)
    assert np.allclose(f2[:, 4], (fl.astype(np.int64) + 7) / (n * 100))


def test_features_bipartite_closed_form():
    dims = [6, 8]
    n, E = 48, 96
    w = np.ones(E, np.int8)
    board = np.where(oracle.colours(dims) == 0, 1, -1).astype(np.int8)[None, :]
    _, en = oracle.cut_energy(dims, w, board)
    f = learn.features(dims, w, board, en, np.zeros(1, np.uint32), learn.new_track(1), 10, 10, 10, 1.0, 1)
    assert en[0] == -E and f[0, 0] == -1.0
    assert f[0, 8] == 1.0 and f[0, 7:14].sum() == 1.0  # every site has s f = -4


def test_cull_order_and_clone():
    score = np.array([0.5, 2.0, np.nan, 2.0, -1.0, 0.5, 3.0])
    order = learn.cull_order(score)
    assert order.tolist() == [6, 1, 3, 0, 5, 4, 2]
    spins = np.arange(7)[:, None].repeat(3, axis=1).astype(np.int8)
    tr = learn.new_track(7)
    tr["h_min"][:] = np.arange(7) * 10
    learn.cull_clone(order, spins, tr)
    # worst three (2, 4, 5) take the best three (6, 1, 3); the middle (0) stays
    assert spins[:, 0].tolist() == [0, 1, 6, 3, 1, 3, 6]
    assert tr["h_min"].tolist() == [0, 10, 60, 30, 10, 30, 60]


def test_standardize_groups_closed_form_and_invariants():
    """Within each group every column ends with mean 0 and population std 1;
    [1, 2, 3] maps to -sqrt(3/2), 0, sqrt(3/2); a column the whole group shares
    maps to 0; groups do not see each other."""
    x = np.array([[1.0], [2.0], [3.0]], np.float32)
    y = learn.standardize_groups(x, 1, 3, 1)
    assert np.allclose(y[:, 0], [-math.sqrt(1.5), 0.0, math.sqrt(1.5)], atol=1e-7)
    rng = np.random.default_rng(2)
    G, R, C = 3, 50, 4
    a = (rng.standard_normal((G, R, C)) * 7 + 100).astype(np.float32)
    a[1, :, 2] = 5.0
    z = learn.standardize_groups(a.reshape(G * R, C), G, R, C).reshape(G, R, C).astype(np.float64)
    for g in range(G):
        for c in range(C):
            if (g, c) == (1, 2):
                assert (z[g, :, c] == 0).all()
            else:
                assert abs(z[g, :, c].mean()) < 1e-6 and abs(z[g, :, c].std() - 1) < 1e-6
    # shifting and scaling one group leaves every group's result unchanged
    b = a.copy()
    b[0] = b[0] * 3 + 11
    z2 = learn.standardize_groups(b.reshape(G * R, C), G, R, C).reshape(G, R, C)
    assert np.allclose(z2, z, atol=1e-5)
    # a ranking by the standardised column is the ranking by the raw column
    assert (np.argsort(z[0, :, 1], kind="stable") == np.argsort(a[0, :, 1], kind="stable")).all()
