"""GPU parity of the learned-culling kernels against the float64 oracle:
network init, forward, loss gradient and Adam within fp32 tolerances;
features, ranking, cloning and a culled trajectory bit-exact (integer work)."""
import numpy as np
import pytest

import oracle
from oracle import learn as olearn
from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ising():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as m

    m.lib()
    return m


def dev_tensor(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def random_params(ising, seed):
    import torch

    p = torch.zeros(5313, dtype=torch.float32, device="cuda")
    ising.mlp_init(seed, p)
    noise = np.random.default_rng(seed).standard_normal(5313).astype(np.float32) * 0.05
    return p + dev_tensor(noise)


def test_mlp_init_matches_oracle(ising):
    import torch

    p = torch.zeros(5313, dtype=torch.float32, device="cuda")
    ising.mlp_init(42, p)
    ref = olearn.init_params(42)
    got = p.cpu().numpy().astype(np.float64)
    assert np.allclose(got, ref, rtol=2.0**-22, atol=0)
    assert (got[1024:1088] == 0).all() and got[-1] == 0


@pytest.mark.parametrize("B", [1, 63, 1000, 8192])
def test_mlp_forward_matches_oracle(ising, B):
    import torch

    rng = np.random.default_rng(B)
    p = random_params(ising, 7)
    x = rng.standard_normal((B, 16)).astype(np.float32) * 3 + 1
    mean = rng.standard_normal(16).astype(np.float32)
    std = rng.uniform(0.5, 2.0, 16).astype(np.float32)
    y = torch.zeros(B, dtype=torch.float32, device="cuda")
    ising.mlp_forward(p, dev_tensor(x), y, mean=dev_tensor(mean), std=dev_tensor(std))
    z = (x.astype(np.float64) - mean) / std
    ref = olearn.forward(p.cpu().numpy().astype(np.float64), z)
    err = np.abs(y.cpu().numpy() - ref).max() / max(1.0, np.abs(ref).max())
    assert err < 1e-5


def test_mlp_forward_gathers_rows(ising):
    import torch

    rng = np.random.default_rng(3)
    p = random_params(ising, 8)
    x = dev_tensor(rng.standard_normal((3000, 16)).astype(np.float32))
    idx_np = rng.integers(0, 3000, size=700).astype(np.int32)
    y1 = torch.zeros(700, dtype=torch.float32, device="cuda")
    y2 = torch.zeros(700, dtype=torch.float32, device="cuda")
    ising.mlp_forward(p, x, y1, idx=dev_tensor(idx_np))
    ising.mlp_forward(p, x[idx_np.astype(np.int64)].contiguous(), y2)
    assert torch.equal(y1, y2)


def test_mlp_rows_outside_x_read_nothing_and_give_nan(ising):
    """A gathered row index outside x reads nothing: its forward output is
    NaN (the other rows are exact), and the loss and gradient of a batch
    holding it are NaN."""
    import torch

    rng = np.random.default_rng(5)
    p = random_params(ising, 8)
    x = dev_tensor(rng.standard_normal((100, 16)).astype(np.float32))
    idx_np = np.array([0, 99, 100, -1, 2**31 - 1, -2**31, 7], np.int32)
    y = torch.zeros(len(idx_np), dtype=torch.float32, device="cuda")
    ising.mlp_forward(p, x, y, idx=dev_tensor(idx_np))
    ok = np.array([0, 1, 6])
    ref = torch.zeros(3, dtype=torch.float32, device="cuda")
    ising.mlp_forward(p, x[idx_np[ok].astype(np.int64)].contiguous(), ref)
    got = y.cpu().numpy()
    assert np.isnan(got[[2, 3, 4, 5]]).all()
    assert (got[ok] == ref.cpu().numpy()).all()
    grad = torch.zeros(5313, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.zeros(ising.mlp_workspace_floats(len(idx_np)), dtype=torch.float32, device="cuda")
    t = torch.zeros(100, dtype=torch.float32, device="cuda")
    ising.mlp_loss_grad(p, x, t, grad, ws, loss, idx=dev_tensor(idx_np))
    assert np.isnan(loss.item()) and torch.isnan(grad).any().item()


@pytest.mark.parametrize("B", [1, 100, 1000, 8192])
def test_mlp_loss_grad_matches_oracle(ising, B):
    import torch

    rng = np.random.default_rng(B + 1)
    p = random_params(ising, 9)
    x = rng.standard_normal((B, 16)).astype(np.float32)
    t = rng.standard_normal(B).astype(np.float32) * 0.1 + 0.4
    mean = rng.standard_normal(16).astype(np.float32) * 0.1
    std = rng.uniform(0.8, 1.2, 16).astype(np.float32)
    grad = torch.zeros(5313, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = torch.zeros(ising.mlp_workspace_floats(B), dtype=torch.float32, device="cuda")
    args = (p, dev_tensor(x), dev_tensor(t), grad, ws, loss)
    ising.mlp_loss_grad(*args, mean=dev_tensor(mean), std=dev_tensor(std))
    g1 = grad.clone()
    ising.mlp_loss_grad(*args, mean=dev_tensor(mean), std=dev_tensor(std))
    assert torch.equal(g1, grad), "gradient not reproducible"
    z = (x.astype(np.float64) - mean) / std
    ref_loss, ref_grad = olearn.loss_grad(p.cpu().numpy().astype(np.float64), z, t.astype(np.float64))
    got = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref_grad) / np.linalg.norm(ref_grad) < 1e-4
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)


def test_adam_matches_oracle(ising):
    import torch

    rng = np.random.default_rng(5)
    n = 5313
    th = rng.standard_normal(n).astype(np.float32)
    p, m, v = dev_tensor(th), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    rth, rm, rv = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        ising.adam_step(p, dev_tensor(g), m, v, step, lr=1e-3)
        rth, rm, rv = olearn.adam_step(rth, g.astype(np.float64), rm, rv, step, lr=1e-3)
    assert np.allclose(p.cpu().numpy(), rth, rtol=1e-5, atol=1e-6)


def test_feature_stats_match_numpy(ising):
    import torch

    rng = np.random.default_rng(6)
    x = (rng.standard_normal((100003, 16)) * rng.uniform(0.1, 5, 16) + rng.uniform(-3, 3, 16)).astype(np.float32)
    x[:, 5] = 0.25  # constant column: std floored at 1e-6
    mean = torch.zeros(16, device="cuda")
    std = torch.zeros(16, device="cuda")
    ising.feature_stats(dev_tensor(x), mean, std)
    xd = x.astype(np.float64)
    assert np.allclose(mean.cpu().numpy(), xd.mean(axis=0), rtol=1e-6, atol=1e-7)
    ref_std = np.maximum(xd.std(axis=0), 1e-6)
    assert np.allclose(std.cpu().numpy(), ref_std, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("G,R,C", [(3, 1000, 16), (1, 8192, 16), (2, 37, 1), (4, 1, 3)])
def test_standardize_groups_matches_oracle(ising, G, R, C):
    rng = np.random.default_rng(G * 1000 + R + C)
    x = (rng.standard_normal((G * R, C)) * rng.uniform(0.1, 50, C) + rng.uniform(-1e4, 1e4, C)).astype(np.float32)
    x[: R, C - 1] = 0.25  # a column the first group shares
    t = dev_tensor(x)
    ising.standardize_groups(t, G, R, C)
    ref = olearn.standardize_groups(x, G, R, C)
    got = t.cpu().numpy()
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5)
    assert (got[:R, C - 1] == 0).all()


@pytest.mark.parametrize("dims", [[20, 30], [6, 8, 10]])  # 3-D: the +/-6 bins of the s f histogram
def test_features_match_oracle_over_two_checkpoints(ising, dims):
    import torch

    wseed, seed, R, S = 3, 11, 12, 300
    n = oracle.n_sites(dims)
    E = len(dims) * n
    g = ising.create_graph(dims, wseed)
    w = oracle.random_weights(wseed, E)
    spins = torch.zeros((R, n), dtype=torch.int8, device="cuda")
    cut = torch.zeros(R, dtype=torch.int64, device="cuda")
    en = torch.zeros(R, dtype=torch.int64, device="cuda")
    fl = torch.zeros(R, dtype=torch.int32, device="cuda")
    track = ising.new_track(R)
    feats = torch.zeros((R, 16), dtype=torch.float32, device="cuda")
    otrack = olearn.new_track(R)
    os_ = None
    for k, (b, e) in enumerate([(0, 100), (100, 200)]):
        ising.run_trials(g, spins, seed, S, b, e, "geometric", 0.05, 4.0, None, b == 0, "auto", cut, en, fl)
        beta = ising.schedule_beta(S, e - 1, "geometric", 0.05, 4.0)
        ising.features(g, spins, en, fl, track, e, e - b, S, beta, 2, feats)
        os_, ofl = oracle.run(dims, w, seed, R, S, b, e, oracle.SCHED_GEOMETRIC, 0.05, 4.0, spins=os_)
        _, oen = oracle.cut_energy(dims, w, os_)
        ref = olearn.features(dims, w, os_, oen, ofl, otrack, e, e - b, S, beta, 2)
        torch.cuda.synchronize()
        assert (spins.cpu().numpy() == os_).all()
        got = feats.cpu().numpy().astype(np.float64)
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-7), np.abs(got - ref).max()
        t = track.cpu().numpy()
        assert (t[:, 0] == otrack["h_min"]).all() and (t[:, 1] == otrack["h_prev"]).all()
        assert (t[:, 2].astype(np.uint64) == otrack["flips_total"]).all()
        assert ((t[:, 3] & 0xFFFFFFFF) == otrack["checkpoints"]).all()
        assert ((t[:, 3] >> 32) == otrack["last_improve"]).all()


@pytest.mark.parametrize("R", [1, 2, 7, 1000, 8192])
def test_cull_order_and_clone_match_oracle(ising, R):
    import torch

    rng = np.random.default_rng(R)
    n = 33
    score = rng.integers(-5, 5, size=R).astype(np.float32) * 0.5  # many ties
    if R > 3:
        score[rng.integers(0, R, size=3)] = np.nan
        score[0] = -0.0
        score[1] = 0.0
    spins = (2 * rng.integers(0, 2, size=(R, n)) - 1).astype(np.int8)
    tr = rng.integers(-1000, 1000, size=(R, 4)).astype(np.int64)
    s_dev, t_dev = dev_tensor(spins), dev_tensor(tr)
    order = torch.zeros(R, dtype=torch.int32, device="cuda")
    ising.cull_clone(dev_tensor(score), s_dev, t_dev, order)
    ref_order = olearn.cull_order(score)
    assert (order.cpu().numpy() == ref_order).all()
    ref_spins = spins.copy()
    ref_tr = {"rows": tr.copy()}
    olearn.cull_clone(ref_order, ref_spins, ref_tr)
    assert (s_dev.cpu().numpy() == ref_spins).all()
    assert (t_dev.cpu().numpy() == ref_tr["rows"]).all()


def test_energy_score(ising):
    import torch

    e = torch.tensor([5, -3, 0, 100], dtype=torch.int64, device="cuda")
    s = torch.zeros(4, dtype=torch.float32, device="cuda")
    ising.energy_score(e, s)
    assert s.cpu().tolist() == [-5.0, 3.0, 0.0, -100.0]


@pytest.mark.parametrize("method", ["learned", "energy"])
def test_culled_trajectory_replays_on_oracle(ising, method):
    """A culled run on the GPU; the oracle, fed the GPU's rankings, reproduces
    every replica's final spins bit for bit."""
    from paper_2505_18508_amd import learn

    dims, wseed, seed, R, S, window = [12, 16], 5, 21, 20, 400, 100
    n, E = 192, 384
    g = ising.create_graph(dims, wseed)
    model = None
    if method == "learned":
        import torch

        model = learn.Model(random_params(ising, 4), torch.zeros(16, device="cuda"), torch.ones(16, device="cuda"))
    out = learn.anneal(g, R, S, seed, "geometric", 0.05, 4.0, window, method, model)
    orders = [o.cpu().numpy() for o in out["orders"]]
    assert len(orders) == 3
    w = oracle.random_weights(wseed, E)
    os_ = None
    begin = 0
    for k, end in enumerate([100, 200, 300, 400]):
        os_, _ = oracle.run(dims, w, seed, R, S, begin, end, oracle.SCHED_GEOMETRIC, 0.05, 4.0, spins=os_)
        if end < S:
            olearn.cull_clone(orders[k], os_)
        begin = end
    assert (out["spins"].cpu().numpy() == os_).all()
    c, e = oracle.cut_energy(dims, w, os_)
    assert (out["cut"].cpu().numpy() == c).all() and (out["energy"].cpu().numpy() == e).all()
    if method == "energy":
        # the energy-ranked form keeps the lowest-energy replicas at each checkpoint
        assert all(sorted(o.tolist()) == list(range(R)) for o in orders)


def test_final_cut_score_matches_oracle(ising):
    import torch

    rng = np.random.default_rng(12)
    g = ising.create_graph([20, 30], 7)
    gain = rng.standard_normal(50).astype(np.float32) * 1e-3
    feats = rng.standard_normal((50, 16)).astype(np.float32)
    score = torch.zeros(50, dtype=torch.float32, device="cuda")
    ising.final_cut_score(g, dev_tensor(gain), dev_tensor(feats), score)
    ref = olearn.final_cut_score(g.w_total, g.n_edges, gain, feats)
    assert np.allclose(score.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)


def test_cut_labels_match_their_definition(ising):
    """(final - now) * scale in double, rounded to float once; without now,
    final * scale."""
    import torch

    rng = np.random.default_rng(17)
    R = 3000
    final = rng.integers(13000, 14000, size=R).astype(np.int64)
    now = final - rng.integers(0, 200, size=R).astype(np.int64)
    out = torch.zeros(R, dtype=torch.float32, device="cuda")
    scale = 1.0 / 40000
    ising.cut_labels(dev_tensor(final), out, dev_tensor(now), scale)
    want = ((final - now).astype(np.float64) * scale).astype(np.float32)
    assert (out.cpu().numpy() == want).all()
    ising.cut_labels(dev_tensor(final), out)
    assert (out.cpu().numpy() == final.astype(np.float64).astype(np.float32)).all()
