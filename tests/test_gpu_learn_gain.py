"""What the trained network gains over the method without it, at small
scale: the learned-culling protocol (network trained with the library's
kernels on plain runs of four instances, then used to cull replicas on a
held-out fifth) against the plain all-trials run on the same instance, seeds
and schedule.  Everything is seeded and every kernel is deterministic, so
the comparison is exact; the energy-ranked cull is reported beside it."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("label", ["final", "relative"])
def test_learned_culling_reaches_target_faster_than_plain(label):
    import torch

    assert torch.cuda.is_available()
    from paper_2505_18508_amd import experiments

    s = experiments.ttt_experiment(dims=(50, 100), weight_seed=3001, R=1024, S=4000, window=400,
                                   run_seeds=(201, 202, 203), train_seeds=(1001, 1002, 1003, 1004), n_traj=4096,
                                   epochs=20, batch=8192, long_sweeps=4000, label=label, log=print)
    blk = s["targets"]["compared_runs"]
    ttt = {m: blk["methods"][m]["median_TTT_s"] for m in blk["methods"]}
    print("target", blk["target"], "median TTT (s)", ttt)
    assert s["train_loss"][-1] < s["train_loss"][0]
    assert math.isfinite(ttt["learned"])
    assert ttt["learned"] < ttt["plain"]
    assert blk["learned_over_plain_TTT"] < 1.0
