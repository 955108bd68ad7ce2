"""Trial-length campaign: windowed long trials equal one uninterrupted run
and the oracle; the readout follows eq. (3)-(5)."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ising():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2505_18508_amd as m

    m.lib()
    return m


def test_windowed_trials_equal_one_run_and_oracle(ising):
    from paper_2505_18508_amd import campaign

    dims, wseed, R, S, seed = [20, 32], 5, 24, 250, 77
    g = ising.create_graph(dims, wseed)
    a, _ = campaign.one_campaign(g, R, S, seed, window=37)
    b, _ = campaign.one_campaign(g, R, S, seed, window=S)
    assert (a == b).all()
    n = 640
    s, _ = oracle.run(dims, oracle.random_weights(wseed, 2 * n), seed, R, S, schedule=oracle.SCHED_GEOMETRIC,
                      beta0=0.05, beta1=4.0)
    cut, _ = oracle.cut_energy(dims, oracle.random_weights(wseed, 2 * n), s)
    assert (a == cut).all()
    g.close()


def test_campaign_readout(ising):
    from paper_2505_18508_amd import campaign, metrics

    out = campaign.campaign((20, 32), 5, 64, (50, 200, 800), seed=11)
    assert [c["sweeps"] for c in out["campaigns"]] == [50, 200, 800]
    assert out["best_cut"] == max(c["best"] for c in out["campaigns"])
    assert out["target"] == metrics.target_cut(out["best_cut"])
    for c in out["campaigns"]:
        assert sum(c["cut_counts"]) == 64 and c["min"] <= c["mean"] <= c["best"]
        if c["P_s"] > 0:
            assert c["r"] == pytest.approx(metrics.repetitions(c["P_s"]))
            assert c["STT_sweeps"] == pytest.approx(c["sweeps"] * c["r"])
            assert c["TTT_s"] == pytest.approx(c["t_trial_s"] * c["r"])
        else:
            assert c["TTT_s"] is None
    fastest = out["best_trial_length"]
    assert fastest["TTT_s"] == min(c["TTT_s"] for c in out["campaigns"] if c["TTT_s"] is not None)
