"""GPU: exhaustive schedule sweep on a 256^3 Navier-Stokes grid, then the
device-trained MLP cost model: it must rank schedules well enough that its
pick is close to the best measured one, and beat the default schedule."""
import numpy as np
import pytest

from paper_1709_02125_amd import ns3d as N, ooc, tune
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_cost_model_proposal_has_small_regret():
    # a third of the footprint leaves room for 15 of these 36 schedules (the
    # skew of a multi-step chain is a large part of a small grid)
    n = 256
    budget = N.footprint_bytes(n) // 3
    say("case: tune sweep ns3d 256^3")
    app, plan_ctx, q, cells, rb = tune.ns3d_workload(n, budget)
    cands = tune.grid([4, 6, 8, 12, 16, 0], [1, 2], [2, 3, 4])
    recs = tune.sweep(app, plan_ctx, q, cells, rb, budget, cands, chains=2, log=say)
    app.close()
    assert len(recs) >= 12
    t = np.array([r["sec_per_cell_step"] for r in recs])
    best = t.min()
    model = tune.CostModel(n_hidden=32, seed=5)
    loss = model.fit(recs, epochs=4000, lr=3e-3)
    say("cost model training loss (standardised log time):", loss)
    (h, k, S), _ = model.propose([((r["h"], r["k"], r["S"]), r["features"]) for r in recs])
    chosen = [r for r in recs if (r["h"], r["k"], r["S"]) == (h, k, S)][0]["sec_per_cell_step"]
    regret = chosen / best - 1.0
    default = [r for r in recs if (r["h"], r["k"], r["S"]) == (0, 1, 3)]
    say("regret %.3f; default/best %.3f" % (regret, default[0]["sec_per_cell_step"] / best if default else -1))
    assert regret <= 0.10
    if default:
        assert chosen <= default[0]["sec_per_cell_step"] * 1.05
    model.close()
    # held out: trained on half of the measured schedules, it picks among all
    # of them from their planned features alone
    held = [tune.holdout_regret(recs, 0.5, seed) for seed in (1, 2, 3)]
    for r in held:
        say("held-out pick", r["pick"], "regret %.3f gain over default %s" % (r["regret"], r["gain_over_default"]))
    assert sorted(r["regret"] for r in held)[1] <= 0.10
