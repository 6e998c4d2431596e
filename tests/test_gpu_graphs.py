"""Captured (hipGraph) coupled steps and training blocks must reproduce the
eagerly launched kernels exactly: same kernels, same order, same inputs.
Every replay is compared, with synchronising reads between replays."""
import os

import numpy as np
import pytest

from helpers import problem, say, scenario_for

pytestmark = pytest.mark.gpu


def _pair(prec, **over):
    prob = problem("c1", **over)
    os.environ["CRV_NO_GRAPH"] = "1"
    try:
        eager = scenario_for(prob, prec)
    finally:
        del os.environ["CRV_NO_GRAPH"]
    graph = scenario_for(prob, prec)
    return eager, graph


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp64"])
def test_graph_replays_equal_eager(prec):
    say("graphs", prec)
    eager, graph = _pair(prec)
    for sc in (eager, graph):
        sc.pretrain_pressure(250)      # two captured 100-iteration blocks + 50 eager
    le, lg = eager.loss_history(), graph.loss_history()
    assert np.array_equal(le, lg)
    for k in range(3):
        eager.step(2e-5)
        graph.step(2e-5)
        pe, se, _ = eager.fields()
        pg, sg, _ = graph.fields()
        say(f"  step {k}: max |dp| {np.abs(pe - pg).max():.3e} max |dS| {np.abs(se - sg).max():.3e}")
        assert np.array_equal(pe, pg) and np.array_equal(se, sg)
    assert np.array_equal(eager.loss_history(), graph.loss_history())
