"""The 257^2 configuration's whole trajectory against stored FP64 oracle
values (tests/golden/c2_trajectory.npz, written by tests/golden/make_goldens.py
from the oracle alone): 2000 pretraining iterations and 10 coupled steps of
100 Adam iterations (IGA-ADS-CRVPINN algorithm, steps 2-8), lr 1e-4, the
network pressure and saturation compared after the pretraining and after
steps 1, 2, 5 and 10, and the loss history over all 3000 iterations.  Bounds
are the targets for the pressure and saturation fields: 1e-3 relative L2 in
FP32, 5e-3 with the bf16 network (mixed form), each with the elementwise
error normalised by the field's largest value under the same bound."""
import os

import numpy as np
import pytest

from helpers import check, problem, rel, say, scenario_for

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_trajectory.npz")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("bf16x3f", 5e-3)])
def test_c2_trajectory_against_golden(prec, tol):
    if not os.path.exists(GOLD):
        pytest.skip("tests/golden/c2_trajectory.npz has not been generated")
    g = np.load(GOLD)
    say(f"c2 257^2 trajectory {prec}: {int(g['pretrain'])} pretraining + {int(g['steps'])} steps")
    prob = problem("c2")
    sc = scenario_for(prob, prec)
    sc.pretrain_pressure(int(g["pretrain"]))
    p, _, _ = sc.fields()
    check("after pretraining, p", p, g["u_pre"], tol)
    dt = float(g["dt"])
    marks = set(int(k) for k in g["checkpoints"])
    for k in range(1, int(g["steps"]) + 1):
        sc.step(dt)
        if k in marks:
            p, s, _ = sc.fields()
            check(f"step {k}, p", p, g[f"u_step{k}"], tol)
            check(f"step {k}, S", s, g[f"s_step{k}"], tol)
    lh = sc.loss_history()
    ref = g["loss"]
    assert lh.size == ref.size
    e = rel(lh, ref)
    say(f"  loss history over {ref.size} iterations: relL2 {e:.2e}")
    assert e < tol
    sc.close()
