"""Continuous batching: scenarios admitted while others run on the device
give the same results as when run alone (bitwise: no shared state, fixed
reduction orders), and the server reports sane statistics."""
import numpy as np
import pytest

from helpers import say
from paper_2604_20731_amd import inputs

pytestmark = pytest.mark.gpu


def _mix():
    arr = []
    t = 0.0
    for k, (ne, w, nw) in enumerate([(32, 32, 1), (64, 64, 3), (32, 64, 5), (64, 32, 2),
                                     (48, 64, 8), (64, 64, 4)]):
        arr.append(inputs.Arrival(t=t, n_elem=ne, width=w, seed=100 + k, n_wells=nw))
        t += 0.002
    return arr


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_alone_equals_mix(prec):
    from paper_2604_20731_amd.serve import Server
    arrivals = _mix()
    srv = Server(hbm_budget_bytes=1 << 30, max_active=4, precision=prec, pretrain_iters=30,
                 steps=3, keep_fields=True)
    mix = srv.run(arrivals)
    say(f"mix {prec}: {mix['scenarios']} scenarios, {mix['scenarios_per_s']:.1f}/s, "
        f"p50 {mix['p50_step_ms']:.2f} ms p99 {mix['p99_step_ms']:.2f} ms")
    assert mix["scenarios"] == len(arrivals)
    for a in arrivals:
        alone = Server(hbm_budget_bytes=1 << 30, max_active=1, precision=prec, pretrain_iters=30,
                       steps=3, keep_fields=True).run([a])
        pm, sm, _ = mix["results"][a.seed]["fields"]
        pa, sa, _ = alone["results"][a.seed]["fields"]
        assert np.array_equal(pm, pa) and np.array_equal(sm, sa), a
        assert len(mix["results"][a.seed]["latencies_ms"]) == 3


def test_budget_limits_concurrency():
    from paper_2604_20731_amd import crv
    from paper_2604_20731_amd.serve import Server
    arrivals = _mix()
    one = crv.workspace_size(crv.config(n_elem=64, width=64, hidden=4, precision="bf16x3"))
    srv = Server(hbm_budget_bytes=int(1.5 * one), max_active=8, precision="bf16x3",
                 pretrain_iters=10, steps=2)
    out = srv.run(arrivals)
    assert out["scenarios"] == len(arrivals)
    assert out["max_queue_wait_s"] >= 0.0
