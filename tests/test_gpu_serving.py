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


def test_step_batch_equals_single_steps():
    """crv_step_batch over scenarios on their own streams gives bitwise the
    fields of one crv_step per scenario; invalid batches are rejected before
    anything is enqueued."""
    import torch
    from paper_2604_20731_amd import crv
    from paper_2604_20731_amd.serve import cfl_dt, scenario_problem

    arrivals = _mix()[:3]

    def build():
        out = []
        for a in arrivals:
            prob = scenario_problem(a)
            cfg = crv.config(dim=2, n_elem=prob.n_elem, degree=prob.degree, width=prob.width,
                             hidden=prob.hidden, precision="bf16x3")
            sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0,
                              stream=torch.cuda.Stream())
            sc.pretrain_pressure(20)
            dt = cfl_dt(sc.fields()[0], prob.log_perm, prob.porosity, prob.n_elem)
            out.append((sc, dt))
        return out

    batch, single = build(), build()
    for _ in range(2):
        crv.step_batch([sc for sc, _ in batch], [dt for _, dt in batch])
        for sc, dt in single:
            sc.step(dt)
    for (sb, _), (ss, _) in zip(batch, single):
        pb, cb, _ = sb.fields()
        ps, cs, _ = ss.fields()
        assert np.array_equal(pb, ps) and np.array_equal(cb, cs)
    with pytest.raises(crv.CrvError) as ei:
        crv.step_batch([sc for sc, _ in batch], [1e-3, -1.0, 1e-3])
    assert ei.value.status == crv.CRV_EINVAL
    say(f"step_batch: {len(batch)} scenarios bitwise equal to single steps")
