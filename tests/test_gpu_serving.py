"""Continuous batching: scenarios admitted while others run on the device
give the same results as when run alone (bitwise: no shared state, fixed
reduction orders), and the server reports sane statistics."""
import numpy as np
import pytest

from helpers import say
from paper_2604_20731_amd import inputs

pytestmark = pytest.mark.gpu


def _mix(big=False):
    """Arrivals 2 ms apart; with big, one 256^2 scenario and one of width 128
    join the small ones (quadratic elements, 4 hidden layers)."""
    shapes = [(32, 32, 1), (64, 64, 3), (32, 64, 5), (64, 32, 2), (48, 64, 8), (64, 64, 4)]
    if big:
        shapes = [(256, 64, 5), (32, 32, 1), (64, 128, 3), (64, 64, 2), (48, 64, 8)]
    arr = []
    t = 0.0
    for k, (ne, w, nw) in enumerate(shapes):
        arr.append(inputs.Arrival(t=t, n_elem=ne, width=w, seed=100 + k, n_wells=nw))
        t += 0.002
    return arr


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,big", [("bf16x3f", False), ("bf16x3f", True), ("bf16x3", False),
                                      ("fp32", False)])
def test_alone_equals_mix(prec, big):
    """Scenarios on their own streams: the default served form (the mixed
    network) included, with a 256^2 scenario and a width-128 one in the mix;
    the mix must actually overlap (two or more scenarios active at once) and
    every result is bitwise the one of the scenario alone."""
    from paper_2604_20731_amd.serve import Server
    arrivals = _mix(big)
    srv = Server(hbm_budget_bytes=4 << 30, max_active=4, precision=prec, pretrain_iters=30,
                 steps=3, keep_fields=True, batch=False)
    mix = srv.run(arrivals)
    say(f"mix {prec} big={big}: {mix['scenarios']} scenarios, {mix['scenarios_per_s']:.1f}/s, "
        f"p50 {mix['p50_step_ms']:.2f} ms p99 {mix['p99_step_ms']:.2f} ms, "
        f"at most {mix['max_active_seen']} active")
    assert mix["scenarios"] == len(arrivals)
    assert mix["max_active_seen"] >= 2
    for a in arrivals:
        alone = Server(hbm_budget_bytes=4 << 30, max_active=1, precision=prec, pretrain_iters=30,
                       steps=3, keep_fields=True, batch=False).run([a])
        pm, sm, _ = mix["results"][a.seed]["fields"]
        pa, sa, _ = alone["results"][a.seed]["fields"]
        assert np.array_equal(pm, pa) and np.array_equal(sm, sa), a
        assert len(mix["results"][a.seed]["latencies_ms"]) == 3


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["bf16x3f", "fp32"])
def test_batched_serving_alone_equals_mix(prec):
    """The batched server (slot pools; each pool advances in rounds, every run
    of consecutive ready slots as one crv_step_batch): arrivals of three
    shapes, several of each, so that batches form (the largest holds two or
    more scenarios); every scenario's pressure and saturation are bitwise
    those of its run alone."""
    from paper_2604_20731_amd.serve import Server
    shapes = [(64, 64), (64, 64), (48, 32), (64, 64), (48, 32), (96, 128), (96, 128), (64, 64)]
    arrivals = [inputs.Arrival(t=0.0005 * k, n_elem=ne, width=w, seed=300 + k, n_wells=1 + k % 5)
                for k, (ne, w) in enumerate(shapes)]
    srv = Server(hbm_budget_bytes=4 << 30, max_active=8, precision=prec, pretrain_iters=30,
                 steps=3, keep_fields=True, batch=True, pool_slots=4)
    mix = srv.run(arrivals)
    say(f"batched mix {prec}: {mix['scenarios']} scenarios, largest batch {mix['largest_batch']}, "
        f"p50 {mix['p50_step_ms']:.2f} ms p99 {mix['p99_step_ms']:.2f} ms")
    assert mix["scenarios"] == len(arrivals)
    assert mix["largest_batch"] >= 2
    for a in arrivals:
        alone = Server(hbm_budget_bytes=4 << 30, max_active=1, precision=prec, pretrain_iters=30,
                       steps=3, keep_fields=True, batch=True).run([a])
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
                 pretrain_iters=10, steps=2, batch=False)
    out = srv.run(arrivals)
    assert out["scenarios"] == len(arrivals)
    assert out["max_queue_wait_s"] >= 0.0
    assert out["peak_workspace_bytes"] <= int(1.5 * one)


def test_arrival_larger_than_budget_is_refused():
    """An arrival whose workspace alone exceeds the budget is refused (it
    would otherwise wait forever); the others still run."""
    from paper_2604_20731_amd import crv
    from paper_2604_20731_amd.serve import Server
    arrivals = _mix()[:3]
    big = inputs.Arrival(t=0.0, n_elem=512, width=128, seed=999, n_wells=2)
    small = crv.workspace_size(crv.config(n_elem=64, width=64, hidden=4, precision="bf16x3f"))
    srv = Server(hbm_budget_bytes=4 * small, max_active=4, precision="bf16x3f",
                 pretrain_iters=5, steps=1)
    out = srv.run([big] + arrivals)
    assert out["refused"] == [999]
    assert out["scenarios"] == len(arrivals)


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
