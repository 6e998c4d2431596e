"""Host-side logic of the serving scheduler (no GPU): how many slots a pool
of each scenario shape gets under the step-cost cap."""
from paper_2604_20731_amd import inputs
from paper_2604_20731_amd.serve import Server, scenario_problem


def _prob(ne, width):
    return scenario_problem(inputs.Arrival(t=0.0, n_elem=ne, width=width, seed=7, n_wells=2))


def test_pool_slots_follow_the_step_cost_cap():
    srv = Server(hbm_budget_bytes=1 << 30)  # default cap: two 512^2 width-128 scenarios
    assert srv.slots_for(_prob(512, 128)) == 2
    assert srv.slots_for(_prob(512, 64)) == 8        # a quarter of the cost: pool_slots
    assert srv.slots_for(_prob(256, 128)) == 8
    assert srv.slots_for(_prob(64, 64)) == 8
    assert Server(hbm_budget_bytes=1 << 30, pool_slots=3).slots_for(_prob(64, 64)) == 3
    # a cap below one scenario's cost still leaves one slot
    assert Server(hbm_budget_bytes=1 << 30, batch_cost_cap=1.0).slots_for(_prob(512, 128)) == 1
