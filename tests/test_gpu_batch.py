"""Batched multi-scenario launches: scenarios of one configuration whose
workspaces lie at a fixed stride in one allocation (crv.Bucket) advance with
one launch per kernel of the coupled step, blockIdx.z selecting the scenario
(the unit batched is the coupled step of the IGA-ADS-CRVPINN algorithm,
steps 4-7).  Every kernel reduces in a fixed order that does not depend on
the batch, so the results must equal single-scenario steps bitwise."""
import numpy as np
import pytest

from helpers import say
from paper_2604_20731_amd import inputs

pytestmark = pytest.mark.gpu


def _problems(n, ne, width):
    return [inputs.make_problem("b512", seed=20 + k, n_elem=ne, width=width,
                                wells=inputs.wells_balanced(1 + 2 * k, 20 + k)) for k in range(n)]


def _dt(sc, prob):
    from paper_2604_20731_amd.serve import cfl_dt
    return cfl_dt(sc.fields()[0], prob.log_perm, prob.porosity, prob.n_elem)


def _same(a, b):
    pa, ca, na = a.fields()
    pb, cb, nb = b.fields()
    ta, ma, va, sa = a.get_state()
    tb, mb, vb, sb = b.get_state()
    return (np.array_equal(pa, pb) and np.array_equal(ca, cb) and np.array_equal(na, nb)
            and np.array_equal(ta, tb) and np.array_equal(ma, mb) and np.array_equal(va, vb)
            and sa == sb and np.array_equal(a.loss_history(), b.loss_history()))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,ne,width,n", [("bf16x3f", 64, 64, 3), ("fp32", 48, 32, 2),
                                             ("bf16x3f", 128, 128, 2), ("bf16", 64, 64, 3),
                                             ("bf16x3", 40, 32, 4), ("bf16x3f", 512, 64, 3)])
def test_bucket_step_equals_single_steps(prec, ne, width, n):
    from paper_2604_20731_amd import crv
    say("bucket", prec, ne, width, n)
    probs = _problems(n, ne, width)
    cfg = crv.config(dim=2, n_elem=ne, degree=2, width=width, hidden=4, precision=prec)
    bucket = crv.Bucket(cfg, probs)
    singles = [crv.Scenario(cfg, p.log_perm, p.porosity, p.wells, p.theta0) for p in probs]
    for sc in bucket.scenarios + singles:
        sc.pretrain_pressure(20)
    dts = [_dt(sc, p) for sc, p in zip(singles, probs)]
    for _ in range(2):
        bucket.step(dts)
        for sc, dt in zip(singles, dts):
            sc.step(dt)
    for k, (a, b) in enumerate(zip(bucket.scenarios, singles)):
        assert _same(a, b), (prec, ne, width, k)
    # a run of consecutive scenarios of the bucket is itself a batch
    crv.step_batch(bucket.scenarios[1:], dts[1:])
    for sc, dt in zip(singles[1:], dts[1:]):
        sc.step(dt)
    for a, b in zip(bucket.scenarios, singles):
        if a is not bucket.scenarios[0]:
            assert _same(a, b)
    bucket.close()
    for sc in singles:
        sc.close()
    say(f"  {n} scenarios bitwise equal to single steps")


def test_unordered_or_mixed_batches_fall_back_to_streams():
    """Scenarios not at increasing equal spacing (reversed order, or
    different shapes) still step correctly, each on its own stream."""
    from paper_2604_20731_amd import crv
    probs = _problems(3, 32, 32)
    cfg = crv.config(dim=2, n_elem=32, degree=2, width=32, hidden=4, precision="bf16x3f")
    bucket = crv.Bucket(cfg, probs)
    singles = [crv.Scenario(cfg, p.log_perm, p.porosity, p.wells, p.theta0) for p in probs]
    for sc in bucket.scenarios + singles:
        sc.pretrain_pressure(10)
    dts = [_dt(sc, p) for sc, p in zip(singles, probs)]
    crv.step_batch(bucket.scenarios[::-1], dts[::-1])
    other = inputs.make_problem("b512", seed=5, n_elem=24, width=32)
    cfg2 = crv.config(dim=2, n_elem=24, degree=2, width=32, hidden=4, precision="bf16x3f")
    lone = crv.Scenario(cfg2, other.log_perm, other.porosity, other.wells, other.theta0)
    lone.pretrain_pressure(10)
    crv.step_batch([bucket.scenarios[0], lone], [dts[0], _dt(lone, other)])
    for sc, dt in zip(singles, dts):
        sc.step(dt)
    singles[0].step(dts[0])
    for a, b in zip(bucket.scenarios, singles):
        assert _same(a, b)
