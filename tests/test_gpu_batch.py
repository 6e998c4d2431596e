"""Batched multi-scenario launches: scenarios of one configuration whose
workspaces lie at a fixed stride in one allocation (crv.Bucket) advance with
one launch per kernel of the coupled step, blockIdx.z selecting the scenario
(the unit batched is the coupled step of the IGA-ADS-CRVPINN algorithm,
steps 4-7).

crv_step_batch: every kernel reduces in an order that does not depend on the
batch, so bucket steps equal single steps bitwise.

crv_step_batch_shared: the network backward spreads the device's resident
blocks over the batch, so each scenario's parameter gradient is the same sum
grouped into fewer partial rows; Adam's normalised steps carry the rounding
into the parameters and the network's output (a small difference of large
terms) amplifies it: after 2 coupled steps the fields, parameters and loss
history agree within each form's trajectory parity bound against the oracle
(FP32 1e-3, split bf16 1e-3, mixed 5e-3; measured worst cases: pressure 3e-5
FP32 at width 32 and 1.1e-4 at width 128, 4e-4 split bf16, 2e-3 mixed; the
saturation and parameters 1e-5 or less).  Plain bf16 is compared
on its parameters, saturation and loss history only, to 1e-2: its
bf16-rounded forward makes the pressure swing by tens of percent under
parameter changes of 3e-5 (the same ill-conditioning that puts it 10% off
the oracle).  A batch of one is bitwise a single step either way."""
import numpy as np
import pytest

from helpers import check, say
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


def _close(a, b, tol=1e-4, pressure=True):
    pa, ca, _ = a.fields()
    pb, cb, _ = b.fields()
    ta, _, _, sa = a.get_state()
    tb, _, _, sb = b.get_state()
    if pressure:
        check("p", pa, pb, tol)
    check("S", ca, cb, tol)
    check("theta", ta, tb, tol)
    check("loss history", a.loss_history(), b.loss_history(), tol)
    assert sa == sb


CASES = [("bf16x3f", 64, 64, 3), ("fp32", 48, 32, 2), ("bf16x3f", 128, 128, 2), ("bf16", 64, 64, 3),
         ("bf16x3", 40, 32, 4), ("bf16x3f", 512, 64, 3), ("fp32", 64, 128, 2)]


def _run(prec, ne, width, n, shared, part=1, **cfg_kw):
    from paper_2604_20731_amd import crv
    probs = _problems(n, ne, width)
    cfg = crv.config(dim=2, n_elem=ne, degree=2, width=width, hidden=4, precision=prec, **cfg_kw)
    bucket = crv.Bucket(cfg, probs)
    singles = [crv.Scenario(cfg, p.log_perm, p.porosity, p.wells, p.theta0) for p in probs]
    for sc in bucket.scenarios + singles:
        sc.pretrain_pressure(20)
    dts = [_dt(sc, p) for sc, p in zip(singles, probs)]
    for _ in range(2):
        bucket.step(dts, shared, part)
        for sc, dt in zip(singles, dts):
            sc.step(dt)
    return crv, bucket, singles, dts


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,ne,width,n", CASES)
def test_bucket_step_equals_single_steps(prec, ne, width, n):
    say("bucket", prec, ne, width, n)
    crv, bucket, singles, dts = _run(prec, ne, width, n, False)
    for k, (a, b) in enumerate(zip(bucket.scenarios, singles)):
        assert _same(a, b), (prec, ne, width, k)
    # a run of consecutive scenarios of the bucket is itself a batch
    crv.step_batch(bucket.scenarios[1:], dts[1:])
    for sc, dt in zip(singles[1:], dts[1:]):
        sc.step(dt)
    for a, b in zip(bucket.scenarios[1:], singles[1:]):
        assert _same(a, b)
    bucket.close()
    for sc in singles:
        sc.close()
    say(f"  {n} scenarios bitwise equal to single steps")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,ne,width", [("bf16x3f", 64, 64), ("fp32", 48, 32)])
def test_bucket_step_with_distance_factor_equals_single_steps(prec, ne, width):
    """The distance trial factor rides in the batched kernels' geometry: a
    bucket of such scenarios still steps bitwise as single steps."""
    say("bucket, distance factor", prec, ne, width)
    crv, bucket, singles, dts = _run(prec, ne, width, 2, False, boundary_factor=1)
    for k, (a, b) in enumerate(zip(bucket.scenarios, singles)):
        assert _same(a, b), (prec, ne, width, k)
    assert bucket.scenarios[0].cfg.boundary_factor == 1
    bucket.close()
    for sc in singles:
        sc.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,ne,width,n", CASES)
def test_shared_bucket_step_matches_single_steps(prec, ne, width, n):
    say("shared bucket", prec, ne, width, n)
    crv, bucket, singles, dts = _run(prec, ne, width, n, True)
    tol = {"fp32": 1e-3, "bf16x3": 1e-3, "bf16x3f": 5e-3, "bf16": 1e-2}[prec]
    with_p = prec != "bf16"
    for k, (a, b) in enumerate(zip(bucket.scenarios, singles)):
        say(f"  scenario {k}")
        _close(a, b, tol, with_p)
    bucket.close()
    for sc in singles:
        sc.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,ne,width,n,part", [("bf16x3f", 512, 64, 2, 2), ("fp32", 64, 64, 3, 4)])
def test_shared_part_bucket_step_matches_single_steps(prec, ne, width, n, part):
    """crv_step_batch_shared_part: the batch's backward on 1/part of the
    device's blocks (the grouping of the gradient sums changes again), within
    the same bounds as the shared form."""
    say("shared part bucket", prec, ne, width, n, part)
    crv, bucket, singles, dts = _run(prec, ne, width, n, True, part)
    tol = {"fp32": 1e-3, "bf16x3f": 5e-3}[prec]
    for k, (a, b) in enumerate(zip(bucket.scenarios, singles)):
        say(f"  scenario {k}")
        _close(a, b, tol, True)
    bucket.close()
    for sc in singles:
        sc.close()


def test_batch_of_one_is_a_single_step_bitwise():
    from paper_2604_20731_amd import crv
    probs = _problems(2, 64, 64)
    cfg = crv.config(dim=2, n_elem=64, degree=2, width=64, hidden=4, precision="bf16x3f")
    bucket = crv.Bucket(cfg, probs)
    single = crv.Scenario(cfg, probs[0].log_perm, probs[0].porosity, probs[0].wells,
                          probs[0].theta0)
    for sc in (bucket.scenarios[0], single):
        sc.pretrain_pressure(20)
    dt = _dt(single, probs[0])
    for _ in range(2):
        crv.step_batch(bucket.scenarios[:1], [dt], shared=True)
        single.step(dt)
    assert _same(bucket.scenarios[0], single)


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


@pytest.mark.timeout(600)
def test_bucket_group_concurrent_equals_sequential():
    """crv.BucketGroup steps its buckets on their own streams at once (the
    bench's headline form); the result must not depend on that concurrency:
    bitwise the same buckets stepped one after another with a device
    synchronisation in between."""
    import torch
    from paper_2604_20731_amd import crv
    probs = _problems(4, 64, 64)
    cfg = crv.config(dim=2, n_elem=64, degree=2, width=64, hidden=4, precision="bf16x3f")
    conc = crv.BucketGroup(cfg, probs, groups=2)
    seq = crv.BucketGroup(cfg, probs, groups=2)
    for sc in conc.scenarios + seq.scenarios:
        sc.pretrain_pressure(20)
    dts = [_dt(sc, p) for sc, p in zip(seq.scenarios, probs)]
    for _ in range(2):
        conc.step(dts, True, 2)
        k = 0
        for b in seq.buckets:
            b.step(dts[k:k + len(b.scenarios)], True, 2)
            k += len(b.scenarios)
            torch.cuda.synchronize()
    for a, b in zip(conc.scenarios, seq.scenarios):
        assert _same(a, b)
    say("  concurrent bucket group bitwise equal to sequential buckets")
    conc.close()
    seq.close()
